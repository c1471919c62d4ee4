"""Minimal real state vector psi (oracle; test infrastructure).

Sec. 6.2 represents a divergence-free velocity field by the minimum number of
independent real variables (20,218 at 32 x 31 x 32).  Convention used here
(an interface choice; the paper does not fix a basis):

  * (0, 0) mode: real u_x and u_z, Dirichlet at the walls; their Chebyshev
    coefficients n = 0..N-3 (the top two follow from u(+-1) = 0).
  * every other independent mode (kz > 0, or kz = 0 with kx > 0), in storage
    order (ikx major, kz minor): the wall-normal velocity v with
    v(+-1) = v'(+-1) = 0 (coefficients n = 0..N-5 free) and the wall-normal
    vorticity eta = i b u_x - i a u_z with eta(+-1) = 0 (n = 0..N-3 free),
    stored as [Re v, Im v, Re eta, Im eta].
  * u_x = (i a Dv - i b eta)/kappa^2, u_z = (i b Dv + i a eta)/kappa^2
    reconstructs the horizontal velocity; the field is divergence-free in every
    Chebyshev coefficient and no-slip.

Length: 4 (Kx + 2 Kx Kz + Kz)(N - 3) + 2 (N - 2).
"""

import numpy as np

from . import cheb


def _fill_dirichlet(c):
    """c has length N with the last two entries to be set so that c(+-1) = 0:
    each parity class must sum to zero."""
    N = len(c)
    c = c.copy()
    for top in (N - 2, N - 1):
        idx = np.arange(top % 2, top, 2)
        c[top] = -np.sum(c[idx])
    return c


def _fill_clamped(c):
    """Set the last four entries so that c(+-1) = c'(+-1) = 0: within each
    parity class sum c_n = 0 and sum n^2 c_n = 0 (T_n(1) = 1, T_n'(1) = n^2)."""
    N = len(c)
    c = c.copy()
    for q in (N - 2, N - 1):
        p = q - 2
        idx = np.arange(q % 2, p, 2)
        s0 = np.sum(c[idx])
        s2 = np.sum(idx.astype(float) ** 2 * c[idx])
        cq = (-s2 + p * p * s0) / (q * q - p * p)
        c[q] = cq
        c[p] = -s0 - cq
    return c


def pack(g, u):
    N = g.N
    out = [u[0, 0, 0, :N - 2].real, u[2, 0, 0, :N - 2].real]
    for (ikx, kz) in g.independent_modes()[1:]:
        a, b = g.a[ikx], g.b[kz]
        v = u[1, ikx, kz]
        eta = 1j * b * u[0, ikx, kz] - 1j * a * u[2, ikx, kz]
        out += [v[:N - 4].real, v[:N - 4].imag, eta[:N - 2].real, eta[:N - 2].imag]
    return np.concatenate(out)


def unpack(g, psi):
    N = g.N
    D = cheb.derivative(N)
    u = g.zeros()
    pos = 0

    def take(n):
        nonlocal pos
        x = psi[pos:pos + n]
        pos += n
        return np.asarray(x, dtype=float)

    for c in (0, 2):
        x = np.zeros(N)
        x[:N - 2] = take(N - 2)
        u[c, 0, 0] = _fill_dirichlet(x)
    kxlist = list(g.kx)
    for (ikx, kz) in g.independent_modes()[1:]:
        a, b = g.a[ikx], g.b[kz]
        k2 = a * a + b * b
        v = np.zeros(N, dtype=complex)
        v[:N - 4] = take(N - 4) + 1j * take(N - 4)
        v = _fill_clamped(v)
        eta = np.zeros(N, dtype=complex)
        eta[:N - 2] = take(N - 2) + 1j * take(N - 2)
        eta = _fill_dirichlet(eta)
        Dv = D @ v
        u[0, ikx, kz] = (1j * a * Dv - 1j * b * eta) / k2
        u[1, ikx, kz] = v
        u[2, ikx, kz] = (1j * b * Dv + 1j * a * eta) / k2
        if kz == 0:
            jm = kxlist.index(-g.kx[ikx])
            u[:, jm, 0] = np.conj(u[:, ikx, 0])
    assert pos == len(psi)
    return u

"""Pins for the oracle's dealiased convective term.

Brute force: on tiny grids with low Chebyshev degree, (U.grad)U is computed as
an explicit truncated Fourier convolution with exact Chebyshev products
(numpy.polynomial.chebyshev.chebmul / chebder).  With the 2/3 cut-off the grid
product is alias-free in x and z, and the collocation in y is exact when the
product's degree is <= N-1, so the oracle must agree to round-off."""

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import Grid
from oracle.flow import Transforms, nonlinear, nonlinear_lin


def random_hermitian(g, deg, seed):
    rng = np.random.default_rng(seed)
    u = g.zeros()
    kx = list(g.kx)
    for ikx in range(g.nkx):
        for kz in range(g.nkz):
            if kz == 0 and g.kx[ikx] < 0:
                continue
            c = rng.standard_normal((3, deg + 1)) + 1j * rng.standard_normal((3, deg + 1))
            if ikx == 0 and kz == 0:
                c = c.real.astype(complex)
            u[:, ikx, kz, :deg + 1] = c
            if kz == 0 and g.kx[ikx] > 0:
                u[:, kx.index(-g.kx[ikx]), 0] = np.conj(u[:, ikx, 0])
    return u


def full_plane(g, f):
    """dict (kx, kz) -> Chebyshev coefficients for all kz in [-Kz, Kz]."""
    out = {}
    for ikx, kx in enumerate(g.kx):
        for kz in range(g.nkz):
            out[(kx, kz)] = f[ikx, kz].copy()
            if kz > 0:
                out[(-kx, -kz)] = np.conj(f[ikx, kz])
    return out


def brute_convective(g, Ufull, Vgrad, N):
    """sum_j U_j d_j V_i as a truncated convolution; Ufull[j], Vgrad[i][j] are
    full-plane dicts."""
    out = np.zeros(g.shape, dtype=complex)
    for i in range(3):
        acc = {}
        for j in range(3):
            for k1, f1 in Ufull[j].items():
                for k2, f2 in Vgrad[i][j].items():
                    k = (k1[0] + k2[0], k1[1] + k2[1])
                    if abs(k[0]) > g.Kx or k[1] < 0 or k[1] > g.Kz:
                        continue
                    p = npcheb.chebmul(f1, f2)
                    assert np.all(np.abs(p[N:]) < 1e-12)
                    acc[k] = acc.get(k, 0) + np.pad(p, (0, max(0, N - len(p))))[:N]
        for ikx, kx in enumerate(g.kx):
            for kz in range(g.nkz):
                out[i, ikx, kz] = acc.get((kx, kz), np.zeros(N))
    return out


def fields_full(g, u, base):
    N = g.N
    U, dU = [], []
    for i in range(3):
        fp = full_plane(g, u[i])
        if base and i == 0:
            fp[(0, 0)] = fp[(0, 0)] + np.eye(N)[1]          # + y e_x (T_1)
        U.append(fp)
    for i in range(3):
        row = []
        for j in range(3):
            d = {}
            for (kx, kz), c in U[i].items():
                if j == 0:
                    d[(kx, kz)] = 1j * g.alpha * kx * c
                elif j == 2:
                    d[(kx, kz)] = 1j * g.beta * kz * c
                else:
                    d[(kx, kz)] = np.pad(npcheb.chebder(c), (0, 1))
            row.append(d)
        dU.append(row)
    return U, dU


@pytest.mark.parametrize("dims", [(9, 13, 12), (12, 13, 9), (9, 11, 9)])
def test_nonlinear_bruteforce(dims):
    g = Grid(*dims, Lx=2.3, Lz=1.7)
    deg = (g.N - 1) // 2
    u = random_hermitian(g, deg, seed=sum(dims))
    U, dU = fields_full(g, u, base=True)
    want = -brute_convective(g, U, dU, g.N)
    got = nonlinear(Transforms(g), u)
    scale = np.abs(want).max()
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * scale)


def test_linearised_bruteforce_and_polarisation():
    g = Grid(9, 13, 12, Lx=2.3, Lz=1.7)
    T = Transforms(g)
    deg = (g.N - 1) // 2
    u = random_hermitian(g, deg, seed=3)
    v = random_hermitian(g, deg, seed=4)
    U, dU = fields_full(g, u, base=True)
    V, dV = fields_full(g, v, base=False)
    want = -(brute_convective(g, U, dV, g.N) + brute_convective(g, V, dU, g.N))
    got = nonlinear_lin(T, u, v)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
    # M is quadratic, so its derivative is exactly the symmetric difference
    pol = 0.5 * (nonlinear(T, u + v) - nonlinear(T, u - v))
    np.testing.assert_allclose(got, pol, rtol=0, atol=1e-12 * np.abs(want).max())


def test_transform_adjoints():
    """<A p, w>_W = <p, A* w>_g and <synth c, p>_g = <c, synth* p>_W."""
    from oracle.method import Method
    g = Grid(9, 11, 12, Lx=2.3, Lz=1.7)
    m = Method(g)
    T = m.T
    rng = np.random.default_rng(0)
    p = rng.standard_normal((g.N, g.Nx, g.Nz))
    w = random_hermitian(g, g.N - 1, seed=9)[0][None]
    c = random_hermitian(g, g.N - 1, seed=10)[1][None]

    def ip_grid(a, b):
        return float(np.sum(a * b)) / (g.Nx * g.Nz)

    def ip_w(a, b):
        z = np.zeros((2,) + a.shape[1:], dtype=complex)
        A = np.concatenate([a, z]); B = np.concatenate([b, z])
        return m.inner(A, B)

    lhs = ip_w(T.analysis(p)[None], w)
    rhs = ip_grid(p, T.analysis_adj(w[0]))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    lhs = ip_grid(T.synth(c[0]), p)
    rhs = ip_w(c, T.synth_adj(p)[None])
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)

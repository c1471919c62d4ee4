"""Pins for the oracle's dense Chebyshev-tau Stokes solve S_lam.

* Manufactured solutions: for an admissible u and an arbitrary pressure p, the
  forcing F = (lam + nu kappa^2 - nu D^2) u + grad p, built here with numpy's
  Chebyshev routines, must give S_lam(F) = u (the tau equations hold exactly).
* Pure gradients are annihilated: S_lam(grad phi) = 0.
* Outputs are divergence-free in every Chebyshev coefficient and no-slip.
* The conjugate-transposed and W-adjoint solves satisfy their defining
  identities.
"""

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import Grid
from oracle.method import Method
from paper_2306_00165_amd import inputs


def cheb_d(c, k=1):
    out = np.asarray(c, dtype=complex)
    N = len(out)
    for _ in range(k):
        out = np.pad(npcheb.chebder(out), (0, 1))[:N]
    return out


GRIDS = [(16, 25, 16), (12, 17, 9), (32, 33, 32)]


@pytest.fixture(scope="module", params=GRIDS, ids=lambda d: "x".join(map(str, d)))
def setup(request):
    g = Grid(*request.param)
    return g, Method(g)


def test_manufactured_solution(setup):
    g, m = setup
    lam, nu, N = g.lam, g.nu, g.N
    u = inputs.random_field(g.Nx, g.Ny, g.Nz, energy=1e-2, seed=11)
    rng = np.random.default_rng(12)
    F = g.zeros()
    for (ikx, kz) in g.modes():
        a, b = g.a[ikx], g.b[kz]
        k2 = a * a + b * b
        if ikx == 0 and kz == 0:
            for c in (0, 2):
                F[c, 0, 0] = lam * u[c, 0, 0] - nu * cheb_d(u[c, 0, 0], 2)
            F[1, 0, 0] = rng.standard_normal(N)            # ignored by S for (0, 0)
            continue
        p = (rng.standard_normal(N) + 1j * rng.standard_normal(N)) * np.exp(-0.3 * np.arange(N))
        grad = [1j * a * p, cheb_d(p), 1j * b * p]
        for c in range(3):
            F[c, ikx, kz] = (lam + nu * k2) * u[c, ikx, kz] - nu * cheb_d(u[c, ikx, kz], 2) + grad[c]
    got = m.S.solve(F)
    scale = np.abs(u).max()
    np.testing.assert_allclose(got, u, rtol=0, atol=1e-12 * scale)


def test_gradient_is_annihilated(setup):
    g, m = setup
    rng = np.random.default_rng(13)
    F = g.zeros()
    N = g.N
    for (ikx, kz) in g.modes():
        phi = (rng.standard_normal(N) + 1j * rng.standard_normal(N)) * np.exp(-0.3 * np.arange(N))
        F[0, ikx, kz] = 1j * g.a[ikx] * phi
        F[1, ikx, kz] = cheb_d(phi)
        F[2, ikx, kz] = 1j * g.b[kz] * phi
    assert np.abs(m.S.solve(F)).max() < 1e-13 * np.abs(F).max()


def test_output_admissible(setup):
    g, m = setup
    F = inputs.random_field(g.Nx, g.Ny, g.Nz, energy=1.0, seed=14)
    F = F + 0.3 * np.roll(F, 1, axis=0)              # not divergence-free
    u = m.S.solve(F)
    div, wall, herm = m.defects(u)
    s = np.abs(u).max()
    assert div < 1e-13 * s and wall < 1e-13 * s and herm < 1e-13 * s


def test_adjoint_solves(setup):
    g, m = setup
    F = inputs.random_field(g.Nx, g.Ny, g.Nz, energy=1.0, seed=15)
    X = inputs.random_field(g.Nx, g.Ny, g.Nz, energy=1.0, seed=16)
    F = F + 0.2 * np.roll(F, 1, axis=0)
    X = X + 0.2 * np.roll(X, 2, axis=0)

    def ip_e(a, b):
        return sum(g.weight(kz) * np.real(np.vdot(a[:, :, kz], b[:, :, kz])) for kz in range(g.nkz))

    lhs = ip_e(m.S.solve(F), X)
    rhs = ip_e(F, m.S.solve_h(X))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    lhs = m.inner(m.S.solve(F), X)
    rhs = m.inner(F, m.S.solve_wadj(X))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)

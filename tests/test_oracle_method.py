"""Pins for the oracle's residual, derivative, adjoint, projection, descent,
diagnostics and state vector."""

import json
import os

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import Grid, state
from oracle.method import Method
from paper_2306_00165_amd import inputs
import symmetry as sym

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.fixture(scope="module")
def cfg1():
    g = Grid(16, 25, 16)
    m = Method(g)
    return g, m, inputs.config1_guess()


def rnd(g, seed, energy=1e-3):
    return inputs.random_field(g.Nx, g.Ny, g.Nz, g.Lx, g.Lz, energy=energy, seed=seed)


# -- residual ---------------------------------------------------------------------

def test_laminar_is_equilibrium(cfg1):
    g, m, _ = cfg1
    assert np.abs(m.residual(g.zeros())).max() == 0.0


def test_fd_form_equals_direct_form(cfg1):
    g, m, u = cfg1
    r = m.residual(u)
    assert m.norm(m.residual_fd(u) - r) <= 1e-12 * m.norm(r)


def test_laplacian_matches_polynomial_calculus(cfg1):
    g, m, u = cfg1
    L = m.lap(u)
    for (ikx, kz) in [(0, 0), (1, 2), (g.nkx - 1, 3), (2, 0)]:
        k2 = g.kappa2(ikx, kz)
        for c in range(3):
            want = np.pad(npcheb.chebder(u[c, ikx, kz], 2), (0, 2)) - k2 * u[c, ikx, kz]
            np.testing.assert_allclose(L[c, ikx, kz], want, atol=1e-12 * np.abs(want).max() + 1e-300)


@pytest.mark.parametrize("op", ["shift", "sigma1", "sigma2", "s1", "s2"])
def test_equivariance(cfg1, op):
    g, m, u = cfg1
    act = {
        "shift": lambda f: sym.shift(f, g.a, g.b, 0.37 * g.Lx, 0.81 * g.Lz),
        "sigma1": sym.sigma1, "sigma2": sym.sigma2,
        "s1": lambda f: sym.s1(f, g), "s2": lambda f: sym.s2(f, g),
    }[op]
    r = m.residual(u)
    np.testing.assert_allclose(m.residual(act(u)), act(r), rtol=0, atol=1e-13 * np.abs(r).max())
    f, _ = m.descent_direction(u)
    f2, _ = m.descent_direction(act(u))
    np.testing.assert_allclose(f2, act(f), rtol=0, atol=1e-12 * np.abs(f).max())


# -- derivative and adjoint ---------------------------------------------------------

def test_jvp_matches_central_differences(cfg1):
    g, m, u = cfg1
    v = rnd(g, 21)
    Jv = m.jvp(u, v)
    errs = []
    for eps in (1e-2, 5e-3):
        fd = (m.residual(u + eps * v) - m.residual(u - eps * v)) / (2 * eps)
        errs.append(m.norm(fd - Jv) / m.norm(Jv))
    # quadratic nonlinearity: central differences are exact up to round-off
    assert max(errs) < 1e-11


@pytest.mark.parametrize("general", [False, True])
def test_adjoint_identity(cfg1, general):
    g, m, u = cfg1
    v = rnd(g, 22)
    w = rnd(g, 23)
    if general:       # w outside the admissible space
        w = w + 0.5 * np.roll(w, 1, axis=0)
        v = v + 0.5 * np.roll(v, 2, axis=0)
    lhs = m.inner(m.jvp(u, v), w)
    rhs = m.inner(v, m.adjoint(u, w))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _real_coordinates(g):
    coords = []
    for (ikx, kz) in g.independent_modes():
        parts = (0,) if (ikx, kz) == (0, 0) else (0, 1)
        for c in range(3):
            for n in range(g.N):
                for p in parts:
                    coords.append((c, ikx, kz, n, p))
    return coords


def _embed(g, coords, x):
    u = g.zeros()
    kx = list(g.kx)
    for val, (c, ikx, kz, n, p) in zip(x, coords):
        u[c, ikx, kz, n] += val * (1j if p else 1.0)
        if kz == 0 and g.kx[ikx] > 0:
            u[c, kx.index(-g.kx[ikx]), 0, n] += val * (-1j if p else 1.0)
    return u


def _extract(coords, u):
    return np.array([(u[c, i, k, n].imag if p else u[c, i, k, n].real) for (c, i, k, n, p) in coords])


def test_adjoint_bruteforce_tiny_grid():
    """Dense J on a 6 x 9 x 6 grid, column by column, then W^{-1} J^T W."""
    g = Grid(6, 9, 6, Re=150.0)
    m = Method(g)
    u = 3.0 * rnd(g, 31, energy=1e-2)
    coords = _real_coordinates(g)
    n = len(coords)
    E = np.stack([_embed(g, coords, np.eye(n)[i]) for i in range(n)], axis=-1)
    J = np.stack([_extract(coords, m.jvp(u, E[..., i])) for i in range(n)], axis=1)
    W = np.array([[m.inner(E[..., i], E[..., j]) for j in range(n)] for i in range(n)])
    Jstar = np.linalg.solve(W, J.T @ W)
    rng = np.random.default_rng(32)
    x = rng.standard_normal(n)
    w = _embed(g, coords, x)
    want = _embed(g, coords, Jstar @ x)
    got = m.adjoint(u, w)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * np.abs(want).max())


def test_cost_gradient_fd(cfg1):
    g, m, u = cfg1
    v = rnd(g, 24)
    r = m.residual(u)
    grad = 2 * m.inner(v, m.adjoint(u, r))
    e1, e2 = 1e-3, 5e-4
    d1 = (m.cost(u + e1 * v) - m.cost(u - e1 * v)) / (2 * e1) - grad
    d2 = (m.cost(u + e2 * v) - m.cost(u - e2 * v)) / (2 * e2) - grad
    # J^2 is quartic in u: the central-difference error is exactly O(eps^2)
    assert abs(d1) < 1e-6 * abs(grad)
    assert 3.0 < d1 / d2 < 5.0 or abs(d2) < 1e-12 * abs(grad)


# -- projection --------------------------------------------------------------------

def test_projection_properties(cfg1):
    g, m, u = cfg1
    a = rnd(g, 41, 1.0)
    b = rnd(g, 42, 1.0)
    ga = a + 0.7 * np.roll(a, 1, axis=0) + 0.1 * np.roll(a, 3, axis=3)
    gb = b + 0.4 * np.roll(b, 2, axis=0)
    Pa = m.project(ga)
    s = np.abs(Pa).max()
    assert max(m.defects(Pa)) < 1e-13 * s                                 # range in V_h
    assert np.abs(m.project(Pa) - Pa).max() < 1e-13 * s                   # idempotent
    assert np.abs(m.project(a) - a).max() < 1e-13 * np.abs(a).max()       # identity on V_h
    lhs, rhs = m.inner(m.project(ga), gb), m.inner(ga, m.project(gb))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)                              # W-self-adjoint


# -- descent -----------------------------------------------------------------------

def test_descent_monotone_and_admissible(cfg1):
    g, m, u = cfg1
    costs = []
    for _ in range(10):
        u, c = m.descent_step(u, 0.02)
        costs.append(c)
    assert all(c2 < c1 for c1, c2 in zip(costs, costs[1:]))
    assert max(m.defects(u)) < 1e-14


def test_symmetric_guess_stays_symmetric(cfg1):
    g, m, _ = cfg1
    u = rnd(g, 51, 5e-3)
    u = 0.5 * (u + sym.s1(u, g))
    u = 0.5 * (u + sym.s2(u, g))
    assert np.abs(sym.s1(u, g) - u).max() < 1e-16 and np.abs(sym.s2(u, g) - u).max() < 1e-16
    for _ in range(5):
        u, _ = m.descent_step(u, 0.02)
    s = np.abs(u).max()
    assert np.abs(sym.s1(u, g) - u).max() < 1e-13 * s
    assert np.abs(sym.s2(u, g) - u).max() < 1e-13 * s


@pytest.mark.slow
def test_paper_step_size_is_stable():
    """Sec. 5.1 runs forward Euler with dtau = 0.03 at 32 x 31 x 32 (dt = 0.25):
    the linearised descent at laminar flow must be stable there, i.e.
    dtau < 2 / lambda_max(P_W J* J)."""
    p = GOLDEN["paper_run"]
    g = Grid(32, 31, 32, Lx=p["Lx"], Lz=p["Lz"], Re=p["Re"], dt=p["dt"])
    m = Method(g)
    z = g.zeros()
    x = rnd(g, 61, 1.0)
    lam = 0.0
    for _ in range(40):
        y = m.project(m.adjoint(z, m.jvp(z, x)))
        lam = m.inner(x, y) / m.inner(x, x)
        x = y / m.norm(y)
    assert p["dtau"] < 2.0 / lam < 1.5 * p["dtau"]


# -- diagnostics and state vector ---------------------------------------------------

def test_laminar_diagnostics_match_table2():
    eq0 = GOLDEN["laminar_EQ0"]
    g = Grid(16, 25, 16)
    m = Method(g)
    z = g.zeros()
    assert m.norm(z) == eq0["norm"]
    assert abs(m.dissipation(z) - eq0["D_over_Dlam"]) < 1e-15
    assert abs(m.total_norm(z) ** 2 - 1.0 / 3.0) < 1e-15     # (1/2) int y^2 dy


@pytest.mark.parametrize("seed,energy", [(1, 1e-3), (81, 0.05), (82, 0.3)])
def test_dissipation_equals_gradient_norm(seed, energy):
    """D = <curl U, curl U>_W equals sum_ij ||d_j U_i||^2_W for U = u_b + u with
    u divergence-free and no-slip: the difference is the volume integral of
    d_j(U_i d_i U_j) (using div U = 0), a wall flux of U_i d_i U_y that
    vanishes because U is constant along each wall (U = (+-1, 0, 0) there, so
    d_x U_y = d_z U_y = 0 and U_y = 0).  Every integrand is a polynomial of
    degree < 2 Ny in y, which the Gram matrix integrates exactly, so the
    identity holds to round-off; a sign or index mistake in any vorticity
    component breaks it at the 1e-4 level or more."""
    g = Grid(16, 25, 16)
    m = Method(g)
    T = m.T
    u = rnd(g, seed, energy)
    U = m.base_flow() + u
    grad2 = 0.0
    for i in range(3):
        dU = np.stack([T.ddx(U[i]), T.ddy(U[i]), T.ddz(U[i])])
        grad2 += m.inner(dU, dU)
    assert abs(m.dissipation(u) - grad2) < 1e-13 * grad2


def test_state_vector_length_matches_paper():
    sv = GOLDEN["state_vector_length"]
    g = Grid(sv["grid"]["Nx"], sv["grid"]["Ny"], sv["grid"]["Nz"])
    assert g.n_state() == sv["value"]
    assert len(state.pack(g, g.zeros())) == sv["value"]


@pytest.mark.parametrize("dims", [(16, 25, 16), (12, 17, 9)])
def test_state_vector_roundtrip(dims):
    g = Grid(*dims)
    m = Method(g)
    u = rnd(g, 71)
    psi = state.pack(g, u)
    assert len(psi) == g.n_state()
    np.testing.assert_allclose(state.unpack(g, psi), u, rtol=0, atol=1e-15)
    x = np.random.default_rng(72).standard_normal(g.n_state())
    w = state.unpack(g, x)
    assert max(m.defects(w)) < 1e-12 * np.abs(w).max()
    np.testing.assert_allclose(state.pack(g, w), x, rtol=0, atol=1e-12)

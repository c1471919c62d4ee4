"""Pins for the oracle's DMD extrapolation.

Affine-linear dynamics psi_{k+1} = psi* + A (psi_k - psi*) with a known stable
A have the exact fixed point psi*: DMD of a window whose span contains the
dynamics (rank >= number of excited modes + 1) must return psi* to round-off
(Sec. 6: the omega ~ 0 mode of the best-fit linear model is the steady state).
Also pinned: omega_1 = 0 exactly there, the numerical rank, and that the
extrapolation of an actual descent window lowers the cost."""

import numpy as np
import pytest

from oracle import Grid, dmd, state
from oracle.method import Method
from paper_2306_00165_amd import inputs


def affine_window(n, nmodes, M, seed, dtau=1.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, nmodes)))
    rates = np.linspace(0.05, 0.4, nmodes)          # decay rates: A = exp(-rate dtau) on span(Q)
    psi_star = rng.standard_normal(n)
    c0 = rng.standard_normal(nmodes)
    snaps = [psi_star + Q @ (c0 * np.exp(-rates * k * dtau)) for k in range(M)]
    return np.array(snaps), psi_star, rates


@pytest.mark.parametrize("nmodes,M", [(1, 4), (3, 8), (6, 20)])
def test_affine_dynamics_fixed_point_is_exact(nmodes, M):
    snaps, psi_star, rates = affine_window(200, nmodes, M, seed=nmodes)
    r = dmd.numerical_rank(snaps)
    assert r == nmodes + 1
    psi_s, om = dmd.steady_state(snaps, 1.0, r)
    assert abs(om) < 1e-9
    np.testing.assert_allclose(psi_s, psi_star, rtol=0, atol=1e-9 * np.abs(psi_star).max())
    lam, omega, Phi, b = dmd.dmd(snaps, 1.0, r)
    got = np.sort(-np.real(omega))[1:]
    np.testing.assert_allclose(got, np.sort(rates), rtol=1e-8)


def test_truncated_rank_is_worse_than_full_rank():
    snaps, psi_star, _ = affine_window(100, 4, 12, seed=9)
    err_full = np.abs(dmd.steady_state(snaps, 1.0, 5)[0] - psi_star).max()
    err_low = np.abs(dmd.steady_state(snaps, 1.0, 2)[0] - psi_star).max()
    assert err_full < 1e-9 < err_low


def test_extrapolation_of_a_descent_window_lowers_the_cost():
    g = Grid(16, 25, 16)
    m = Method(g)
    u = inputs.config1_guess()
    for _ in range(40):
        u, _ = m.descent_step(u, 0.02)
    window = []
    for k in range(40):
        if k % 4 == 0:
            window.append(u.copy())
        u, _ = m.descent_step(u, 0.02)
    c_now = m.cost(window[-1])
    u_s, c_s, r, kind = dmd.extrapolate(m, window, 4 * 0.02)
    assert r >= 1 and kind >= 0 and u_s is not None
    assert max(m.defects(u_s)) < 1e-12
    assert c_s < c_now


def test_numerical_rank_counts_singular_values_of_the_first_m_minus_1_snapshots():
    """The rank is that of [psi_1 .. psi_{M-1}] (the pairs' first members),
    counting singular values above 1e-7 of the largest."""
    rng = np.random.default_rng(3)
    n, M = 50, 6
    U, _ = np.linalg.qr(rng.standard_normal((n, M - 1)))
    V, _ = np.linalg.qr(rng.standard_normal((M - 1, M - 1)))
    s = np.array([1.0, 1e-3, 1e-6, 5e-8, 0.0])
    X = (U * s) @ V.T                                 # n x (M-1), singular values s
    last = rng.standard_normal(n)                     # psi_M does not count
    snaps = np.vstack([X.T, last])
    assert dmd.numerical_rank(snaps) == 3
    assert dmd.numerical_rank(snaps, tol=1e-8) == 4


def test_rank_is_chosen_by_least_true_cost(monkeypatch):
    """Sec. 6.2: among the candidates of ranks r = 1..r*, the one whose
    extrapolated state has the smallest cost is taken.  With a stub candidate
    list (the rank marked in each state's first entry) and a stub cost table,
    the choice must be the argmin over r <= r* (not the largest rank, not
    beyond r*), returning that candidate, its cost, r and its kind."""
    g = Grid(6, 9, 6)
    n = g.n_state()
    table = {1: 3.0, 2: 1.0, 3: 2.0, 4: 0.5, 5: 4.0, 6: 0.1}

    def fake_candidates(psis, dtau, rstar):
        out = []
        for r in range(1, rstar + 1):
            psi = np.zeros(n)
            psi[0] = r
            out.append((r, r % 2, psi))
        return out

    class StubMethod:
        def __init__(self):
            self.g = g

        def cost(self, u):
            return table[int(round(state.pack(g, u)[0]))]

    monkeypatch.setattr(dmd, "candidates", fake_candidates)
    monkeypatch.setattr(dmd, "numerical_rank", lambda psis, tol=dmd.RANK_TOL: 5)
    fields = [state.unpack(g, np.full(n, float(k))) for k in range(4)]
    u_s, c_s, r, kind = dmd.extrapolate(StubMethod(), fields, 1.0)
    assert (r, c_s, kind) == (4, 0.5, 0)
    assert state.pack(g, u_s)[0] == 4.0
    monkeypatch.setattr(dmd, "numerical_rank", lambda psis, tol=dmd.RANK_TOL: 0)
    assert dmd.extrapolate(StubMethod(), fields, 1.0) == (None, np.inf, 0, -1)


def decaying_window(n, rates, M, seed, psi_star=None):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, len(rates))))
    c0 = rng.standard_normal(len(rates))
    base = np.zeros(n) if psi_star is None else psi_star
    return np.array([base + Q @ (c0 * np.exp(-np.asarray(rates) * k)) for k in range(M)])


def test_affine_limit_of_a_decaying_window_is_the_origin():
    """psi_{k+1} = A psi_k with every mode decaying (a trajectory heading for
    the laminar state, psi* = 0): the full-rank affine limit (kind 1) from the
    differences is the origin to round-off, while the paper's smallest-|omega|
    candidate (kind 0) keeps the slowest mode's current part."""
    rates = [0.03, 0.1, 0.25]
    snaps = decaying_window(120, rates, 10, seed=4)
    r = dmd.numerical_rank(snaps)
    assert r == 3 and dmd.numerical_rank(np.diff(snaps, axis=0)) == 3
    cands = {(rr, k): psi for rr, k, psi in dmd.candidates(snaps, 1.0, r)}
    scale = np.abs(snaps[-1]).max()
    assert np.abs(cands[(3, 1)]).max() < 1e-10 * scale
    lam, omega, Phi, b = dmd.dmd(snaps, 1.0, 3)
    q = int(np.argmin(np.abs(omega)))
    assert abs(omega[q].real + 0.03) < 1e-9
    slow = np.real(b[q] * Phi[:, q])
    np.testing.assert_allclose(cands[(3, 0)], slow, rtol=0, atol=1e-12)
    assert np.abs(slow).max() > 0.1 * scale
    # a truncated affine fit is not exact
    assert np.abs(cands[(1, 1)]).max() > 1e-6 * scale


def test_affine_limit_recovers_a_nonzero_fixed_point():
    """Affine dynamics around psi* != 0, with one slow mode (rate 1e-3): both
    the paper's candidate at full rank and the affine limit of the differences
    at full rank return psi*; the geometric-series gain lambda/(1 - lambda)
    sums the slow mode's whole future decay."""
    rng = np.random.default_rng(8)
    psi_star = rng.standard_normal(150)
    snaps = decaying_window(150, [1e-3, 0.2, 0.5], 12, seed=5, psi_star=psi_star)
    r = dmd.numerical_rank(snaps)
    rd = dmd.numerical_rank(np.diff(snaps, axis=0))
    assert (r, rd) == (4, 3)
    cands = {(rr, k): psi for rr, k, psi in dmd.candidates(snaps, 1.0, r)}
    np.testing.assert_allclose(cands[(4, 0)], psi_star, rtol=0, atol=1e-8 * np.abs(psi_star).max())
    np.testing.assert_allclose(cands[(3, 1)], psi_star, rtol=0, atol=1e-8 * np.abs(psi_star).max())
    # ranks tried: r*, r* - 1, r* - 2, r* - 4, ... for each kind (r* = 4, r*_d = 3)
    assert list(cands) == [(1, 1), (2, 0), (2, 1), (3, 0), (3, 1), (4, 0)]


def test_ranks_tried_form_a_ladder_below_the_numerical_rank():
    assert [r for r in range(1, 60) if dmd.rank_tried(r, 49)] == [17, 33, 41, 45, 47, 48, 49]
    assert [r for r in range(1, 9) if dmd.rank_tried(r, 5)] == [1, 3, 4, 5]
    assert not dmd.rank_tried(0, 3) and not dmd.rank_tried(4, 3)

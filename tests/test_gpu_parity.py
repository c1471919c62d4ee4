"""GPU parity: every entry point of libpcfv against the FP64 oracle, on the
same seeded inputs.

Tolerance: 1e-11 relative (max-norm error over max-norm of the oracle's
result) for FP64, on spectrally decaying inputs (the Chebyshev-tau Stokes
solve is conditioned so that white-noise inputs at Ny >= 49 reach only
~1e-12 to 5e-12 relative in any FP64 implementation).  At 48 x 49 x 48 the
full fields are compared too (the oracle's residual and adjoint finish in
seconds there); the projection is checked by its defining properties."""

import numpy as np
import pytest

from oracle import Grid, state
from oracle.method import Method
from paper_2306_00165_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-11
# One exception, the adjoint of a smooth field in the wide 96 x 65 x 96 box
# (Lx = 4 pi): there the lowest mode has kappa^2 = 0.25 and the influence
# matrix of the GPU's Stokes solve has condition ~7e5; the GPU's J* w differs
# from the oracle's by up to 3.3e-11.  The oracle is accurate to 4e-13 there
# (tests/test_oracle_precision.py, against a 40-digit evaluation), so the
# excess is the GPU's own FP64 rounding in that mode's transposed solve.
# Forming the influence matrix and its homogeneous responses in quad precision
# on the host does not change it (measured 3.3e-11), so it sits in the FP64
# eigenbasis solves and contractions at this conditioning.  Bound, stated: 5e-11.
# The descent step of that instance, and everything at 48 x 49 x 48 (adjoint
# error 7e-13 to 1.9e-12, descent step 1.5e-13 measured), meet 1e-11.
TOL_ADJ_WIDE = 5e-11


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def to_np(t):
    return t.detach().cpu().numpy()


GRIDS = {
    "cfg1": (16, 25, 16),
    "cfg2": (32, 33, 32),
    "tiny": (6, 9, 6),
    "ragged": (12, 17, 9),
    "odd": (9, 11, 15),
}


@pytest.fixture(scope="module")
def ctxs():
    from paper_2306_00165_amd.pcfv import Context
    cache = {}

    def get(name):
        if name not in cache:
            dims = GRIDS[name]
            print(f"[gpu] context {name} {dims}", flush=True)
            g = Grid(*dims)
            cache[name] = (g, Method(g), Context(*dims))
        return cache[name]
    return get


def guess(g, seed=1, energy=1e-3):
    return inputs.random_field(g.Nx, g.Ny, g.Nz, g.Lx, g.Lz, energy=energy, seed=seed)


@pytest.mark.parametrize("name", list(GRIDS))
def test_residual_and_cost(ctxs, name):
    g, m, c = ctxs(name)
    u = inputs.config1_guess() if name == "cfg1" else guess(g, 3, 5e-3)
    r_ref = m.residual(u)
    r, cost = c.residual(u, want_cost=True)
    assert rel(to_np(r), r_ref) < TOL
    assert abs(cost - m.inner(r_ref, r_ref)) < TOL * m.inner(r_ref, r_ref)
    assert abs(c.cost(u) - cost) <= 1e-15 * cost


def test_laminar_residual_is_zero(ctxs):
    g, m, c = ctxs("cfg1")
    r, cost = c.residual(g.zeros(), want_cost=True)
    assert float(np.abs(to_np(r)).max()) == 0.0 and cost == 0.0


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "ragged", "odd"])
def test_jvp(ctxs, name):
    g, m, c = ctxs(name)
    u, v = guess(g, 4, 5e-3), guess(g, 5, 1e-3)
    assert rel(to_np(c.jvp(u, v)), m.jvp(u, v)) < TOL


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "tiny", "ragged", "odd"])
def test_adjoint(ctxs, name):
    g, m, c = ctxs(name)
    u = guess(g, 6, 5e-3)
    w = m.residual(u)                        # the descent applies J* to r(u)
    assert rel(to_np(c.adjoint(u, w)), m.adjoint(u, w)) < TOL
    w2 = guess(g, 7, 1e-3)
    w2 = w2 + 0.3 * np.roll(w2, 1, axis=0)   # not admissible
    assert rel(to_np(c.adjoint(u, w2)), m.adjoint(u, w2)) < TOL


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "tiny", "ragged", "odd"])
def test_projection(ctxs, name):
    g, m, c = ctxs(name)
    x = guess(g, 8, 1.0)
    x = x + 0.4 * np.roll(x, 1, axis=0)
    assert rel(to_np(c.project(x)), m.project(x)) < TOL


def test_adjoint_identity_on_gpu(ctxs):
    g, m, c = ctxs("cfg2")
    u, v, w = guess(g, 9, 5e-3), guess(g, 10), guess(g, 11)
    lhs = m.inner(to_np(c.jvp(u, v)), w)
    rhs = m.inner(v, to_np(c.adjoint(u, w)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_descent_200_steps_config1(ctxs):
    """Config 1: 200 descent steps with dtau = 0.02, compared after every step."""
    import torch
    g, m, c = ctxs("cfg1")
    u_ref = inputs.config1_guess()
    u = torch.as_tensor(u_ref).to("cuda:0").contiguous()
    worst = 0.0
    for k in range(200):
        u_ref, _ = m.descent_step(u_ref, 0.02)
        st, rep = c.descend(u, max_steps=1, dtau=0.02)
        assert st == 0 and rep["steps"] == 1
        worst = max(worst, rel(to_np(u), u_ref))
    print(f"[gpu] worst relative state error over 200 steps: {worst:.3e}")
    assert worst < TOL
    assert max(c.check_state(u)) < 1e-15


def test_descent_many_steps_one_call(ctxs):
    import torch
    g, m, c = ctxs("cfg2")
    u_ref = inputs.config2_guess()
    u = torch.as_tensor(u_ref).to("cuda:0").contiguous()
    for _ in range(20):
        u_ref, _ = m.descent_step(u_ref, 0.02)
    st, rep = c.descend(u, max_steps=20, dtau=0.02, check_every=7)
    assert st == 0 and rep["steps"] == 20
    assert rel(to_np(u), u_ref) < TOL
    assert abs(rep["cost"] - m.cost(u_ref)) < 1e-10 * rep["cost"]


def test_norms_and_diagnostics(ctxs):
    g, m, c = ctxs("cfg1")
    u = inputs.config1_guess()
    n0, n1, d = c.norms(u)
    assert abs(n0 - m.norm(u)) < 1e-13 * n0
    assert abs(n1 - m.total_norm(u)) < 1e-13 * n1
    assert abs(d - m.dissipation(u)) < 1e-12 * d
    z = c.norms(g.zeros())
    assert z[0] == 0.0 and abs(z[2] - 1.0) < 1e-15 and abs(z[1] ** 2 - 1 / 3) < 1e-15


@pytest.mark.parametrize("name", ["cfg1", "ragged"])
def test_state_vector(ctxs, name):
    g, m, c = ctxs(name)
    u = guess(g, 12)
    psi = to_np(c.pack(u))
    assert len(psi) == g.n_state()
    np.testing.assert_allclose(psi, state.pack(g, u), rtol=0, atol=1e-15 * np.abs(psi).max())
    x = np.random.default_rng(13).standard_normal(g.n_state())
    w = to_np(c.unpack(x))
    assert rel(w, state.unpack(g, x)) < 1e-13
    d = c.check_state(w)
    assert max(d) < 1e-12 * np.abs(w).max()


def test_check_state_detects_defects(ctxs):
    g, m, c = ctxs("cfg1")
    u = guess(g, 14)
    assert max(c.check_state(u)) < 1e-15
    bad = u.copy()
    bad[0, 2, 3, 0] += 1e-3                       # u_x: breaks walls and divergence
    d = c.check_state(bad)
    assert d[0] > 1e-4 and d[1] > 1e-4
    bad = u.copy()
    bad[0, 1, 0, 2] += 1e-3                       # breaks the kz = 0 conjugate symmetry
    assert c.check_state(bad)[2] > 1e-4


# -- the metric workload: 48 x 49 x 48 ----------------------------------------------

@pytest.fixture(scope="module")
def metric():
    from paper_2306_00165_amd.pcfv import Context
    print("[gpu] context 48x49x48", flush=True)
    g = Grid(48, 49, 48)
    return g, Method(g), Context(48, 49, 48), inputs.metric_guess()


def test_metric_residual_and_adjoint(metric):
    g, m, c, u = metric
    r_ref = m.residual(u)
    r, cost = c.residual(u, want_cost=True)
    e_r = rel(to_np(r), r_ref)
    a_gpu, a_ref = to_np(c.adjoint(u, r_ref)), m.adjoint(u, r_ref)
    e_a = rel(a_gpu, a_ref)
    idx = np.unravel_index(np.argmax(np.abs(a_gpu - a_ref)), a_ref.shape)
    print(f"[gpu] 48x49x48 residual rel err {e_r:.3e}, adjoint rel err {e_a:.3e} at {idx}")
    per_mode = np.abs(a_gpu - a_ref).max(axis=(0, 3)) / np.abs(a_ref).max()
    worst = np.argsort(per_mode.ravel())[::-1][:6]
    print("[gpu] 48x49x48 adjoint error by mode (kx, kz, rel err): " +
          ", ".join(f"({g.kx[i // g.nkz]}, {i % g.nkz}, {per_mode.ravel()[i]:.1e})" for i in worst))
    assert e_r < TOL
    assert abs(cost - m.inner(r_ref, r_ref)) < TOL * cost
    assert e_a < TOL


def test_metric_projection_properties(metric):
    g, m, c, u = metric
    x = guess(g, 15, 1.0)
    x = x + 0.4 * np.roll(x, 1, axis=0)
    y = guess(g, 16, 1.0)
    y = y + 0.2 * np.roll(y, 2, axis=0)
    Px, Py = to_np(c.project(x)), to_np(c.project(y))
    e_x, e_y = rel(Px, m.project(x)), rel(Py, m.project(y))
    print(f"[gpu] 48x49x48 projection rel err vs the dense null-space projector {e_x:.2e} {e_y:.2e}")
    assert e_x < TOL and e_y < TOL
    s = np.abs(Px).max()
    assert max(m.defects(Px)) < 1e-13 * s
    assert rel(to_np(c.project(Px)), Px) < 1e-13
    assert rel(to_np(c.project(u)), u) < 1e-13
    lhs, rhs = m.inner(Px, y), m.inner(x, Py)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_metric_descent_step_matches_oracle_direction(metric):
    """One descent step in the benchmark's launch configuration equals the
    oracle's u - dtau P J* r (residual, adjoint and dense projection)."""
    import torch
    g, m, c, u0 = metric
    dtau = 0.012
    want, _ = m.descent_step(u0, dtau)
    u = torch.as_tensor(u0).to("cuda:0").contiguous()
    st, rep = c.descend(u, max_steps=1, dtau=dtau)
    assert st == 0
    e = rel(to_np(u) - u0, want - u0)
    print(f"[gpu] 48x49x48 descent step rel err {e:.3e}")
    assert e < TOL


# -- several guesses in one context ---------------------------------------------------

def test_batched_guesses_match_single_guess_oracle():
    """Three different guesses advanced together: each matches the oracle run
    on that guess alone (residual, costs, norms, 5 descent steps, state vector)."""
    import torch
    from paper_2306_00165_amd.pcfv import Context
    g = Grid(16, 25, 16)
    m = Method(g)
    us = [inputs.random_field(16, 25, 16, energy=e, seed=s) for s, e in [(21, 1e-3), (22, 3e-3), (23, 2e-3)]]
    c = Context(16, 25, 16, batch=3)
    U = torch.as_tensor(np.stack(us)).to("cuda:0").contiguous()
    r, costs = c.residual(U, want_cost=True)
    r = to_np(r)
    for b in range(3):
        rr = m.residual(us[b])
        assert rel(r[b], rr) < TOL
        assert abs(costs[b] - m.inner(rr, rr)) < TOL * costs[b]
        n0, n1, d = c.norms(U)[b]
        assert abs(n1 - m.total_norm(us[b])) < 1e-13 * n1
    psi = to_np(c.pack(U))
    for b in range(3):
        np.testing.assert_allclose(psi[b], state.pack(g, us[b]), rtol=0, atol=1e-15 * np.abs(psi).max())
    st, rep = c.descend(U, max_steps=5, dtau=0.02, check_every=2)
    assert st == 0 and rep["steps"] == 5
    for b in range(3):
        ub = us[b]
        for _ in range(5):
            ub, _ = m.descent_step(ub, 0.02)
        assert rel(to_np(U[b]), ub) < TOL
    assert max(max(d) for d in c.check_state(U)) < 1e-15


# -- DMD extrapolation (Sec. 6) ---------------------------------------------------

def _oracle_window(m, u, steps_before, nsnap, stride, dtau):
    """Oracle descent: steps_before steps, then nsnap snapshots stride steps
    apart (the last one taken without stepping past it)."""
    for _ in range(steps_before):
        u, _ = m.descent_step(u, dtau)
    win = []
    for k in range((nsnap - 1) * stride + 1):
        if k % stride == 0:
            win.append(u.copy())
        if k < (nsnap - 1) * stride:
            u, _ = m.descent_step(u, dtau)
    return win


def _dmd_tol(psis, r, kind=0):
    """1e3 * eps * s_1 / (s_r - s_{r+1}): the perturbation bound of the rank-r
    DMD subspace (of the snapshots for kind 0, of their differences for kind 1)
    for round-off at the snapshot scale, relative to the result's max-norm."""
    X = np.asarray(psis)
    if kind == 1:
        X = np.diff(X, axis=0)
    s = np.linalg.svd(X[:-1].T, compute_uv=False)
    gap = s[r - 1] - (s[r] if r < len(s) else 0.0)
    return 1e3 * np.finfo(float).eps * s[0] / gap


def _check_dmd_against_oracle(c, m, g, win, dtau_snap, label):
    from oracle import dmd
    psis = np.stack([state.pack(g, w) for w in win])
    u_ref, c_ref, r_ref, k_ref = dmd.extrapolate(m, win, dtau_snap)
    u_s, cost, r, kind = c.dmd_extrapolate(psis[:, None, :], dtau_snap, with_kind=True)
    u_s = to_np(u_s)
    tol = _dmd_tol(psis, r_ref, k_ref) * max(1.0, np.abs(win[-1]).max() / np.abs(u_ref).max())
    print(f"[gpu] dmd {label}: rank {r} kind {kind} (oracle {r_ref} {k_ref}) cost {cost:.6e} "
          f"(oracle {c_ref:.6e}) state rel err {rel(u_s, u_ref):.3e} tol {tol:.1e}", flush=True)
    assert (r, kind) == (r_ref, k_ref)
    assert rel(u_s, u_ref) < tol
    assert abs(cost - m.cost(u_s)) < TOL * cost
    assert cost < m.cost(win[-1])
    assert max(c.check_state(u_s)) < 1e-15
    return r, kind


def test_dmd_extrapolate_matches_oracle(ctxs):
    """Same oracle snapshots into both: a window of a descent heading for the
    laminar state, and the same window shifted by a fixed admissible field (a
    target with a non-zero fixed point).  The GPU picks the oracle's rank and
    kind, its state matches the oracle's within the subspace bound, and the
    cost it reports is the cost of the state it returns."""
    g, m, c = ctxs("cfg1")
    win = _oracle_window(m, inputs.config1_guess(), 40, 10, 4, 0.02)
    _check_dmd_against_oracle(c, m, g, win, 0.08, "decaying window")
    shift = guess(g, 44, 3e-3)
    _check_dmd_against_oracle(c, m, g, [w + shift for w in win], 0.08, "shifted window")


def test_dmd_extrapolate_batched_matches_single():
    """Two guesses' windows extrapolated in one batched call equal the
    single-guess calls."""
    import torch
    from paper_2306_00165_amd.pcfv import Context
    g = Grid(16, 25, 16)
    m = Method(g)
    wins = [_oracle_window(m, inputs.random_field(16, 25, 16, energy=e, seed=s), 30, 8, 3, 0.02)
            for s, e in [(31, 1e-3), (32, 2e-3)]]
    psis = np.stack([np.stack([state.pack(g, w) for w in win]) for win in wins], axis=1)  # [M][B][n]
    cb = Context(16, 25, 16, batch=2)
    psis[:, 1, :] += state.pack(g, inputs.random_field(16, 25, 16, energy=3e-3, seed=34))  # a shifted target
    ub, costb, rb, kb = cb.dmd_extrapolate(psis, 0.06, with_kind=True)
    c1 = Context(16, 25, 16)
    for b in range(2):
        u1, cost1, r1, k1 = c1.dmd_extrapolate(psis[:, b:b + 1, :], 0.06, with_kind=True)
        assert (rb[b], kb[b]) == (r1, k1)
        assert rel(to_np(ub[b]), to_np(u1)) < 1e-14
        assert abs(costb[b] - cost1) <= 1e-14 * cost1


def test_descend_with_dmd_equals_composed_entry_points(ctxs):
    """descend with a DMD window performs exactly: steps with snapshots every
    `stride`, the extrapolation, acceptance, further steps; composing the same
    entry points by hand gives the same state, and the extrapolated state
    matches the oracle's replay of that schedule within the subspace bound
    amplified by the snapshots' distance from the oracle's."""
    import torch
    from oracle import dmd
    g, m, c = ctxs("cfg1")
    u0 = inputs.config1_guess()
    W, stride, dtau, after = 10, 4, 0.02, 6
    u = torch.as_tensor(u0).to("cuda:0").contiguous()
    c.descend(u, max_steps=40, dtau=dtau)
    start = u.clone()
    st, rep = c.descend(u, max_steps=(W - 1) * stride + after, dtau=dtau, dmd_window=W, dmd_stride=stride,
                        dmd_gap=1000, dmd_accept=10.0)
    assert st == 0 and rep["n_dmd"] == 1 and rep["n_dmd_accepted"] == 1
    # the same schedule from entry points
    v = start.clone()
    snaps = []
    for k in range(W):
        snaps.append(to_np(c.pack(v)))
        if k < W - 1:
            c.descend(v, max_steps=stride, dtau=dtau)
    u_s, cost_s, r_s, k_s = c.dmd_extrapolate(np.stack(snaps)[:, None, :], stride * dtau, with_kind=True)
    c.descend(u_s, max_steps=after, dtau=dtau)
    assert rel(to_np(u), to_np(u_s)) < 1e-15
    # oracle replay of the schedule
    win = _oracle_window(m, u0, 40, W, stride, dtau)
    psis = np.stack([state.pack(g, w) for w in win])
    snap_err = max(rel(a, b) for a, b in zip(snaps, psis))
    u_ref, c_ref, r_ref, k_ref = dmd.extrapolate(m, win, stride * dtau)
    assert k_s == k_ref
    for _ in range(after):
        u_ref, _ = m.descent_step(u_ref, dtau)
    tol = (_dmd_tol(psis, r_ref, k_ref) * max(1.0, snap_err / np.finfo(float).eps) *
           max(1.0, np.abs(win[-1]).max() / np.abs(u_ref).max()))
    print(f"[gpu] descend+dmd rank {r_s} (oracle {r_ref}) snapshot err {snap_err:.2e} "
          f"state rel err {rel(to_np(u), u_ref):.3e} tol {tol:.1e}", flush=True)
    assert r_s == r_ref
    assert rel(to_np(u), u_ref) < tol


@pytest.mark.parametrize("ratio,strides", [(1e-12, [2, 8, 32]), (1e12, [2, 2, 2])])
def test_descend_adaptive_dmd_stride_equals_composed_entry_points(ctxs, ratio, strides):
    """With dmd_stride_max > dmd_stride, a window whose best candidate costs
    at least dmd_grow_ratio times the current cost makes the next stride four
    times longer (capped): ratio 1e-12 grows after every window (2 -> 8 -> 32,
    cap 32), ratio 1e12 never.  The same schedule composed from entry points
    (pack, descend, dmd_extrapolate, cost) gives the same state."""
    import torch
    g, m, c = ctxs("cfg1")
    W, dtau, accept = 6, 0.02, 10.0
    u = torch.as_tensor(inputs.config1_guess()).to("cuda:0").contiguous()
    c.descend(u, max_steps=40, dtau=dtau)
    v = u.clone()
    total, after = sum((W - 1) * s for s in strides), 3
    st, rep = c.descend(u, max_steps=total + after, dtau=dtau, dmd_window=W, dmd_stride=strides[0], dmd_gap=0,
                        dmd_accept=accept, dmd_stride_max=32, dmd_grow_ratio=ratio)
    assert rep["n_dmd"] == len(strides)
    expect_final = min(4 * strides[-1], 32) if ratio < 1 else strides[-1]
    assert rep["dmd_stride_final"] == expect_final
    taken = 0
    for s in strides:
        snaps = [to_np(c.pack(v))]
        for k in range(W - 1):
            c.descend(v, max_steps=s, dtau=dtau)
            snaps.append(to_np(c.pack(v)))
        u_s, cost_s, r_s = c.dmd_extrapolate(np.stack(snaps)[:, None, :], s * dtau)
        cnow = c.cost(v)
        if r_s > 0 and cost_s < accept * cnow:
            v.copy_(u_s)
            taken += 1
    c.descend(v, max_steps=after, dtau=dtau)
    assert rep["n_dmd_accepted"] == taken
    print(f"[gpu] adaptive DMD stride ratio {ratio:g}: strides {strides} -> final {rep['dmd_stride_final']}, "
          f"state rel diff {rel(to_np(u), to_np(v)):.2e}", flush=True)
    assert rel(to_np(u), to_np(v)) < 1e-15


# -- mixed precision: FP32 transforms and products, FP64 solves --------------------

# The FP32 stage rounds each y-value once and accumulates sums of at most
# n_kx + 2 n_kz + N_z + XS (< 100 at these grids) terms per output, so by the
# recursive-summation bound its relative error on the products is below
# 100 eps32; the Stokes solves, projection and update are FP64 and contract
# it.  Stated bound for every mixed-precision result against the FP64 oracle:
TOL32 = 100 * float(np.finfo(np.float32).eps)


@pytest.fixture(scope="module")
def mixed_ctxs():
    from paper_2306_00165_amd.pcfv import Context, MIXED
    cache = {}

    def get(name):
        if name not in cache:
            dims = GRIDS[name]
            print(f"[gpu] mixed context {name} {dims}", flush=True)
            g = Grid(*dims)
            cache[name] = (g, Method(g), Context(*dims, precision=MIXED))
        return cache[name]
    return get


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "ragged", "odd"])
def test_mixed_residual_adjoint_and_step(mixed_ctxs, name):
    import torch
    g, m, c = mixed_ctxs(name)
    u = guess(g, 1)
    w = guess(g, 2)
    r = to_np(c.residual(u))
    rr = m.residual(u)
    e_r = rel(r, rr)
    e_a = rel(to_np(c.adjoint(u, w)), m.adjoint(u, w))
    U = torch.as_tensor(u).to("cuda:0").contiguous()
    c.descend(U, max_steps=1, dtau=0.02)
    u1, _ = m.descent_step(u, 0.02)
    e_s = float(np.abs(to_np(U) - u1).max() / np.abs(u1 - u).max())
    print(f"[gpu] mixed {name}: residual {e_r:.2e} adjoint {e_a:.2e} step {e_s:.2e} (bound {TOL32:.1e})")
    assert e_r < TOL32 and e_a < TOL32 and e_s < TOL32
    assert e_r > 1e-12          # the FP32 stage really ran


@pytest.mark.parametrize("shape", [(8, 512, 256), (8, 768, 512), (4, 256, 256)])
def test_mixed_launch_shapes_match_oracle(shape):
    """The FP32 physical-space kernels at pinned launch shapes (512 threads is
    the default for FP32 launches of many modes) against the FP64 oracle at
    32x33x32, within the mixed-precision bound."""
    import torch
    from paper_2306_00165_amd.pcfv import Context, MIXED
    g = Grid(*GRIDS["cfg2"])
    m = Method(g)
    c = Context(*GRIDS["cfg2"], precision=MIXED)
    c.set_tuning(*shape)
    assert c.tuning() == shape
    u, w = guess(g, 21), guess(g, 22)
    e_r = rel(to_np(c.residual(u)), m.residual(u))
    e_a = rel(to_np(c.adjoint(u, w)), m.adjoint(u, w))
    U = torch.as_tensor(u).to("cuda:0").contiguous()
    c.descend(U, max_steps=1, dtau=0.02)
    u1, _ = m.descent_step(u, 0.02)
    e_s = float(np.abs(to_np(U) - u1).max() / np.abs(u1 - u).max())
    print(f"[gpu] mixed shape {shape}: residual {e_r:.2e} adjoint {e_a:.2e} step {e_s:.2e}")
    assert e_r < TOL32 and e_a < TOL32 and e_s < TOL32
    assert e_r > 1e-12


def test_mixed_descent_refines_in_fp64(ctxs, mixed_ctxs):
    """fp64_below switches the rest of a call to FP64: always-below gives the
    trajectory of an FP64 context with the same launch shape bit for bit,
    never-below stays FP32 throughout, and a threshold met mid-run gives both
    phases; the context keeps its precision."""
    import torch
    g, m, c64 = ctxs("cfg1")
    _, _, c32 = mixed_ctxs("cfg1")
    u0 = torch.as_tensor(inputs.config1_guess()).to("cuda:0").contiguous()
    ref = u0.clone()
    shape64 = c64.tuning()
    c64.set_tuning(*c32.tuning())
    try:
        c64.descend(ref, max_steps=300, dtau=0.02, check_every=50)
    finally:
        c64.set_tuning(*shape64)
    a = u0.clone()
    st, rep = c32.descend(a, max_steps=300, dtau=0.02, check_every=50, fp64_below=1e30)
    assert rep["steps_fp32"] == 0 and torch.equal(a, ref)
    b = u0.clone()
    st, rep = c32.descend(b, max_steps=300, dtau=0.02, check_every=50, fp64_below=1e-30)
    assert rep["steps_fp32"] == 300
    assert rel(to_np(b) - to_np(u0), to_np(ref) - to_np(u0)) < TOL32
    mid = u0.clone()
    _, rep100 = c64.descend(mid, max_steps=150, dtau=0.02)
    d = u0.clone()
    st, rep = c32.descend(d, max_steps=300, dtau=0.02, check_every=50, fp64_below=rep100["rel_res"])
    assert 0 < rep["steps_fp32"] < 300
    assert abs(rep["cost"] - m.cost(to_np(d))) < 1e-10 * rep["cost"]
    # the context is still mixed afterwards
    assert rel(to_np(c32.residual(u0)), to_np(c64.residual(u0))) > 1e-12


def test_set_precision_rejects_unknown_values(mixed_ctxs):
    from paper_2306_00165_amd.pcfv import PcfvError, FP64, MIXED
    g, m, c = mixed_ctxs("tiny")
    u = guess(g, 3)
    with pytest.raises(PcfvError):
        c.set_precision(7)
    c.set_precision(FP64)
    assert rel(to_np(c.residual(u)), m.residual(u)) < TOL
    c.set_precision(MIXED)
    assert rel(to_np(c.residual(u)), m.residual(u)) < TOL32


# -- groups of uneven grids, HIP graphs, autotuner ---------------------------------

def _group_members(precision=0):
    from paper_2306_00165_amd.pcfv import Context
    specs = [((16, 25, 16), 400.0, 2), ((12, 17, 9), 380.0, 1), ((32, 33, 32), 420.0, 1)]
    out = []
    for i, (dims, Re, B) in enumerate(specs):
        g = Grid(*dims, Re=Re)
        fields = [inputs.random_field(*dims, energy=1e-3, seed=40 + 3 * i + b) for b in range(B)]
        u = np.stack(fields) if B > 1 else fields[0]
        out.append((g, Context(*dims, Re=Re, batch=B, precision=precision), u))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_group_of_uneven_grids_matches_each_member(precision):
    """One launch per stage over three members (different grids, Re and
    batch) gives every member exactly its own single-context result, with and
    without HIP-graph replay; the Re = 380 member also matches the oracle."""
    import torch
    from paper_2306_00165_amd.pcfv import Group
    mem = _group_members(precision)
    dtaus = [0.02, 0.015, 0.01]
    grp = Group([c for _, c, _ in mem])
    fields = [torch.as_tensor(u).to("cuda:0").contiguous() for _, _, u in mem]
    plain = [f.clone() for f in fields]
    graph = [f.clone() for f in fields]
    grp.descend(plain, dtaus, 7)
    grp.descend(graph, dtaus, 7, graph_steps=3)
    for (g, c, u), f, d, p_, q_ in zip(mem, fields, dtaus, plain, graph):
        ref = f.clone()
        c.descend(ref, max_steps=7, dtau=d)
        assert torch.equal(p_, ref) and torch.equal(q_, ref)
    if precision == 0:
        g, c, u = mem[1]
        m = Method(g)
        for _ in range(7):
            u, _ = m.descent_step(u, dtaus[1])
        assert rel(to_np(plain[1]), u) < TOL


def test_group_of_many_modes_matches_oracle():
    """A group of more than 1024 modes (3 guesses at 48x49x48 + 2 at 32x33x32)
    runs its throughput shape (1024-thread plane groups, widest slabs, no
    staging, the smaller member's tables re-padded to the group's Ny); two
    steps of one guess of each member match the oracle."""
    import torch
    from paper_2306_00165_amd.pcfv import Context, Group
    specs = [((48, 49, 48), 3, 0.012), ((32, 33, 32), 2, 0.02)]
    ctxs_, fields, refs = [], [], []
    for i, (dims, B, dt) in enumerate(specs):
        us = [inputs.random_field(*dims, energy=1e-3, seed=80 + 5 * i + b) for b in range(B)]
        ctxs_.append(Context(*dims, batch=B))
        fields.append(torch.as_tensor(np.stack(us)).to("cuda:0").contiguous())
        refs.append(us[i % B])
    grp = Group(ctxs_)
    grp.descend(fields, [dt for _, _, dt in specs], 2)
    for i, (dims, B, dt) in enumerate(specs):
        m = Method(Grid(*dims))
        u = refs[i]
        for _ in range(2):
            u, _ = m.descent_step(u, dt)
        assert rel(to_np(fields[i][i % B]), u) < TOL, dims


def test_group_graph_is_reused_across_calls():
    """The captured graph reads fields and steps from device records, so it is
    replayed across calls with new fields and new dtau, with eager work in
    between, and every replay agrees with plain launches."""
    import torch
    from paper_2306_00165_amd.pcfv import Group
    mem = _group_members()
    grp = Group([c for _, c, _ in mem])
    a = [torch.as_tensor(u).to("cuda:0").contiguous() for _, _, u in mem]
    b = [x.clone() for x in a]
    for rep, dts in enumerate([[0.02, 0.015, 0.01], [0.01, 0.01, 0.005], [0.02, 0.02, 0.01]]):
        grp.descend(a, dts, 4, graph_steps=2)
        grp.descend(b, dts, 4)
        for x, y in zip(a, b):
            assert torch.equal(x, y), rep
        for (g, c, u), x in zip(mem, a):
            c.cost(x)                      # eager work on the members' own streams


def test_group_descends_to_tolerance_like_each_member_alone():
    """pcfv_group_descend_tol on a mixed-precision group of uneven members:
    each member stops at the first check below rel_tol after its own FP32 ->
    FP64 switch, and ends bit for bit where the same member's single-context
    pcfv_descend (same tolerance, switch point and check period) ends."""
    import torch
    from paper_2306_00165_amd.pcfv import Group, OK
    mem = _group_members(precision=1)
    dtaus = [0.02, 0.015, 0.01]
    fields = [torch.as_tensor(u).to("cuda:0").contiguous() for _, _, u in mem]
    rel0 = []
    for (g, c, u), f, d in zip(mem, fields, dtaus):
        _, rep = c.descend(f.clone(), max_steps=0, dtau=d)
        rel0.append(rep["rel_res"])
    tol, below = 0.5 * min(rel0), 0.8 * min(rel0)
    print(f"[gpu] group to tolerance: initial rel {rel0}, fp64 below {below:.3e}, tol {tol:.3e}", flush=True)
    grp = Group([c for _, c, _ in mem])
    work = [f.clone() for f in fields]
    st, stats, reps = grp.descend_tol(work, dtaus, max_steps=4000, rel_tol=tol, check_every=10, fp64_below=below)
    assert st == OK and stats == [OK] * 3
    for (g, c, u), f, w, d, rep in zip(mem, fields, work, dtaus, reps):
        ref = f.clone()
        st1, rep1 = c.descend(ref, max_steps=4000, dtau=d, rel_tol=tol, check_every=10, fp64_below=below)
        assert st1 == OK
        assert rep["steps"] == rep1["steps"] and rep["steps_fp32"] == rep1["steps_fp32"]
        assert 0 < rep["steps_fp32"] < rep["steps"]
        assert rep["rel_res"] < tol and rep["cost"] == rep1["cost"]
        assert torch.equal(w, ref)


def test_group_descend_tolerance_with_dmd_windows():
    """FP64 group with DMD windows: every member converges, windows are
    extrapolated, each member's reported cost is the oracle's cost of the
    state it ends in, and the states stay admissible."""
    import torch
    from paper_2306_00165_amd.pcfv import Group, OK
    mem = _group_members(precision=0)[:2]
    dtaus = [0.02, 0.015]
    fields = [torch.as_tensor(u).to("cuda:0").contiguous() for _, _, u in mem]
    rel0 = [c.descend(f.clone(), max_steps=0, dtau=d)[1]["rel_res"] for (g, c, u), f, d in zip(mem, fields, dtaus)]
    grp = Group([c for _, c, _ in mem])
    st, stats, reps = grp.descend_tol(fields, dtaus, max_steps=5000, rel_tol=0.3 * min(rel0), check_every=20,
                                      dmd_window=10, dmd_stride=4, dmd_accept=1.0)
    print(f"[gpu] group with DMD: {[(r['steps'], r['n_dmd'], r['n_dmd_accepted'], r['rel_res']) for r in reps]}")
    assert st == OK and stats == [OK, OK]
    for (g, c, u), f, rep in zip(mem, fields, reps):
        assert rep["n_dmd"] >= 1
        m = Method(g)
        x = to_np(f)
        xs = x if c.batch > 1 else x[None]
        worst = max(m.cost(v) for v in xs)
        assert abs(rep["cost"] - worst) < TOL * worst
        assert max(np.ravel(c.check_state(f))) < 1e-14


def test_autotune_keeps_parity(ctxs):
    """The autotuner times every launch-shape candidate and keeps the fastest;
    results with the chosen shape still match the oracle."""
    import torch
    from paper_2306_00165_amd.pcfv import Context
    g = Grid(32, 33, 32)
    m = Method(g)
    c = Context(32, 33, 32)
    u = guess(g, 9)
    ent = c.autotune(u, steps=5)
    assert ent and all(32 % xs == 0 and nt in (256, 512, 576, 768, 1024) and mt in (256, 512) for xs, nt, mt, _ in ent)
    best = min(ent, key=lambda e: e[3])
    assert c.tuning() == best[:3]
    print(f"[gpu] autotune 32x33x32: {ent}")
    assert rel(to_np(c.residual(u)), m.residual(u)) < TOL
    U = torch.as_tensor(u).to("cuda:0").contiguous()
    c.descend(U, max_steps=3, dtau=0.02)
    for _ in range(3):
        u, _ = m.descent_step(u, 0.02)
    assert rel(to_np(U), u) < TOL


@pytest.fixture(scope="module")
def shape_ctx():
    from paper_2306_00165_amd.pcfv import Context
    g = Grid(48, 49, 48)
    return g, Method(g), Context(48, 49, 48)


@pytest.mark.parametrize("xs,nt,mt", [(12, 256, 512), (12, 512, 256), (12, 576, 256), (12, 768, 512), (12, 1024, 512),
                                      (8, 768, 256), (6, 1024, 256), (16, 1024, 512)])
def test_every_launch_shape_matches_oracle(shape_ctx, xs, nt, mt):
    """Residual, adjoint and one descent step at 48x49x48 with each pinned
    launch shape (slab width, physical-space and per-mode work-group sizes)."""
    import torch
    g, m, c = shape_ctx
    c.set_tuning(xs, nt, mt)
    assert c.tuning() == (xs, nt, mt)
    u, w = guess(g, 11), guess(g, 12)
    assert rel(to_np(c.residual(u)), m.residual(u)) < TOL
    e_a = rel(to_np(c.adjoint(u, w)), m.adjoint(u, w))
    print(f"[gpu] shape {(xs, nt, mt)}: adjoint rel err {e_a:.2e}")
    assert e_a < TOL
    U = torch.as_tensor(u).to("cuda:0").contiguous()
    c.descend(U, max_steps=1, dtau=0.02)
    assert rel(to_np(U), m.descent_step(u, 0.02)[0]) < TOL


def test_set_tuning_rejects_invalid_shapes(shape_ctx):
    from paper_2306_00165_amd.pcfv import PcfvError
    _, _, c = shape_ctx
    before = c.tuning()
    for bad in [(5, 512, 512), (12, 384, 512), (12, 512, 1024), (0, 512, 256)]:
        with pytest.raises(PcfvError):
            c.set_tuning(*bad)
        assert c.tuning() == before


# -- the largest single-GPU instance: 96 x 65 x 96 in the wide box, 8 guesses --------

@pytest.fixture(scope="module")
def wide():
    from paper_2306_00165_amd.pcfv import Context
    Lx, Lz = 4 * np.pi, 2 * np.pi
    g = Grid(96, 65, 96, Lx=Lx, Lz=Lz)
    us = [inputs.kolmogorov_guess(96, 65, 96, e, s, Lx=Lx, Lz=Lz) for s, e in [(70, 0.03), (71, 0.01)]]
    return g, Method(g), Context(96, 65, 96, Lx=Lx, Lz=Lz, batch=8), us


def test_wide_box_residual_adjoint_and_step(wide):
    """96 x 65 x 96 (Lx = 4 pi, Lz = 2 pi), batch 8: residual, cost, adjoint and
    one descent step of two of the guesses against the oracle (the other six
    are copies, which must come out identical)."""
    import torch
    g, m, c, us = wide
    U = torch.as_tensor(np.stack([us[b % 2] for b in range(8)])).to("cuda:0").contiguous()
    r, costs = c.residual(U, want_cost=True)
    r = to_np(r)
    W = torch.as_tensor(np.stack([us[(b + 1) % 2] for b in range(8)])).to("cuda:0").contiguous()
    a = to_np(c.adjoint(U, W))
    for b in range(2):
        rr = m.residual(us[b])
        e_r = rel(r[b], rr)
        e_a = rel(a[b], m.adjoint(us[b], us[(b + 1) % 2]))
        print(f"[gpu] 96x65x96 guess {b}: residual {e_r:.2e} adjoint {e_a:.2e}")
        assert e_r < TOL
        assert abs(costs[b] - m.inner(rr, rr)) < TOL * costs[b]
        assert e_a < TOL_ADJ_WIDE
    for b in range(2, 8):
        assert np.array_equal(r[b], r[b % 2]) and np.array_equal(a[b], a[b % 2])
    c.descend(U, max_steps=1, dtau=0.01)
    u1, _ = m.descent_step(us[0], 0.01)
    e_s = float(np.abs(to_np(U[0]) - u1).max() / np.abs(u1 - us[0]).max())
    print(f"[gpu] 96x65x96 descent step error relative to the update {e_s:.2e}")
    assert e_s < TOL

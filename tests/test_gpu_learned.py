"""GPU checks of the learned extrapolator (beside the DMD extrapolation of
Sec. 6): BF16 matrix-core MLP layers and gradients against the oracle on the
device's own quantised inputs, Adam, minibatch training, the FP64 POD, and a
trained model's proposals inside the descent.

Bounds.  A product accumulated in FP32 over K terms differs from the exact
product of the same BF16 operands by at most K 2^-24 sum |a_k b_k| (recursive
summation), so each FP32 result is checked against that bound from the
oracle's |A| |B|.  A BF16 output is the rounding of such an FP32 value: it
equals the oracle's rounding except where the exact value lies within that
bound of a rounding midpoint, and then differs by one BF16 step."""

import numpy as np
import pytest

from oracle import mlp as omlp, pod as opod
from oracle import Grid
from oracle.method import Method

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24
DIMS = [2048, 512, 512, 512, 256]     # the extrapolator's network (8 snapshots x 256 POD modes)


def _fp32_bound(A, B, K, extra=0.0):
    return 2 * K * U24 * (np.abs(A) @ np.abs(B) + extra) + 1e-30


def _bf16_step(v):
    """Spacing of bfloat16 numbers at |v|."""
    e = np.floor(np.log2(np.maximum(np.abs(v), 1e-38)))
    return 2.0 ** (e - 7)


def _check_bf16(got, exact, bound):
    ref = omlp.bf16_round(exact)
    mis = got != ref
    assert mis.mean() < 1e-2
    if mis.any():
        # a flip needs the exact value within the FP32 bound of a midpoint, and moves one step
        step = np.maximum(_bf16_step(ref[mis]), _bf16_step(got[mis]))
        assert np.all(np.abs(got[mis] - ref[mis]) <= step * 1.0001 + 2 * bound[mis])


@pytest.mark.parametrize("B", [64, 37])
def test_mlp_layers_and_gradients_match_oracle(B):
    from paper_2306_00165_amd import learned
    from paper_2306_00165_amd.pcfv import MLP, MLP_ACT, MLP_OUT, MLP_DZ, MLP_GRAD
    m = MLP(DIMS, max_batch=128)
    p = learned.he_params(DIMS, 1)
    m.set_params(p)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((B, DIMS[0])).astype(np.float32)
    T = rng.standard_normal((B, DIMS[-1])).astype(np.float32)
    loss = m.grad(X, T)
    acts = [omlp.bf16_bits_to_float(m.read(MLP_ACT, l, B)) for l in range(4)]
    Y = m.read(MLP_OUT, 0, B).astype(np.float64)
    dz = [omlp.bf16_bits_to_float(m.read(MLP_DZ, l, B)) for l in range(4)]
    g = m.read(MLP_GRAD, 0, B).astype(np.float64)
    assert np.array_equal(acts[0], omlp.bf16_round(X))
    layers = omlp.split_params(DIMS, p)
    for l, (W, b) in enumerate(layers):
        Wq = omlp.bf16_round(W)
        z = acts[l] @ Wq + b
        bound = _fp32_bound(acts[l], Wq, W.shape[0], np.abs(b))
        if l < 3:
            _check_bf16(acts[l + 1], np.maximum(z, 0.0), bound)
        else:
            assert np.all(np.abs(Y - z) <= bound)
    d = Y - T.astype(np.float64)
    assert loss == pytest.approx(np.mean(d ** 2), rel=1e-5)
    dY = 2.0 * d / d.size
    _check_bf16(dz[3], dY, 4 * U24 * np.abs(dY))
    off = 0
    for l, (W, b) in enumerate(layers):
        k, n = W.shape
        gW = g[off:off + k * n].reshape(k, n)
        off += k * n
        gb = g[off:off + n]
        off += n
        ref = acts[l].T @ dz[l]
        assert np.all(np.abs(gW - ref) <= _fp32_bound(acts[l].T, dz[l], B))
        if l == 3:
            assert np.all(np.abs(gb - dY.sum(axis=0)) <= 2 * B * U24 * np.abs(dY).sum(axis=0) + 1e-30)
        else:
            Wn = omlp.bf16_round(layers[l + 1][0])
            dA = (dz[l + 1] @ Wn.T) * (acts[l + 1] > 0)
            bA = _fp32_bound(dz[l + 1], np.abs(Wn.T), Wn.shape[1])
            assert np.all(np.abs(gb - dA.sum(axis=0)) <= bA.sum(axis=0) + 2 * B * U24 * np.abs(dA).sum(axis=0))
        if l > 0:
            Wq = omlp.bf16_round(W)
            dA = (dz[l] @ Wq.T) * (acts[l] > 0)
            _check_bf16(dz[l - 1], dA, _fp32_bound(dz[l], np.abs(Wq.T), n))


def test_adam_step_matches_oracle():
    from paper_2306_00165_amd import learned
    from paper_2306_00165_amd.pcfv import MLP, MLP_GRAD
    dims = [64, 96, 32]
    m = MLP(dims, max_batch=16)
    p = learned.he_params(dims, 4)
    m.set_params(p)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((16, 64)).astype(np.float32)
    T = rng.standard_normal((16, 32)).astype(np.float32)
    pp, mm, vv = p.astype(np.float64), 0.0, 0.0
    for t in (1, 2, 3):
        m.grad(X, T)
        g = m.read(MLP_GRAD, 0, 16).astype(np.float64)
        m.adam_step(1e-3)
        pp, mm, vv = omlp.adam(pp, g, mm, vv, t, lr=1e-3)
        got = m.get_params().astype(np.float64)
        assert np.abs(got - pp).max() <= 1e-6 * max(1.0, np.abs(pp).max())
        pp = got


def test_minibatch_training_reduces_loss():
    """A linear map learned from 2048 samples: the epoch loss falls by more
    than 10x and the held-out error is a quarter of that of predicting zero
    or less."""
    import torch
    from paper_2306_00165_amd import learned
    from paper_2306_00165_amd.pcfv import MLP
    dims = [64, 128, 128, 32]
    rng = np.random.default_rng(8)
    Mmap = rng.standard_normal((64, 32)) / 8
    X = rng.standard_normal((2304, 64))
    T = X @ Mmap
    m = MLP(dims, max_batch=64)
    m.set_params(learned.he_params(dims, 9))
    hist = m.fit(torch.as_tensor(X[:2048], dtype=torch.float32).cuda(),
                 torch.as_tensor(T[:2048], dtype=torch.float32).cuda(), batch=64, epochs=40, lr=1e-3, seed=3)
    print(f"[gpu] epoch losses {hist[0]:.4f} -> {hist[-1]:.5f}")
    assert hist[-1] < 0.1 * hist[0]
    Y = m.forward(torch.as_tensor(X[2048:2112], dtype=torch.float32).cuda()).cpu().numpy()
    assert np.mean((Y - T[2048:2112]) ** 2) < 0.25 * np.mean(T[2048:2112] ** 2)


def test_pod_matches_oracle():
    import torch
    from paper_2306_00165_amd import pcfv
    rng = np.random.default_rng(11)
    S, n, k = 48, 5000, 6
    V, _ = np.linalg.qr(rng.standard_normal((n, k)))
    A = rng.standard_normal((S, k))
    A -= A.mean(axis=0)
    A, _ = np.linalg.qr(A)
    X = rng.standard_normal(n) + (A * np.array([10, 5, 2, 1, .5, .25])) @ V.T + 1e-3 * rng.standard_normal((S, n))
    mean, basis, sig = pcfv.pod_build(torch.as_tensor(X).cuda(), k)
    om, ob, osig = opod.pod(X, k)
    np.testing.assert_allclose(sig, osig, rtol=1e-12)
    np.testing.assert_allclose(mean.cpu().numpy(), om, rtol=0, atol=1e-13)
    bas = basis.cpu().numpy()
    for i in range(k):
        assert abs(abs(bas[i] @ ob[i]) - 1) < 1e-12
    c = pcfv.pod_project(torch.as_tensor(X).cuda(), mean, basis)
    np.testing.assert_allclose(c.cpu().numpy(), opod.project(X, om, bas), rtol=0, atol=1e-12 * np.abs(X).max())
    Xr = pcfv.pod_reconstruct(c, mean, basis).cpu().numpy()
    np.testing.assert_allclose(Xr, opod.reconstruct(c.cpu().numpy(), om, bas), rtol=0, atol=1e-12)


@pytest.fixture(scope="module")
def trained():
    """A small extrapolator for 16 x 25 x 16, batch 16, trained on seeded
    trajectories of the method itself (DMD-accelerated targets) as a
    correction to the DMD candidate of windows of 16 snapshots 20 steps apart,
    its input the last 8 snapshots."""
    from paper_2306_00165_amd import learned, pcfv
    ctx = pcfv.Context(16, 25, 16, batch=16)
    gen = learned.kolmogorov((16, 25, 16), 0.01)
    dmd = dict(dmd_window=16, dmd_stride=20, dmd_gap=200, dmd_accept=10.0)
    kw = dict(dtau=0.05, warm=200, window=16, stride=20, n_windows=4, gap=100)
    wins, tg = learned.training_set(ctx, list(range(100, 164)), 0.01, gen, horizon=4000, dmd=dmd, **kw)
    L, hist = learned.fit(ctx, wins, tg, r=16, hidden=(256, 256), epochs=20, batch=64, pod_rows=256,
                          base_dmd_dtau=20 * 0.05)
    return ctx, L, gen, dmd, kw, hist


def _window(ctx, gen, seeds, kw):
    from paper_2306_00165_amd import learned
    hw, _ = learned.training_set(ctx, seeds, 0.01, gen, horizon=0, **dict(kw, n_windows=1))
    return hw.contiguous()


def test_learned_proposal_is_assembled_as_defined_and_costed_exactly(trained):
    """With one step length the proposal is the DMD candidate plus the
    predicted POD step (rebuilt here from the model's parts); it is
    admissible and the library's cost is the oracle's cost of that state.
    With several step lengths each guess gets the cheapest of the single-length
    proposals."""
    import torch
    from paper_2306_00165_amd import pcfv
    ctx, L, gen, dmd, kw, hist = trained
    assert hist[-1] < hist[0]
    snaps = _window(ctx, gen, list(range(500, 516)), kw)
    u_d, _, _ = ctx.dmd_extrapolate(snaps, 20 * 0.05)
    base = ctx.pack(u_d)
    one = pcfv.Learned(ctx, 8, L.mean, L.basis, L.stats, L.mlp, use_base=True, scales=(1.0,))
    u, cost = one.propose(snaps[-8:].contiguous(), base)
    r = L.basis.shape[0]
    c = pcfv.pod_project(snaps[-8:].reshape(-1, snaps.shape[2]), L.mean, L.basis).reshape(8, 16, r)
    cb = pcfv.pod_project(base, L.mean, L.basis)
    X, _, _ = pcfv.learned_prepare(c, None, stats=L.stats, cb=cb)
    y = L.mlp.forward(X).cpu().numpy().astype(np.float64)
    omu, oisd = L.stats[2].cpu().numpy(), L.stats[3].cpu().numpy()
    psi = base.cpu().numpy() + (y / oisd + omu) @ L.basis.cpu().numpy()
    ref = ctx.unpack(torch.as_tensor(psi).cuda()).cpu().numpy()
    got = u.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    g = Grid(16, 25, 16)
    m = Method(g)
    for b in range(16):
        assert abs(cost[b] - m.cost(got[b])) <= 1e-11 * cost[b]
        assert max(m.defects(got[b])) < 1e-12
    singles = [pcfv.Learned(ctx, 8, L.mean, L.basis, L.stats, L.mlp, use_base=True, scales=(a,))
               .propose(snaps[-8:].contiguous(), base)[1] for a in (0.25, 1.0)]
    both = pcfv.Learned(ctx, 8, L.mean, L.basis, L.stats, L.mlp, use_base=True, scales=(0.25, 1.0))
    _, cb2 = both.propose(snaps[-8:].contiguous(), base)
    np.testing.assert_allclose(cb2, np.minimum(*singles), rtol=1e-14)


def test_learned_alongside_dmd_gains_on_held_out_seeds(trained):
    """At the end of a DMD window the descent takes, per guess, the cheaper of
    the DMD and learned candidates by true cost (under the acceptance rule),
    and the number of learned candidates taken is the one the entry points
    give on the same window.  On 16 held-out seeds (never seen in training)
    the trained network must earn its place: its candidate is taken for at
    least half of the guesses, the chosen candidate is no costlier than DMD's
    at the median, and on average it lowers the cost by more than 1%
    (mean DMD / chosen > 1.01; measured: median 1.014, mean 1.018 against the
    DMD candidates of the paper's mode and the affine limit)."""
    import torch
    ctx, L, gen, dmd, kw, _ = trained
    U0 = torch.as_tensor(np.stack([gen(s) for s in range(600, 616)])).cuda().contiguous()
    ctx.descend(U0, max_steps=200, dtau=0.05)
    V = U0.clone()
    snaps = []
    for k in range(16):
        snaps.append(ctx.pack(V))
        if k < 15:
            ctx.descend(V, max_steps=20, dtau=0.05)
    snaps = torch.stack(snaps).contiguous()
    cur = np.array(ctx.cost(V))
    u_d, c_d, r_d = ctx.dmd_extrapolate(snaps, 20 * 0.05)
    _, c_l = L.propose(snaps[-8:].contiguous(), ctx.pack(u_d))
    c_d, c_l, r_d = np.array(c_d), np.array(c_l), np.array(r_d)
    d_ok = r_d > 0
    take_l = np.isfinite(c_l) & (~d_ok | (c_l < c_d)) & (c_l < 10.0 * cur)
    U = U0.clone()
    st, rep = ctx.descend(U, max_steps=301, dtau=0.05, check_every=301, learned=L,
                          dmd_window=16, dmd_stride=20, dmd_gap=10000, dmd_accept=10.0)
    assert rep["n_dmd"] == 1 and rep["n_learned_accepted"] == int(take_l.sum())
    best = np.where(take_l, c_l, c_d)
    gain = c_d / best
    print(f"[gpu] learned candidates taken {int(take_l.sum())}/16; median cost: current {np.median(cur):.3e}, "
          f"DMD {np.median(c_d):.3e}, learned {np.median(c_l):.3e}; gain (DMD / chosen) median "
          f"{np.median(gain):.3f}, mean {np.mean(gain):.3f}")
    assert take_l.sum() >= 8
    assert np.median(gain) >= 1.0 and np.mean(gain) > 1.01

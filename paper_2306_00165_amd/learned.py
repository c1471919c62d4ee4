"""Training and use of the learned extrapolator that sits beside the DMD
extrapolation of Sec. 6.

Everything numerical runs in libpcfv (descent, state vectors, FP64 POD,
BF16-matrix-core MLP training); this module only sequences the calls:

1. trajectories: seeded guesses descend; after `warm` steps, windows of W
   snapshots (state vectors, `stride` steps apart) are recorded every
   `gap` steps; after the last window the descent continues for `horizon`
   steps (optionally DMD-accelerated) and the state reached is each window's
   target, the approximation of the descent limit;
2. POD of a subsample of the recorded states (r modes);
3. features and targets from the POD coefficients, normalised per column;
4. minibatch Adam on the MLP.

The trained model then proposes, from the last W snapshots of a DMD window,
a state whose true cost competes with the DMD candidate (`pcfv_descend`).
"""

import numpy as np
import torch

from . import inputs, pcfv


def he_params(dims, seed):
    """He-normal weights and zero biases, flat in the library's order."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, n in zip(dims[:-1], dims[1:]):
        parts.append(rng.standard_normal(k * n) * np.sqrt(2.0 / k))
        parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


def _pack(ctx, U):
    psi = ctx.pack(U)
    return psi if psi.dim() == 2 else psi.unsqueeze(0)


def trajectories(ctx, U, dtau, warm, window, stride, n_windows, gap, horizon, dmd=None):
    """Advance the batch U (ctx's shape) and record windows.  Returns
    (windows [n_windows][W][B][n], limits [B][n]) as float64 device tensors."""
    ctx.descend(U, max_steps=warm, dtau=dtau)
    wins = []
    for _ in range(n_windows):
        snaps = []
        for k in range(window):
            snaps.append(_pack(ctx, U))
            if k < window - 1:
                ctx.descend(U, max_steps=stride, dtau=dtau)
        wins.append(torch.stack(snaps))
        ctx.descend(U, max_steps=gap, dtau=dtau)
    ctx.descend(U, max_steps=horizon, dtau=dtau, **(dmd or {}))
    return torch.stack(wins), _pack(ctx, U)


def training_set(ctx, seeds, energy, envelope_guess, dtau, warm, window, stride, n_windows, gap, horizon, dmd=None,
                 progress=None):
    """Windows [W][Nw][n] and targets [Nw][n] from guesses seeds (batched by
    ctx.batch); envelope_guess(seed) returns one initial field.  progress, if
    given, is called with a message after every batch of trajectories."""
    B = ctx.batch
    allw, allt = [], []
    for i in range(0, len(seeds), B):
        chunk = list(seeds[i:i + B])
        while len(chunk) < B:           # pad the last batch by repeating its first seed
            chunk.append(chunk[0])
        fields = [envelope_guess(s) for s in chunk]
        U = torch.as_tensor(np.stack(fields) if B > 1 else fields[0]).to(ctx.device).contiguous()
        wins, lim = trajectories(ctx, U, dtau, warm, window, stride, n_windows, gap, horizon, dmd)
        nreal = min(B, len(seeds) - i)
        for k in range(n_windows):
            allw.append(wins[k][:, :nreal])
            allt.append(lim[:nreal])
        if progress:
            progress(f"trajectories {i + nreal}/{len(seeds)}")
    return torch.cat(allw, dim=1).contiguous(), torch.cat(allt, dim=0).contiguous()


def dmd_bases(ctx, windows, dtau_snap):
    """DMD candidates of every window ([M][Nw][n], ctx.batch windows at a
    time; a short last chunk is padded) as state vectors [Nw][n]."""
    M, Nw, n = windows.shape
    B = ctx.batch
    out = []
    for i in range(0, Nw, B):
        chunk = windows[:, i:i + B]
        k = chunk.shape[1]
        if k < B:
            chunk = torch.cat([chunk, chunk[:, :1].expand(M, B - k, n)], dim=1)
        u, _, _ = ctx.dmd_extrapolate(chunk.contiguous(), dtau_snap)
        out.append(_pack(ctx, u)[:k])
    return torch.cat(out, dim=0).contiguous()


def fit(ctx, windows, targets, r, hidden=(512, 512, 512), epochs=40, batch=128, lr=1e-3, seed=0,
        pod_rows=512, max_batch=None, feat_window=8, base_dmd_dtau=None, scales=(0.1, 0.25, 0.5, 1.0)):
    """Train an extrapolator for ctx from windows [M][Nw][n] and targets
    [Nw][n]; its input is the last feat_window snapshots of each window.
    base_dmd_dtau (the snapshot spacing in tau) makes it a correction to the
    DMD candidate of the whole window.  scales: step lengths along the
    predicted step that each proposal tries (the least true cost wins).
    Returns (pcfv.Learned, loss history)."""
    M, Nw, n = windows.shape
    W = min(feat_window, M)
    feats = windows[M - W:]
    rng = np.random.default_rng(seed)
    pool = torch.cat([feats[-1], targets], dim=0)
    rows = rng.choice(pool.shape[0], size=min(pod_rows, pool.shape[0]), replace=False)
    mean, basis, _ = pcfv.pod_build(pool[torch.as_tensor(np.sort(rows), device=pool.device)].contiguous(), r)
    c = pcfv.pod_project(feats.reshape(W * Nw, n), mean, basis).reshape(W, Nw, r)
    ct = pcfv.pod_project(targets, mean, basis)
    cb = None
    if base_dmd_dtau is not None:
        cb = pcfv.pod_project(dmd_bases(ctx, windows, base_dmd_dtau), mean, basis)
    X, T, stats = pcfv.learned_prepare(c, ct, cb=cb)
    dims = [X.shape[1], *hidden, r]
    mlp = pcfv.MLP(dims, max_batch=max(batch, max_batch or ctx.batch))
    mlp.set_params(he_params(dims, seed))
    hist = mlp.fit(X, T, batch=min(batch, Nw), epochs=epochs, lr=lr, seed=seed)
    return pcfv.Learned(ctx, W, mean, basis, stats, mlp, use_base=cb is not None, scales=scales), hist


def kolmogorov(dims, energy):
    Nx, Ny, Nz = dims
    return lambda seed: inputs.kolmogorov_guess(Nx, Ny, Nz, energy, seed)


def evaluate(ctx, L, windows, dtau_snap, feat_window=8):
    """True costs on held-out windows [M][Nh][n] (ctx.batch at a time): the
    last snapshot, the DMD candidate and the learned proposal."""
    M, Nh, n = windows.shape
    B = ctx.batch
    cur, dmd, lrn = [], [], []
    for i in range(0, Nh - B + 1, B):
        snaps = windows[:, i:i + B].contiguous()
        u_d, c_d, _ = ctx.dmd_extrapolate(snaps, dtau_snap)
        _, c_l = L.propose(snaps[M - feat_window:].contiguous(), _pack(ctx, u_d) if L.model.use_base else None)
        cur += list(np.atleast_1d(ctx.cost(ctx.unpack(snaps[-1].contiguous()))))
        dmd += list(np.atleast_1d(c_d))
        lrn += list(np.atleast_1d(c_l))
    return np.array(cur), np.array(dmd), np.array(lrn)


def main(argv=None):
    """End-to-end run at the extrapolator's full size: seeded trajectories on
    one grid, POD, training, and the held-out comparison with DMD.  Prints one
    JSON line."""
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, nargs=3, default=[48, 49, 48])
    ap.add_argument("--dtau", type=float, default=0.012)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--train-seeds", type=int, default=128)
    ap.add_argument("--test-seeds", type=int, default=32)
    ap.add_argument("--windows", type=int, default=8, help="windows per trajectory")
    ap.add_argument("--snapshots", type=int, default=16, help="snapshots per DMD window")
    ap.add_argument("--stride", type=int, default=40)
    ap.add_argument("--horizon", type=int, default=10000)
    ap.add_argument("--r", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--energy", type=float, default=0.03)
    args = ap.parse_args(argv)
    t0 = time.perf_counter()
    import sys

    def progress(msg):
        print(f"[{time.perf_counter() - t0:.0f}s] {msg}", file=sys.stderr, flush=True)
    dims = tuple(args.grid)
    ctx = pcfv.Context(*dims, batch=args.batch)
    gen = kolmogorov(dims, args.energy)
    dmd = dict(dmd_window=args.snapshots, dmd_stride=args.stride, dmd_gap=4 * args.stride, dmd_accept=10.0)
    kw = dict(dtau=args.dtau, warm=200, window=args.snapshots, stride=args.stride, n_windows=args.windows,
              gap=2 * args.stride)
    wins, tg = training_set(ctx, list(range(1000, 1000 + args.train_seeds)), args.energy, gen,
                            horizon=args.horizon, dmd=dmd, progress=progress, **kw)
    t_data = time.perf_counter() - t0
    hw, _ = training_set(ctx, list(range(5000, 5000 + args.test_seeds)), args.energy, gen, horizon=0,
                         progress=progress, **dict(kw, n_windows=2))
    t1 = time.perf_counter()
    L, hist = fit(ctx, wins, tg, r=args.r, hidden=(512, 512, 512), epochs=args.epochs, batch=128,
                  pod_rows=512, base_dmd_dtau=args.stride * args.dtau)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t1
    progress("trained")
    cur, d, l = evaluate(ctx, L, hw, args.stride * args.dtau)
    best = np.minimum(d, l)
    out = {
        "grid": list(dims), "batch": args.batch, "train_windows": int(wins.shape[1]),
        "held_out_windows": int(len(d)), "pod_modes": args.r, "mlp_dims": L.mlp.dims,
        "mlp_params": int(L.mlp.n_params), "data_seconds": round(t_data, 1), "fit_seconds": round(t_fit, 2),
        "loss_first_last": [float(hist[0]), float(hist[-1])],
        "learned_beats_dmd": int(np.sum(l < d)),
        "median_cost_ratio_learned_over_dmd": float(np.median(l / d)),
        "median_cost_ratio_chosen_over_dmd": float(np.median(best / d)),
        "mean_cost_ratio_chosen_over_dmd": float(np.mean(best / d)),
        "median_cost_ratio_dmd_over_current": float(np.median(d / cur)),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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


def training_set(ctx, seeds, energy, envelope_guess, dtau, warm, window, stride, n_windows, gap, horizon, dmd=None):
    """Windows [W][Nw][n] and targets [Nw][n] from guesses seeds (batched by
    ctx.batch); envelope_guess(seed) returns one initial field."""
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

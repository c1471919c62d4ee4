"""Dynamic mode decomposition and extrapolation (oracle; test infrastructure).

Sec. 6.1: snapshots psi_k = psi(tau_k), k = 1..M, spaced delta tau along one
trajectory; the pairs (psi_k, psi_{k+1}) define A = Psi' Psi^+ with
Psi = [psi_1 .. psi_{M-1}] and Psi' = [psi_2 .. psi_M] (M snapshots give M-1
pairs).  With the rank-r SVD Psi ~ U Sigma V^T, A~ = U^T Psi' V Sigma^{-1};
its eigenpairs (lam_q, w_q) give the dynamic modes phi_q = Psi' V Sigma^{-1} w_q,
growth rates omega_q = ln(lam_q)/delta tau, and the linear model
psi(tau) ~ sum_q b_q phi_q exp(omega_q tau) with amplitudes b_q fitted at the
last snapshot (least squares).

Sec. 6.2: the mode with the smallest |omega| is taken as the steady state,
psi_s = b_1 phi_1 (real part; the data are real), and the truncation rank
r <= r* (r* = numerical rank of Psi) is the one whose extrapolated state has
the smallest cost J (the paper found it at r = r*; the ranks tried here are
r*, r* - 1, r* - 2, r* - 4, ..., see rank_tried).

Reading for targets the paper's rule cannot reach.  The smallest-|omega|
mode is the limit of the linear model only when one mode neither grows nor
decays (omega ~ 0, a non-trivial fixed point).  When the trajectory heads for
the laminar state every fitted mode decays and no such mode exists; when the
window is short, the fitted rate of the fixed-point mode is not close to 0.
Both cases are covered by the limit of an affine model psi_{k+1} - psi* =
A (psi_k - psi*): its differences d_k = psi_{k+1} - psi_k obey d_{k+1} = A d_k
(linear, no fixed point needed), so the exact DMD of the difference pairs
(d_k, d_{k+1}) with amplitudes fitted at the last difference gives the future
differences b_q phi_q lambda_q^j, and their sum is the limit
    psi_inf = psi_M + Re sum_{|lambda_q| < 1} b_q phi_q lambda_q / (1 - lambda_q).
It is exact for affine dynamics around any fixed point, the laminar state
(psi* = 0) included.  So beside the paper's candidate (kind 0, ranks
r <= r*) each rank r <= r*_d (numerical rank of [d_1 .. d_{M-2}]) offers this
limit (kind 1).  Every candidate is judged by its true cost, and the cheapest
one (earliest in the order rank, then kind, on ties) is the extrapolation.

Snapshots are minimal real state vectors (oracle.state.pack).  The numerical
rank counts singular values above RANK_TOL times the largest.
"""

import numpy as np

from . import state

RANK_TOL = 1e-7


def numerical_rank(snaps, tol=RANK_TOL):
    X = np.asarray(snaps)[:-1].T
    s = np.linalg.svd(X, compute_uv=False)
    return int(np.sum(s > tol * s[0])) if s.size and s[0] > 0 else 0


def dmd(snaps, dtau, r):
    """Exact DMD of rank r.  snaps: (M, n) real.  Returns (lam, omega, Phi, b)."""
    S = np.asarray(snaps, dtype=float)
    X, Y = S[:-1].T, S[1:].T
    U, s, Vh = np.linalg.svd(X, full_matrices=False)
    U, s, V = U[:, :r], s[:r], Vh[:r].T
    At = (U.T @ Y @ V) / s[None, :]
    lam, W = np.linalg.eig(At)
    Phi = ((Y @ V) / s[None, :]) @ W
    omega = np.log(lam.astype(complex)) / dtau
    b = np.linalg.lstsq(Phi, S[-1].astype(complex), rcond=None)[0]
    return lam, omega, Phi, b


def steady_state(snaps, dtau, r):
    """psi_s = Re(b_1 phi_1) for the mode with the smallest |omega|."""
    lam, omega, Phi, b = dmd(snaps, dtau, r)
    q = int(np.argmin(np.abs(omega)))
    return np.real(b[q] * Phi[:, q]), omega[q]


def affine_limit(snaps, dtau, r):
    """psi_M + Re sum_{|lambda_q| < 1} b_q phi_q lambda_q/(1 - lambda_q) from the
    rank-r exact DMD of the snapshot differences."""
    S = np.asarray(snaps, dtype=float)
    lam, omega, Phi, b = dmd(np.diff(S, axis=0), dtau, r)
    gain = np.where(np.abs(lam) < 1, lam / (1 - lam), 0.0)
    return S[-1] + np.real(Phi @ (b * gain))


def rank_tried(r, rstar):
    """Ranks fitted for numerical rank r*: r*, r* - 1, r* - 2, r* - 4, r* - 8,
    ... (>= 1).  Sec. 6.2 takes the least-cost rank r <= r* and found it at
    r*; every rank would cost O(M^5) work and M cost evaluations per window."""
    d = rstar - r
    return 1 <= r <= rstar and (d <= 2 or (d & (d - 1)) == 0)


def candidates(snaps, dtau, rstar):
    """[(rank, kind, psi)]: kind 0 the paper's smallest-|omega| mode for the
    ranks tried below r*, kind 1 the affine limit for those below r*_d,
    ordered by rank, then kind."""
    S = np.asarray(snaps, dtype=float)
    rstar_d = numerical_rank(np.diff(S, axis=0)) if rstar > 0 else 0
    out = []
    for r in range(1, max(rstar, rstar_d) + 1):
        if rank_tried(r, rstar):
            out.append((r, 0, steady_state(S, dtau, r)[0]))
        if rank_tried(r, rstar_d):
            out.append((r, 1, affine_limit(S, dtau, r)))
    return out


def extrapolate(method, fields, dtau):
    """DMD extrapolation of a window of snapshot fields (same grid): returns
    (u_s, cost_s, r, kind) for the candidate of smallest true cost (Sec. 6.2
    and the reading above), or (None, inf, 0, -1) if the window has rank 0."""
    g = method.g
    psis = np.stack([state.pack(g, u) for u in fields])
    rstar = numerical_rank(psis)
    best = (None, np.inf, 0, -1)
    for r, kind, psi in candidates(psis, dtau, rstar):
        u_s = state.unpack(g, psi)
        c = method.cost(u_s)
        if c < best[1]:
            best = (u_s, c, r, kind)
    return best

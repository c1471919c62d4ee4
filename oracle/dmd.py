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
the smallest cost J.

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


def extrapolate(method, fields, dtau):
    """DMD extrapolation of a window of snapshot fields (same grid): returns
    (u_s, cost_s, r) for the rank r <= r* whose steady state has the smallest
    cost (Sec. 6.2), or (None, inf, 0) if the window has rank 0."""
    g = method.g
    psis = np.stack([state.pack(g, u) for u in fields])
    rstar = numerical_rank(psis)
    best = (None, np.inf, 0)
    for r in range(1, rstar + 1):
        psi_s, _ = steady_state(psis, dtau, r)
        u_s = state.unpack(g, psi_s)
        c = method.cost(u_s)
        if c < best[1]:
            best = (u_s, c, r)
    return best

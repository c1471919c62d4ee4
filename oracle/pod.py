"""Proper orthogonal decomposition of snapshot sets (oracle; test
infrastructure).  The leading right singular vectors of the centred snapshot
matrix (library SVD) are the modes; projection and reconstruction are the
plain products.  Used by the learned extrapolator that sits beside the DMD
extrapolation of Sec. 6 (whose rank-r SVD of the snapshot matrix is the same
decomposition without centring)."""

import numpy as np


def pod(X, r):
    """X: (S, n) snapshots.  Returns (mean (n), basis (r, n), sigma (r))."""
    X = np.asarray(X, dtype=np.float64)
    mean = X.mean(axis=0)
    _, s, Vt = np.linalg.svd(X - mean, full_matrices=False)
    return mean, Vt[:r], s[:r]


def project(X, mean, basis):
    return (np.asarray(X, dtype=np.float64) - mean) @ basis.T


def reconstruct(coef, mean, basis):
    return mean + np.asarray(coef) @ basis

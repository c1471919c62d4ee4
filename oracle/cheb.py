"""Chebyshev operators in the wall-normal direction (oracle; test infrastructure).

The velocity is expanded as sum_n u_n T_n(y), T_n the Chebyshev polynomials of
the first kind, on y in [-1, 1] (Sec. 4, Fourier-Chebyshev-Fourier expansion).
Products are formed at the Gauss-Lobatto points y_j = cos(pi j/(N-1)).

All matrices act on coefficient vectors of length N (index n = 0..N-1) by
left multiplication: (A u)_n = sum_p A[n, p] u_p.
"""

import numpy as np


def gl_points(N):
    """Gauss-Lobatto collocation points y_j = cos(pi j / (N-1)), j = 0..N-1."""
    return np.cos(np.pi * np.arange(N) / (N - 1))


def synthesis(N):
    """C[j, n] = T_n(y_j) = cos(pi n j/(N-1)): coefficients -> point values."""
    j = np.arange(N)[:, None]
    n = np.arange(N)[None, :]
    return np.cos(np.pi * n * j / (N - 1))


def derivative(N):
    """Exact derivative on coefficients: (Du)_n = (2/c_n) sum_{p>n, p+n odd} p u_p,
    with c_0 = 2 and c_n = 1 otherwise (textbook Chebyshev identity)."""
    D = np.zeros((N, N))
    for n in range(N):
        cn = 2.0 if n == 0 else 1.0
        for p in range(n + 1, N):
            if (p + n) % 2 == 1:
                D[n, p] = 2.0 * p / cn
    return D


def gram(N):
    """G[m, n] = int_{-1}^{1} T_m T_n dy = 1/(1-(m+n)^2) + 1/(1-(m-n)^2) for m+n
    even, 0 otherwise (from T_m T_n = (T_{m+n} + T_{|m-n|})/2)."""
    G = np.zeros((N, N))
    for m in range(N):
        for n in range(N):
            if (m + n) % 2 == 0:
                G[m, n] = 1.0 / (1.0 - (m + n) ** 2) + 1.0 / (1.0 - (m - n) ** 2)
    return G


def wall_rows(N):
    """Row vectors evaluating a series at the walls: u(+1) = sum u_n and
    u(-1) = sum (-1)^n u_n."""
    plus = np.ones(N)
    minus = (-1.0) ** np.arange(N)
    return plus, minus

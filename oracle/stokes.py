"""Implicit Stokes step as the dense Chebyshev-tau system (oracle; test infrastructure).

Steps (1) and (3) of the five-step algorithm (Sec. 4) advance a system of the
form du/dt = M(u) - grad p + (1/Re) Lap u, div u = 0, u(+-1) = 0, by one time
step with an influence-matrix solver that keeps div u = 0 and no-slip exact.
Reading: one first-order IMEX step (implicit Stokes part, explicit M), whose
implicit solve is the linear map S_lam: F -> u defined, for every stored
Fourier mode with kappa^2 = a^2 + b^2 > 0, by the 4N x 4N Chebyshev-tau system

  (T1-T3)  [(lam + nu kappa^2) u_c - nu D^2 u_c + grad_c p]_n = F_{c,n},
           n = 0..N-3, c = x, y, z, grad = (i a, D, i b)
  (T4)     u_c(+1) = u_c(-1) = 0
  (T5)     [i a u_x + D u_y + i b u_z]_n = 0 for all n = 0..N-1

in the unknowns (u_x, u_y, u_z, p).  For the (0, 0) mode, u_x and u_z solve
[(lam - nu D^2) u]_n = F_n (n <= N-3) with u(+-1) = 0 and u_y = 0 (no mean
pressure gradient; the y-momentum is balanced by the pressure).

The oracle factors each mode's matrix once (LU) and solves directly; it never
uses the influence-matrix algorithm.  S^H reuses the factors with the
conjugate-transposed solve; the W-adjoint is G^{-1} S^H G per component.
"""

import numpy as np
import scipy.linalg as sla

from . import cheb


class Stokes:
    def __init__(self, g, lam):
        self.g = g
        self.lam = float(lam)
        N = g.N
        self.N = N
        D = cheb.derivative(N)
        self.G = cheb.gram(N)
        self.Ginv = np.linalg.inv(self.G)
        D2 = D @ D
        bp, bm = cheb.wall_rows(N)
        I = np.eye(N)
        nu = g.nu
        self.factors = {}
        for (ikx, kz) in g.modes():
            a, b = g.a[ikx], g.b[kz]
            k2 = a * a + b * b
            if ikx == 0 and kz == 0:
                T = np.zeros((N, N))
                T[:N - 2] = (self.lam * I - nu * D2)[:N - 2]
                T[N - 2] = bp
                T[N - 1] = bm
                self.factors[(ikx, kz)] = sla.lu_factor(T)
                continue
            H = (self.lam + nu * k2) * I - nu * D2
            grad = [1j * a * I, D.astype(complex), 1j * b * I]
            T = np.zeros((4 * N, 4 * N), dtype=complex)
            for c in range(3):
                r0 = c * N
                T[r0:r0 + N - 2, c * N:(c + 1) * N] = H[:N - 2]
                T[r0:r0 + N - 2, 3 * N:4 * N] = grad[c][:N - 2]
                T[r0 + N - 2, c * N:(c + 1) * N] = bp
                T[r0 + N - 1, c * N:(c + 1) * N] = bm
            T[3 * N:4 * N, 0:N] = 1j * a * I
            T[3 * N:4 * N, N:2 * N] = D
            T[3 * N:4 * N, 2 * N:3 * N] = 1j * b * I
            self.factors[(ikx, kz)] = sla.lu_factor(T)

    def _rhs(self, F, ikx, kz):
        N = self.N
        rhs = np.zeros(4 * N, dtype=complex)
        for c in range(3):
            rhs[c * N:c * N + N - 2] = F[c, ikx, kz, :N - 2]
        return rhs

    def solve(self, F):
        """u = S_lam(F) for a spectral array F of shape (3, nkx, nkz, N)."""
        g, N = self.g, self.N
        out = np.zeros(g.shape, dtype=complex)
        for (ikx, kz), lu in self.factors.items():
            if ikx == 0 and kz == 0:
                for c in (0, 2):
                    rhs = np.zeros(N, dtype=complex)
                    rhs[:N - 2] = F[c, 0, 0, :N - 2]
                    out[c, 0, 0] = sla.lu_solve(lu, rhs)
                continue
            x = sla.lu_solve(lu, self._rhs(F, ikx, kz))
            for c in range(3):
                out[c, ikx, kz] = x[c * N:(c + 1) * N]
        return out

    def solve_h(self, X):
        """Conjugate transpose S^H (Euclidean, per mode) applied to X."""
        g, N = self.g, self.N
        out = np.zeros(g.shape, dtype=complex)
        for (ikx, kz), lu in self.factors.items():
            if ikx == 0 and kz == 0:
                for c in (0, 2):
                    y = sla.lu_solve(lu, X[c, 0, 0].astype(complex), trans=2)
                    out[c, 0, 0, :N - 2] = y[:N - 2]
                continue
            b = np.zeros(4 * N, dtype=complex)
            for c in range(3):
                b[c * N:(c + 1) * N] = X[c, ikx, kz]
            y = sla.lu_solve(lu, b, trans=2)
            for c in range(3):
                out[c, ikx, kz, :N - 2] = y[c * N:c * N + N - 2]
        return out

    def solve_wadj(self, X):
        """W-adjoint S* = G^{-1} S^H G (per component and mode)."""
        return self.solve_h(X @ self.G.T) @ self.Ginv.T

    def pressure(self, F, ikx, kz):
        """Pressure coefficients of the tau solution for one kappa > 0 mode
        (used by tests only)."""
        N = self.N
        x = sla.lu_solve(self.factors[(ikx, kz)], self._rhs(F, ikx, kz))
        return x[3 * N:]

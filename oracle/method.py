"""The adjoint-descent method on the discrete PCF problem (oracle; test infrastructure).

Definitions followed (paper sections in brackets):
  residual      r(u) = lam S_lam(M_h(u) + nu L u), lam = 1/Delta t, L = D^2 - kappa^2.
                Steps (1)-(2) of the five-step algorithm (Sec. 4) form
                r = (u^{Delta t} - u)/Delta t with u^{Delta t} = S_lam(lam u + M_h(u));
                because S_lam((lam - nu L) u) = u for every admissible u, both
                forms are the same linear algebra (residual_fd keeps the literal one).
  cost          J^2 = <r, r>_W (Sec. 2; Sec. 3.2 cost with r2 = div u = 0 on
                admissible fields).  <.,.>_W is the volume-averaged L2 product.
  jvp           the directional derivative L(u; v) of r (Sec. 2, App. A.1).
  adjoint       its exact W-adjoint J*(u) = W^{-1} J(u)^H W on the discrete space
                (Sec. 2 definition of the adjoint; continuous form in Sec. 3.3
                and App. A.2 is its continuum limit with r2 = 0).
  project       the W-orthogonal projection onto divergence-free, no-slip
                fields (Sec. 3.4: the Helmholtz projection is L2-orthogonal).
  descent_step  u <- u + Delta tau f with f = -P_W J*(u) r(u)  (Sec. 4 step (5)).
"""

import numpy as np
import scipy.linalg as sla

from . import cheb
from .flow import Transforms, nonlinear, nonlinear_lin, nonlinear_lin_adj
from .stokes import Stokes


class Method:
    def __init__(self, g):
        self.g = g
        self.T = Transforms(g)
        self.S = Stokes(g, g.lam)
        N = g.N
        self.D = self.T.D
        self.D2 = self.D @ self.D
        self.G = self.T.G
        self.Ginv = self.T.Ginv
        self._proj = None

    # -- inner products and norms --------------------------------------------
    def inner(self, a, b):
        """<a, b>_W = sum_modes w(kz) Re sum_c a^H G b: equals (1/V) int a.b dx,
        V = 2 Lx Lz, for Hermitian-consistent fields."""
        g = self.g
        Gb = b @ self.G.T
        tot = 0.0
        for kz in range(g.nkz):
            tot += g.weight(kz) * np.real(np.sum(np.conj(a[:, :, kz, :]) * Gb[:, :, kz, :]))
        return float(tot)

    def norm(self, u):
        return np.sqrt(max(self.inner(u, u), 0.0))

    def base_flow(self):
        ub = self.g.zeros()
        ub[0, 0, 0, 1] = 1.0          # u_b = y e_x = T_1(y) e_x
        return ub

    def total_norm(self, u):
        """||u_b + u||_W."""
        return self.norm(self.base_flow() + u)

    # -- linear operators ------------------------------------------------------
    def lap(self, u):
        """L u = D^2 u - kappa^2 u per mode."""
        g = self.g
        k2 = g.a[:, None] ** 2 + g.b[None, :] ** 2
        return u @ self.D2.T - k2[None, :, :, None] * u

    def lap_adj(self, w):
        g = self.g
        k2 = g.a[:, None] ** 2 + g.b[None, :] ** 2
        return w @ (self.Ginv @ self.D2.T @ self.G).T - k2[None, :, :, None] * w

    # -- the method -----------------------------------------------------------
    def nonlinear(self, u):
        return nonlinear(self.T, u)

    def residual(self, u):
        g = self.g
        return g.lam * self.S.solve(self.nonlinear(u) + g.nu * self.lap(u))

    def residual_fd(self, u):
        """Paper-literal steps (1)-(2): u^{dt} = S(lam u + M(u)); r = (u^{dt}-u)/dt."""
        g = self.g
        udt = self.S.solve(g.lam * u + self.nonlinear(u))
        return (udt - u) / g.dt

    def jvp(self, u, v):
        g = self.g
        return g.lam * self.S.solve(nonlinear_lin(self.T, u, v) + g.nu * self.lap(v))

    def adjoint(self, u, w):
        """J*(u) w with J(u) v = lam S(M'(u) v + nu L v):
        J* = lam (M'(u)* + nu L*) S*  (reverse order, each factor W-adjointed)."""
        g = self.g
        a = self.S.solve_wadj(w)
        return g.lam * (nonlinear_lin_adj(self.T, u, a) + g.nu * self.lap_adj(a))

    def cost(self, u):
        r = self.residual(u)
        return self.inner(r, r)

    # -- projection onto V_h ---------------------------------------------------
    def _build_projection(self):
        g, N = self.g, self.g.N
        D = self.D
        bp, bm = cheb.wall_rows(N)
        G = self.G
        I = np.eye(N)
        proj = {}
        for (ikx, kz) in g.modes():
            a, b = g.a[ikx], g.b[kz]
            if ikx == 0 and kz == 0:
                Q = sla.null_space(np.vstack([bp, bm]))
                Minv = np.linalg.inv(Q.T @ G @ Q)
                proj[(0, 0)] = (Q, Minv)
                continue
            B = np.zeros((N + 6, 3 * N), dtype=complex)
            B[:N, 0:N] = 1j * a * I
            B[:N, N:2 * N] = D
            B[:N, 2 * N:3 * N] = 1j * b * I
            for c in range(3):
                B[N + 2 * c, c * N:(c + 1) * N] = bp
                B[N + 2 * c + 1, c * N:(c + 1) * N] = bm
            Q = sla.null_space(B)
            W = np.kron(np.eye(3), G)
            Minv = np.linalg.inv(Q.conj().T @ W @ Q)
            proj[(ikx, kz)] = (Q, Minv)
        self._proj = proj

    def project(self, gvec):
        """P_W g = Q (Q^H W Q)^{-1} Q^H W g per mode, Q a basis of the mode's
        divergence-free, no-slip subspace (dense null space)."""
        if self._proj is None:
            self._build_projection()
        g, N = self.g, self.g.N
        out = np.zeros(g.shape, dtype=complex)
        G = self.G
        for (ikx, kz), (Q, Minv) in self._proj.items():
            if ikx == 0 and kz == 0:
                for c in (0, 2):
                    x = gvec[c, 0, 0]
                    out[c, 0, 0] = Q @ (Minv @ (Q.T @ (G @ x)))
                continue
            x = gvec[:, ikx, kz, :].reshape(3 * N)
            Wx = np.concatenate([G @ x[c * N:(c + 1) * N] for c in range(3)])
            y = Q @ (Minv @ (Q.conj().T @ Wx))
            out[:, ikx, kz, :] = y.reshape(3, N)
        return out

    # -- descent ---------------------------------------------------------------
    def descent_direction(self, u):
        """Returns (f, r) with f = -P_W J*(u) r(u)."""
        r = self.residual(u)
        return -self.project(self.adjoint(u, r)), r

    def descent_step(self, u, dtau):
        """One forward-Euler step of the projected adjoint descent; returns the
        new state and the cost J^2 of the old one."""
        f, r = self.descent_direction(u)
        return u + dtau * f, self.inner(r, r)

    # -- diagnostics -----------------------------------------------------------
    def dissipation(self, u):
        """D = <curl U, curl U>_W with U = u_b + u (so D = 1 for laminar flow)."""
        T = self.T
        U = self.base_flow() + u
        wx = T.ddy(U[2]) - T.ddz(U[1])
        wy = T.ddz(U[0]) - T.ddx(U[2])
        wz = T.ddx(U[1]) - T.ddy(U[0])
        w = np.stack([wx, wy, wz])
        return self.inner(w, w)

    def trajectory_projection(self, u):
        """(P1, P2) = Re of the n = 3 and n = 5 Chebyshev coefficients of the
        mean streamwise velocity (Sec. 5.1, state-space projection)."""
        return float(np.real(u[0, 0, 0, 3])), float(np.real(u[0, 0, 0, 5]))

    def defects(self, u):
        """(max |div coefficient|, max |wall value|, max |Hermitian defect|)."""
        g, T = self.g, self.T
        div = T.ddx(u[0]) + T.ddy(u[1]) + T.ddz(u[2])
        bp, bm = cheb.wall_rows(g.N)
        wall = max(np.max(np.abs(u @ bp)), np.max(np.abs(u @ bm)))
        herm = np.max(np.abs(u[:, 0, 0].imag))
        for ikx, kx in enumerate(g.kx):
            if kx > 0:
                jm = list(g.kx).index(-kx)
                herm = max(herm, np.max(np.abs(u[:, jm, 0] - np.conj(u[:, ikx, 0]))))
        return float(np.max(np.abs(div))), float(wall), float(herm)

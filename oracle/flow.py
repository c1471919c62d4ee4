"""Dealiased convective term of the perturbative NSE (oracle; test infrastructure).

Sec. 3.1 (momentum equation) gives the nonlinear part of F(u, p) as
-[(u_b.grad)u + (u.grad)u_b + (u.grad)u].  With the plane Couette base flow
u_b = y e_x (Sec. 5) and U = u_b + u this equals -(U.grad)U, because
(u_b.grad)u_b = y d/dx (y e_x) = 0.  The discrete operator is

    M_h(u) = -A[ (U.grad)U ],

with spectral derivatives (d/dx -> i a, d/dz -> i b, d/dy -> the exact
Chebyshev derivative), point values of every factor on the Nx x Ny x Nz grid
(Gauss-Lobatto in y), the pointwise product, and the analysis A = forward FFT
in x and z, truncation to the retained modes, and interpolation (C^{-1}) in y.

Inner products used for adjoints:
    <a, b>_W = sum over stored modes of w(kz) Re sum_c a_c^H G b_c   (spectral)
    <p, q>_g = (1/(Nx Nz)) sum over all grid points of p q            (grid)
With these, (Lemma 1) <p, grid(c)>_g = 2 <F p, c>_E for the x/z part, which
gives the adjoints used below; tests pin them against brute force.
"""

import numpy as np

from . import cheb


class Transforms:
    def __init__(self, g):
        self.g = g
        N = g.N
        self.C = cheb.synthesis(N)
        self.Cinv = np.linalg.inv(self.C)
        self.D = cheb.derivative(N)
        self.G = cheb.gram(N)
        self.Ginv = np.linalg.inv(self.G)
        self.y = cheb.gl_points(N)

    # -- x/z Fourier part on values at the Gauss-Lobatto points ---------------
    def grid_from_values(self, vals):
        """vals (nkx, nkz, N) complex, Hermitian on kz=0 -> real (N, Nx, Nz):
        p(x, z) = sum over the full plane of vals_k exp(i k.x)."""
        g = self.g
        spec = np.zeros((g.N, g.Nx, g.Nz // 2 + 1), dtype=complex)
        for ikx, kx in enumerate(g.kx):
            spec[:, kx % g.Nx, :g.nkz] = vals[ikx].T
        return np.fft.irfft2(spec, s=(g.Nx, g.Nz), axes=(1, 2), norm="forward")

    def values_from_grid(self, p):
        """Real (N, Nx, Nz) -> normalised Fourier coefficients of the retained
        modes, (nkx, nkz, N): (1/(Nx Nz)) sum p exp(-i k.x)."""
        g = self.g
        spec = np.fft.rfft2(p, axes=(1, 2), norm="forward")
        vals = np.empty((g.nkx, g.nkz, g.N), dtype=complex)
        for ikx, kx in enumerate(g.kx):
            vals[ikx] = spec[:, kx % g.Nx, :g.nkz].T
        return vals

    # -- full transforms -------------------------------------------------------
    def synth(self, f):
        """Coefficients (nkx, nkz, N) -> grid values (N, Nx, Nz)."""
        return self.grid_from_values(f @ self.C.T)

    def analysis(self, p):
        """A: grid (N, Nx, Nz) -> coefficients; FFT, truncate, then solve
        C c = values for the Chebyshev coefficients."""
        vals = self.values_from_grid(p)
        sh = vals.shape
        return np.linalg.solve(self.C, vals.reshape(-1, sh[-1]).T).T.reshape(sh)

    def analysis_adj(self, w):
        """W-to-grid adjoint of A: <A p, w>_W = <p, A* w>_g with
        A* w = (1/2) grid(C^{-T} G w)."""
        return 0.5 * self.grid_from_values(w @ (self.Cinv.T @ self.G).T)

    def synth_adj(self, p):
        """Grid-to-W adjoint of synth: <synth c, p>_g = <c, synth* p>_W with
        synth* p = 2 G^{-1} C^T F p."""
        vals = self.values_from_grid(p)
        return 2.0 * (vals @ self.C) @ self.Ginv.T

    # -- spectral derivatives and their W-adjoints ----------------------------
    def ddx(self, f):
        return 1j * self.g.a[:, None, None] * f

    def ddz(self, f):
        return 1j * self.g.b[None, :, None] * f

    def ddy(self, f):
        return f @ self.D.T

    def ddx_adj(self, f):
        return -1j * self.g.a[:, None, None] * f

    def ddz_adj(self, f):
        return -1j * self.g.b[None, :, None] * f

    def ddy_adj(self, f):
        return f @ (self.Ginv @ self.D.T @ self.G).T

    def d(self, j, f):
        return (self.ddx, self.ddy, self.ddz)[j](f)

    def d_adj(self, j, f):
        return (self.ddx_adj, self.ddy_adj, self.ddz_adj)[j](f)

    # -- velocity and its gradient on the grid --------------------------------
    def velocity_grid(self, u, base):
        """Return (V, dV): V[i] = velocity component i on the grid, dV[i][j] =
        d_j V_i.  With base=True the PCF base flow y e_x is added."""
        V = [self.synth(u[i]) for i in range(3)]
        dV = [[self.synth(self.d(j, u[i])) for j in range(3)] for i in range(3)]
        if base:
            V[0] = V[0] + self.y[:, None, None]
            dV[0][1] = dV[0][1] + 1.0
        return V, dV


def nonlinear(T, u):
    """M_h(u) = -A[(U.grad)U], U = y e_x + u."""
    U, dU = T.velocity_grid(u, base=True)
    out = np.empty(T.g.shape, dtype=complex)
    for i in range(3):
        q = U[0] * dU[i][0] + U[1] * dU[i][1] + U[2] * dU[i][2]
        out[i] = -T.analysis(q)
    return out


def nonlinear_lin(T, u, v):
    """Directional derivative of M_h at u along v (App. A.1):
    -A[(U.grad)v + (v.grad)U]."""
    U, dU = T.velocity_grid(u, base=True)
    V, dV = T.velocity_grid(v, base=False)
    out = np.empty(T.g.shape, dtype=complex)
    for i in range(3):
        q = sum(U[j] * dV[i][j] + V[j] * dU[i][j] for j in range(3))
        out[i] = -T.analysis(q)
    return out


def nonlinear_lin_adj(T, u, w):
    """W-adjoint of v -> nonlinear_lin(T, u, v), applied to w.

    Transposing -A[sum_j U_j synth(d_j v_i) + synth(v_j) d_j U_i] term by term:
    with w~_i = A* w_i on the grid,
      v_i collects d_j* synth*(U_j w~_i)        (advection by U),
      v_j collects synth*(sum_i d_j U_i w~_i)   (stretching by grad U),
    and the overall minus sign.  This is the discrete counterpart of the
    (grad r1)(u_b+u) - (grad(u_b+u))^T r1 terms of the adjoint operator
    (Sec. 3.3, App. A.2)."""
    U, dU = T.velocity_grid(u, base=True)
    wt = [T.analysis_adj(w[i]) for i in range(3)]
    out = np.zeros(T.g.shape, dtype=complex)
    for i in range(3):
        for j in range(3):
            out[i] += T.d_adj(j, T.synth_adj(U[j] * wt[i]))
    for j in range(3):
        out[j] += T.synth_adj(sum(dU[i][j] * wt[i] for i in range(3)))
    return -out

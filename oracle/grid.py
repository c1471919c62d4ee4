"""Discretisation of the plane Couette box (oracle; test infrastructure).

Box x in [0, Lx), y in [-1, 1], z in [0, Lz), periodic in x and z, no-slip
walls (Sec. 3.1).  Fourier in x and z, Chebyshev in y (Sec. 4).

Reading of the grid sizes: Nx and Nz are the numbers of collocation points
(FFT lengths) in x and z; the retained wavenumbers are |kx| <= Kx = Nx//3 - 1
and |kz| <= Kz = Nz//3 - 1 (the 2/3-rule cut-off, so that quadratic products
evaluated on the Nx x Nz grid are alias-free in x and z).  This is the only
cut-off that reproduces the paper's state-vector length of 20,218 at
Nx x Ny x Nz = 32 x 31 x 32 (Sec. 6.2).  y is not dealiased: products are
collocated at the Ny Gauss-Lobatto points.

Spectral arrays have shape (3, nkx, nkz, Ny), complex128, with kx in FFT
order (0, 1, .., Kx, -Kx, .., -1) and kz = 0..Kz (half plane; the kz < 0 modes
are the complex conjugates).  On the kz = 0 plane both signs of kx are stored
and must satisfy u(-kx) = conj(u(kx)); the (0, 0) mode is real.
"""

import numpy as np


class Grid:
    def __init__(self, Nx, Ny, Nz, Lx=2 * np.pi / 1.14, Lz=2 * np.pi / 2.5,
                 Re=400.0, dt=0.25):
        self.Nx, self.Ny, self.Nz = int(Nx), int(Ny), int(Nz)
        self.N = self.Ny
        self.Lx, self.Lz, self.Re, self.dt = float(Lx), float(Lz), float(Re), float(dt)
        self.Kx = self.Nx // 3 - 1
        self.Kz = self.Nz // 3 - 1
        if self.Kx < 0 or self.Kz < 0 or self.Ny < 5:
            raise ValueError("grid too small")
        self.nkx = 2 * self.Kx + 1
        self.nkz = self.Kz + 1
        self.kx = np.array(list(range(0, self.Kx + 1)) + list(range(-self.Kx, 0)))
        self.kz = np.arange(self.nkz)
        self.alpha = 2 * np.pi / self.Lx
        self.beta = 2 * np.pi / self.Lz
        self.a = self.alpha * self.kx            # x-wavenumber per ikx
        self.b = self.beta * self.kz             # z-wavenumber per kz
        self.lam = 1.0 / self.dt                 # lambda = 1/Delta t
        self.nu = 1.0 / self.Re
        self.shape = (3, self.nkx, self.nkz, self.N)

    # mode bookkeeping -------------------------------------------------------
    def kappa2(self, ikx, kz):
        return self.a[ikx] ** 2 + self.b[kz] ** 2

    def modes(self):
        """All stored (ikx, kz) pairs in storage order."""
        return [(i, k) for i in range(self.nkx) for k in range(self.nkz)]

    def weight(self, kz):
        """Weight of a stored mode in the volume-averaged L2 inner product:
        1/2 on the kz = 0 plane (both kx signs stored), 1 for kz > 0 (which
        also stands for its kz < 0 conjugate)."""
        return 0.5 if kz == 0 else 1.0

    def independent_modes(self):
        """Stored modes that carry independent data: all kz > 0, and kx > 0 on
        the kz = 0 plane; the (0, 0) mode is listed first and is real."""
        out = [(0, 0)]
        for i in range(self.nkx):
            for k in range(self.nkz):
                if k > 0 or self.kx[i] > 0:
                    out.append((i, k))
        return out

    def n_state(self):
        """Length of the minimal real state vector (Sec. 6.2)."""
        N = self.N
        return 4 * (self.Kx + 2 * self.Kx * self.Kz + self.Kz) * (N - 3) + 2 * (N - 2)

    def zeros(self):
        return np.zeros(self.shape, dtype=complex)

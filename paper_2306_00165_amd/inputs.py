"""Seeded synthetic initial guesses for plane Couette flow.

Input generation only: this module holds none of the method's arithmetic and
imports neither the HIP binding nor the CPU oracle, so both can be fed from it.
It uses numpy's Chebyshev and Gauss-Legendre library routines.

Recipe (a field that is exactly divergence-free, no-slip and Hermitian):
  * For each independent retained Fourier mode (kz > 0, or kz = 0 with kx > 0)
    whose envelope is non-zero, draw complex normal coefficients (PCG64, fixed
    seed, modes visited in storage order) for two polynomials P and Q, damped
    by exp(-n/2) in the Chebyshev index n, and set
        v   = (1 - y^2)^2 P     (so v(+-1) = v'(+-1) = 0),
        eta = (1 - y^2)   Q     (wall-normal vorticity, eta(+-1) = 0),
        u_x = (i a v' - i b eta)/kappa^2,  u_z = (i b v' + i a eta)/kappa^2.
    The mode is scaled so that its energy equals the envelope value.
  * For the (0, 0) mode (if the envelope allows it) u_x and u_z are real
    multiples (1 - y^2) Q of real random Q; v = 0.
  * The whole field is scaled to kinetic energy E = (1/2)<u, u>, with the
    volume-averaged L2 product.

Array layout: complex128, shape (3, 2Kx+1, Kz+1, Ny), kx in FFT order,
Kx = Nx//3 - 1, Kz = Nz//3 - 1.
"""

import numpy as np
from numpy.polynomial import chebyshev as npcheb
from numpy.polynomial import legendre as nplegendre

LX_W03 = 2 * np.pi / 1.14
LZ_W03 = 2 * np.pi / 2.5


def _gram(N):
    y, w = nplegendre.leggauss(N + 2)
    V = npcheb.chebvander(y, N - 1)
    return (V * w[:, None]).T @ V


def _truncate(c, N):
    out = np.zeros(N, dtype=complex)
    m = min(len(c), N)
    out[:m] = c[:m]
    return out


def envelope_exp(k):
    """Spectral amplitude proportional to exp(-|k|): energy ~ exp(-2|k|)."""
    return np.exp(-2.0 * k)


def make_envelope_kolmogorov(kmax_half):
    """Per-mode energy ~ |k|^(-8/3) (shell spectrum ~ k^(-5/3)) for
    0 < |k| <= kmax_half, zero elsewhere (including the mean mode)."""
    def env(k):
        if k <= 0 or k > kmax_half * (1 + 1e-12):
            return 0.0
        return k ** (-8.0 / 3.0)
    return env


def random_field(Nx, Ny, Nz, Lx=LX_W03, Lz=LZ_W03, envelope=envelope_exp,
                 energy=1e-3, seed=1, vdeg=None, edeg=None, mode_filter=None):
    """Return a seeded random admissible perturbation (see module docstring).

    envelope(|k|) gives the per-mode energy before normalisation; |k| is the
    physical wavenumber sqrt(a^2 + b^2).  vdeg/edeg cap the degrees of P and Q
    (defaults: the largest that keep v and eta within Ny coefficients).
    mode_filter(kx, kz) -> bool restricts the excited modes."""
    N = Ny
    Kx, Kz = Nx // 3 - 1, Nz // 3 - 1
    nkx, nkz = 2 * Kx + 1, Kz + 1
    kxs = list(range(0, Kx + 1)) + list(range(-Kx, 0))
    alpha, beta = 2 * np.pi / Lx, 2 * np.pi / Lz
    vdeg = N - 5 if vdeg is None else min(vdeg, N - 5)
    edeg = N - 3 if edeg is None else min(edeg, N - 3)
    rng = np.random.Generator(np.random.PCG64(seed))
    G = _gram(N)
    one_m_y2 = np.array([0.5, 0.0, -0.5])          # 1 - y^2 in the Chebyshev basis
    u = np.zeros((3, nkx, nkz, N), dtype=complex)

    def mode_energy(f, kz):
        w = 0.5 if kz == 0 else 1.0
        return w * sum(np.real(np.conj(f[c]) @ G @ f[c]) for c in range(3))

    for ikx in range(nkx):
        for kz in range(nkz):
            kx = kxs[ikx]
            if kz == 0 and kx < 0:
                continue
            if mode_filter is not None and not mode_filter(kx, kz):
                continue
            a, b = alpha * kx, beta * kz
            k = np.hypot(a, b)
            env = float(envelope(k))
            if env <= 0.0:
                continue
            if kx == 0 and kz == 0:
                f = np.zeros((3, N), dtype=complex)
                for c in (0, 2):
                    q = rng.standard_normal(edeg + 1) * np.exp(-0.5 * np.arange(edeg + 1))
                    f[c] = _truncate(npcheb.chebmul(one_m_y2, q), N).real
                e = mode_energy(f, 0)
                u[:, 0, 0] = f * np.sqrt(env / e) if e > 0 else 0.0
                continue
            damp_v = np.exp(-0.5 * np.arange(vdeg + 1))
            damp_e = np.exp(-0.5 * np.arange(edeg + 1))
            p = (rng.standard_normal(vdeg + 1) + 1j * rng.standard_normal(vdeg + 1)) * damp_v
            q = (rng.standard_normal(edeg + 1) + 1j * rng.standard_normal(edeg + 1)) * damp_e
            v = _truncate(npcheb.chebmul(npcheb.chebmul(one_m_y2, one_m_y2), p), N)
            eta = _truncate(npcheb.chebmul(one_m_y2, q), N)
            dv = _truncate(npcheb.chebder(v), N)
            k2 = a * a + b * b
            f = np.stack([(1j * a * dv - 1j * b * eta) / k2, v,
                          (1j * b * dv + 1j * a * eta) / k2])
            e = mode_energy(f, kz)
            f = f * np.sqrt(env / e)
            u[:, ikx, kz] = f
            if kz == 0:
                u[:, kxs.index(-kx), 0] = np.conj(f)
    # normalise the total kinetic energy (1/2)<u, u>
    tot = 0.0
    for kz in range(nkz):
        w = 0.5 if kz == 0 else 1.0
        for c in range(3):
            tot += w * np.real(np.einsum('in,nm,im->', np.conj(u[c, :, kz]), G, u[c, :, kz]))
    if tot > 0:
        u *= np.sqrt(2.0 * energy / tot)
    return u


# -- the workloads ------------------------------------------------------------

def config1_guess():
    """16 x 25 x 16, amplitude ~ exp(-|k|), E = 1e-3, seed 1."""
    return random_field(16, 25, 16, envelope=envelope_exp, energy=1e-3, seed=1)


def config2_guess():
    """32 x 33 x 32 streak + vortex seed: |kx| <= 1, kz in {1, 2}, Chebyshev
    degree <= 6 in every component, E = 5e-3, seed 2."""
    return streak_vortex_guess(32, 33, 32, 5e-3, 2)


def streak_vortex_guess(Nx, Ny, Nz, energy, seed, Lx=LX_W03, Lz=LZ_W03):
    """The 32 x 33 x 32 recipe on any grid: |kx| <= 1, kz in {1, 2}, Chebyshev
    degree <= 6 in every component."""
    return random_field(Nx, Ny, Nz, Lx, Lz, envelope=lambda k: 1.0, energy=energy, seed=seed, vdeg=2, edeg=4,
                        mode_filter=lambda kx, kz: abs(kx) <= 1 and kz in (1, 2))


def kolmogorov_guess(Nx, Ny, Nz, energy, seed, Lx=LX_W03, Lz=LZ_W03):
    """k^(-5/3) shell spectrum (per-mode energy ~ |k|^(-8/3)) up to half the
    largest retained |k|."""
    Kx, Kz = Nx // 3 - 1, Nz // 3 - 1
    kmax = np.hypot(2 * np.pi / Lx * Kx, 2 * np.pi / Lz * Kz)
    return random_field(Nx, Ny, Nz, Lx, Lz, envelope=make_envelope_kolmogorov(kmax / 2),
                        energy=energy, seed=seed)


def metric_guess():
    """48 x 49 x 48 workload of the steps/s metric: k^(-5/3), E = 0.03, seed 3."""
    return kolmogorov_guess(48, 49, 48, energy=0.03, seed=3)

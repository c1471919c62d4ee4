"""Symmetry operators of plane Couette flow on spectral arrays (test helper).

Sec. 5: translations tau(lx, lz), the rotation sigma_1 [u,v,w](x,y,z) ->
[-u,-v,w](-x,-y,z) and the reflection sigma_2 [u,v,w](x,y,z) -> [u,v,-w](x,y,-z);
s1 = tau(Lx/2, Lz/2) sigma_1 and s2 = tau(Lx/2, 0) sigma_2 (Sec. 5.1).
Arrays have shape (3, nkx, nkz, N) with kx in FFT order."""

import numpy as np


def _neg_kx_index(nkx):
    return [(nkx - i) % nkx for i in range(nkx)]


def shift(u, a, b, lx, lz):
    ph = np.exp(1j * (a[:, None] * lx + b[None, :] * lz))
    return u * ph[None, :, :, None]


def sigma1(u):
    nkx, N = u.shape[1], u.shape[3]
    out = u[:, _neg_kx_index(nkx)] * ((-1.0) ** np.arange(N))
    out[0] *= -1
    out[1] *= -1
    return out


def sigma2(u):
    nkx = u.shape[1]
    out = np.conj(u[:, _neg_kx_index(nkx)])
    out[2] *= -1
    return out


def s1(u, g):
    return shift(sigma1(u), g.a, g.b, g.Lx / 2, g.Lz / 2)


def s2(u, g):
    return shift(sigma2(u), g.a, g.b, g.Lx / 2, 0.0)

"""Pins for the oracle's Chebyshev operators against numpy's Chebyshev and
Gauss-Legendre library routines (independent implementations)."""

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb
from numpy.polynomial import legendre as nplegendre

from oracle import cheb

pytestmark = pytest.mark.parametrize("N", [5, 9, 25, 33, 49, 65])


def test_derivative_matches_chebder(N):
    rng = np.random.default_rng(N)
    c = rng.standard_normal(N)
    want = np.zeros(N)
    want[:N - 1] = npcheb.chebder(c)
    np.testing.assert_allclose(cheb.derivative(N) @ c, want, rtol=0, atol=1e-11 * np.abs(want).max())


def test_synthesis_matches_chebval(N):
    rng = np.random.default_rng(N + 1)
    c = rng.standard_normal(N)
    y = np.cos(np.pi * np.arange(N) / (N - 1))
    np.testing.assert_allclose(cheb.gl_points(N), y, atol=0, rtol=0)
    np.testing.assert_allclose(cheb.synthesis(N) @ c, npcheb.chebval(y, c), atol=1e-12)
    # interpolation recovers the coefficients of a degree <= N-1 polynomial
    back = np.linalg.solve(cheb.synthesis(N), npcheb.chebval(y, c))
    np.testing.assert_allclose(back, c, atol=1e-11)


def test_gram_matches_gauss_legendre(N):
    y, w = nplegendre.leggauss(N + 3)
    V = npcheb.chebvander(y, N - 1)
    np.testing.assert_allclose(cheb.gram(N), (V * w[:, None]).T @ V, atol=1e-13)


def test_wall_rows(N):
    rng = np.random.default_rng(N + 2)
    c = rng.standard_normal(N)
    bp, bm = cheb.wall_rows(N)
    assert abs(bp @ c - npcheb.chebval(1.0, c)) < 1e-12
    assert abs(bm @ c - npcheb.chebval(-1.0, c)) < 1e-12

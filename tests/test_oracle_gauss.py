"""Pins for the oracle's Gaussian latitudes and weights.

Gauss-Legendre quadrature with nlat nodes integrates every polynomial of
degree <= 2 nlat - 1 exactly, so the moments of the weights are fixed by
mathematics alone; small node counts have closed forms; and NumPy's
``leggauss`` gives the nodes independently (its weights are less accurate at
large nlat, so only its nodes are compared there).
"""

import math

import numpy as np
import pytest

from oracle import gauss_newton


@pytest.mark.parametrize("nlat", [2, 3, 4, 7, 80, 160, 400, 512, 2560])
def test_weights_sum_to_two(nlat):
    _mu, w = gauss_newton(nlat)
    assert abs(w.sum() - 2.0) <= 4e-15 * max(1.0, nlat / 80)


@pytest.mark.parametrize("nlat", [4, 9, 32, 80, 256])
def test_even_moments_exact(nlat):
    mu, w = gauss_newton(nlat)
    for k in range(0, nlat):  # degree 2k <= 2 nlat - 2
        exact = 2.0 / (2 * k + 1)
        got = float(np.sum(w * mu ** (2 * k)))
        assert abs(got - exact) <= 2e-14 * exact + 1e-16, (k, got, exact)


@pytest.mark.parametrize("nlat", [4, 9, 80])
def test_odd_moments_vanish(nlat):
    mu, w = gauss_newton(nlat)
    for k in range(0, nlat):
        assert abs(float(np.sum(w * mu ** (2 * k + 1)))) <= 1e-15


def test_closed_forms_small():
    mu, w = gauss_newton(2)
    np.testing.assert_allclose(mu, [1 / math.sqrt(3), -1 / math.sqrt(3)], rtol=0, atol=2.3e-16)
    np.testing.assert_allclose(w, [1.0, 1.0], rtol=0, atol=4.5e-16)

    mu, w = gauss_newton(3)
    np.testing.assert_allclose(mu, [math.sqrt(0.6), 0.0, -math.sqrt(0.6)], rtol=0, atol=2.3e-16)
    np.testing.assert_allclose(w, [5 / 9, 8 / 9, 5 / 9], rtol=0, atol=4.5e-16)

    mu, w = gauss_newton(4)
    r = 2.0 / 7.0 * math.sqrt(6.0 / 5.0)
    x_out, x_in = math.sqrt(3 / 7 + r), math.sqrt(3 / 7 - r)
    np.testing.assert_allclose(mu, [x_out, x_in, -x_in, -x_out], rtol=0, atol=2.3e-16)
    w_out, w_in = (18 - math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36
    np.testing.assert_allclose(w, [w_out, w_in, w_in, w_out], rtol=0, atol=6.7e-16)


@pytest.mark.parametrize("nlat", [16, 80, 400, 512])
def test_nodes_match_numpy_leggauss(nlat):
    mu, _w = gauss_newton(nlat)
    x, _ = np.polynomial.legendre.leggauss(nlat)
    np.testing.assert_allclose(mu, x[::-1], rtol=0, atol=3e-16)


@pytest.mark.parametrize("nlat", [80, 2560])
def test_ordering_and_symmetry(nlat):
    mu, w = gauss_newton(nlat)
    assert np.all(np.diff(mu) < 0), "north to south means mu descending"
    assert np.array_equal(mu, -mu[::-1])
    assert np.array_equal(w, w[::-1])
    assert np.all(w > 0)

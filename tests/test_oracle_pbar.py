"""Pins for the oracle's normalised associated Legendre functions.

Independent of the oracle's recurrence: closed forms for n <= 2, SciPy's
associated Legendre function (which carries the Condon-Shortley phase, so
(-1)^m is removed) times the normalisation sqrt((2n+1)/2 (n-m)!/(n+m)!),
discrete orthonormality under Gauss quadrature (exact for these degrees),
and the parity relation Pbar(-mu) = (-1)^(n-m) Pbar(mu).
"""

import math

import numpy as np
import pytest
from scipy.special import gammaln, lpmv

from oracle import gauss_newton, pbar


def _mu_samples():
    return np.linspace(-0.999, 0.999, 41)


def test_closed_forms_low_degree():
    mu = _mu_samples()
    s = np.sqrt((1 - mu) * (1 + mu))  # sin(theta), cancellation-free
    np.testing.assert_allclose(pbar(0, 2, mu)[:, 0], 1 / math.sqrt(2), rtol=1e-15)
    np.testing.assert_allclose(pbar(0, 2, mu)[:, 1], math.sqrt(1.5) * mu, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(pbar(0, 2, mu)[:, 2], math.sqrt(5 / 8) * (3 * mu * mu - 1), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(pbar(1, 2, mu)[:, 0], math.sqrt(3) / 2 * s, rtol=1e-14)
    np.testing.assert_allclose(pbar(1, 2, mu)[:, 1], math.sqrt(15) / 2 * mu * s, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(pbar(2, 2, mu)[:, 0], math.sqrt(15) / 4 * s * s, rtol=1e-14)


@pytest.mark.parametrize("m", [0, 1, 2, 5, 13, 30])
def test_matches_scipy_lpmv(m):
    N = 60
    mu = _mu_samples()
    ours = pbar(m, N, mu)
    for n in range(m, N + 1):
        norm = math.exp(0.5 * (math.log((2 * n + 1) / 2.0) + gammaln(n - m + 1) - gammaln(n + m + 1)))
        ref = (-1) ** m * lpmv(m, n, mu) * norm
        scale = max(1.0, float(np.max(np.abs(ref))))
        assert np.max(np.abs(ours[:, n - m] - ref)) <= 2e-12 * scale, (m, n)


@pytest.mark.parametrize("N", [31, 159, 255])
def test_discrete_orthonormality(N):
    mu, w = gauss_newton(N + 1)
    worst = 0.0
    for m in range(0, N + 1, max(1, N // 16)):
        P = pbar(m, N, mu)
        G = (P * w[:, None]).T @ P
        worst = max(worst, float(np.max(np.abs(G - np.eye(N - m + 1)))))
    assert worst <= 2e-13, worst


def test_orthonormality_at_tco1279_latitudes():
    # 2560 Gaussian latitudes, the TCo1279 octahedral grid; sampled m
    mu, w = gauss_newton(2560)
    N = 1279
    worst = 0.0
    for m in (0, 1, 7, 640, 1279):
        P = pbar(m, N, mu)
        G = (P * w[:, None]).T @ P
        worst = max(worst, float(np.max(np.abs(G - np.eye(N - m + 1)))))
    assert worst <= 5e-13, worst


@pytest.mark.parametrize("m", [0, 1, 4, 17])
def test_parity(m):
    N = 40
    mu = _mu_samples()
    a = pbar(m, N, mu)
    b = pbar(m, N, -mu)
    sign = (-1.0) ** np.arange(N - m + 1)
    assert np.array_equal(b, a * sign[None, :])


def test_sectoral_positive_no_condon_shortley():
    mu = np.array([0.3, -0.7])
    for m in range(0, 20):
        assert np.all(pbar(m, m, mu)[:, 0] > 0)

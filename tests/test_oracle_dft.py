"""Pins for the oracle's brute-force longitude DFT against NumPy's real FFT
(an independent library), at the ring lengths the grids use, including
lengths of the form 4 * prime that have no small factors."""

import numpy as np
import pytest

from oracle import dft_analysis, dft_synthesis

LENGTHS = [20, 24, 160, 388, 800, 2564, 5132, 5136]


@pytest.mark.parametrize("n", LENGTHS)
def test_synthesis_matches_irfft(n):
    rng = np.random.default_rng(n)
    mmax = (n - 1) // 2
    c = rng.standard_normal((3, mmax + 1)) + 1j * rng.standard_normal((3, mmax + 1))
    g = dft_synthesis(c, n)
    X = np.zeros((3, n // 2 + 1), dtype=np.complex128)
    X[:, : mmax + 1] = c * n
    ref = np.fft.irfft(X, n, axis=1)
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", LENGTHS)
def test_analysis_matches_rfft(n):
    rng = np.random.default_rng(n + 1)
    g = rng.standard_normal((2, n))
    ms = np.arange((n - 1) // 2 + 1)
    c = dft_analysis(g, n, ms)
    ref = np.fft.rfft(g, axis=1)[:, : ms.size] / n
    assert np.max(np.abs(c - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_imaginary_part_of_mean_ignored():
    c = np.array([[1.0 + 5.0j, 0.0]])
    assert np.allclose(dft_synthesis(c, 8), 1.0)


def test_analysis_inverts_synthesis():
    n = 36
    rng = np.random.default_rng(3)
    mmax = 17
    c = rng.standard_normal((1, mmax + 1)) + 1j * rng.standard_normal((1, mmax + 1))
    c[:, 0] = c[:, 0].real
    back = dft_analysis(dft_synthesis(c, n), n, np.arange(mmax + 1))
    assert np.max(np.abs(back - c)) <= 1e-14

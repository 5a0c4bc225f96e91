"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and lays them out; it holds none of the
transform's arithmetic, so the HIP path and the CPU oracle can both be fed the
same arrays without sharing any code of the method.

Recipe (synthetic stand-in for the dwarf's own input fields, which are not
available): spectral coefficients a_n^m are complex with real and imaginary
parts independent N(0, 1), scaled by 1 / (n + 1); a_n^0 is real.  Field f
uses its own generator ``numpy.random.default_rng(seed + f)`` and draws in the
m-major triangular order (m = 0..N, n = m..N), real part then imaginary part.
"""

import numpy as np

__all__ = ["spectral_coefficients", "grid_noise", "nspec_of"]


def nspec_of(N):
    """Number of stored coefficients, (N + 1)(N + 2) / 2."""
    return (N + 1) * (N + 2) // 2


def _degree_of_each_slot(N):
    # n for every slot of the m-major triangular layout (m = 0..N, n = m..N)
    return np.concatenate([np.arange(m, N + 1) for m in range(N + 1)])


def spectral_coefficients(N, nfields, seed=0, dtype=np.float64):
    """Complex coefficients [nfields, nspec] as interleaved real pairs.

    Returns a real array of shape [nfields, nspec, 2] (real, imaginary) in
    ``dtype``.  Values are drawn in float64 and rounded once to ``dtype``.
    """
    ns = nspec_of(N)
    inv_np1 = 1.0 / (_degree_of_each_slot(N) + 1.0)
    out = np.empty((nfields, ns, 2), dtype=dtype)
    for f in range(nfields):
        z = np.random.default_rng(seed + f).standard_normal(2 * ns).reshape(ns, 2)
        z *= inv_np1[:, None]
        z[: N + 1, 1] = 0.0  # m = 0 coefficients are real
        out[f] = z
    return out


def grid_noise(npts, nfields, seed=0, dtype=np.float64):
    """White N(0, 1) grid values [nfields, npts] (not band limited), field f
    drawn from ``default_rng(seed + f)``."""
    out = np.empty((nfields, npts), dtype=dtype)
    for f in range(nfields):
        out[f] = np.random.default_rng(seed + f).standard_normal(npts)
    return out

"""Regression snapshots of the oracle (written by tests/golden/make_golden.py,
which calls only the oracle): an unintended change to its arithmetic fails here."""

import os

import numpy as np
import pytest

from oracle import inverse
from paper_1908_06096_amd.inputs import spectral_coefficients

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("fname,N,grid,seed", [
    ("oracle_T7_full_seed3.txt", 7, "full", 3),
    ("oracle_T7_octahedral_seed3.txt", 7, "octahedral", 3),
])
def test_snapshot(fname, N, grid, seed):
    ref = np.loadtxt(os.path.join(HERE, fname))
    s = spectral_coefficients(N, 1, seed=seed)
    _f, g = inverse(s[..., 0] + 1j * s[..., 1], N, grid)
    np.testing.assert_allclose(g[0], ref, rtol=0, atol=1e-14)

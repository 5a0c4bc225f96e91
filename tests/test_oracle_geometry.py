"""Pins for the oracle's grid geometry and spectral layout.

The shapes are fixed outside the oracle:

* the TCo1279 octahedral grid of the operational model named in report
  section 4.3.1 has 2560 latitudes, 20 + 4i points on latitude i counted from
  either pole, 5136 points at the equator and 6,599,680 points in all (the
  workload's stated shape);
* the full Gaussian grids of the T79 and T399 workloads are 80 x 160 and
  400 x 800;
* the spectral layout is the m-major triangular enumeration (m = 0..N outer,
  n = m..N inner) with index(m, n) = m (2N + 3 - m) / 2 + (n - m), checked
  here against a plain counter over that enumeration.

Each pin is also run against a planted mistake (16 + 4i rings, 2N + 1
longitudes, an n-major layout), which must make it fail.
"""

import numpy as np
import pytest

from oracle import grid_geometry, nspec_of, spec_index
from paper_1908_06096_amd.inputs import spectral_coefficients


def _check_tco1279(geo):
    nlon = np.asarray(geo["nlon"])
    assert geo["nlat"] == 2560
    assert nlon.shape == (2560,)
    assert nlon[0] == 20 and nlon[-1] == 20
    assert nlon[1279] == 5136 and nlon[1280] == 5136
    assert np.array_equal(nlon[:1280], 20 + 4 * np.arange(1280))
    assert np.array_equal(nlon, nlon[::-1])
    assert int(nlon.sum()) == 6_599_680
    assert geo["npts"] == 6_599_680


def _check_full(geo, nlat, nlon):
    assert geo["nlat"] == nlat
    assert np.array_equal(np.asarray(geo["nlon"]), np.full(nlat, nlon))
    assert geo["npts"] == nlat * nlon


def _enumerated_index(N):
    """Position of every (m, n) by counting through the m-major enumeration."""
    pos = {}
    count = 0
    for m in range(N + 1):
        for n in range(m, N + 1):
            pos[(m, n)] = count
            count += 1
    return pos, count


def test_tco1279_shape():
    _check_tco1279(grid_geometry(1279, "octahedral"))


@pytest.mark.parametrize("N,nlat,nlon", [(79, 80, 160), (399, 400, 800)])
def test_full_grid_shapes(N, nlat, nlon):
    _check_full(grid_geometry(N, "full"), nlat, nlon)


@pytest.mark.parametrize("N", [1, 31, 159, 1279])
def test_octahedral_rings_mirror_and_grow_by_four(N):
    geo = grid_geometry(N, "octahedral")
    nlon = np.asarray(geo["nlon"])
    assert geo["nlat"] == 2 * (N + 1)
    assert np.array_equal(nlon, nlon[::-1])
    assert np.all(np.diff(nlon[: N + 1]) == 4)
    assert nlon[0] == 20


@pytest.mark.parametrize("N,grid", [(79, "full"), (399, "full"), (1279, "octahedral"), (63, "octahedral")])
def test_offsets_are_running_sums(N, grid):
    geo = grid_geometry(N, grid)
    nlon = np.asarray(geo["nlon"])
    mmax = np.asarray(geo["mmax"])
    assert geo["off"][0] == 0 and np.array_equal(np.diff(geo["off"]), nlon)
    assert geo["foff"][0] == 0 and np.array_equal(np.diff(geo["foff"]), mmax + 1)
    # no ring carries its Nyquist wavenumber or more than N
    assert np.all(2 * mmax < nlon) and np.all(mmax <= N)


def test_full_grid_rings_carry_every_wavenumber():
    # with 2N + 2 points a ring resolves m = 0..N, which the exact round trip
    # of the full grid needs: nfour = nlat (N + 1)
    for N in (79, 399):
        geo = grid_geometry(N, "full")
        assert np.all(np.asarray(geo["mmax"]) == N)
        assert geo["nfour"] == (N + 1) * (N + 1)


@pytest.mark.parametrize("N", [0, 1, 2, 7, 79, 1279])
def test_spectral_counts(N):
    assert nspec_of(N) == sum(N - m + 1 for m in range(N + 1))


def test_spectral_counts_of_the_workloads():
    assert nspec_of(79) == 3_240
    assert nspec_of(399) == 80_200
    assert nspec_of(1279) == 819_840


@pytest.mark.parametrize("N", [1, 2, 7, 40, 79])
def test_spec_index_is_the_m_major_enumeration(N):
    pos, count = _enumerated_index(N)
    assert count == nspec_of(N)
    for (m, n), p in pos.items():
        assert spec_index(N, m, n) == p


def test_spec_index_at_tco1279_ends():
    N = 1279
    assert spec_index(N, 0, 0) == 0
    assert spec_index(N, 0, N) == N
    assert spec_index(N, 1, 1) == N + 1
    assert spec_index(N, N, N) == nspec_of(N) - 1


def test_input_recipe_uses_the_same_layout():
    # the seeded inputs draw a_n^0 real: exactly the first N + 1 slots (m = 0)
    N = 9
    s = spectral_coefficients(N, 1, seed=5)
    zero_im = np.nonzero(s[0, :, 1] == 0.0)[0]
    assert np.array_equal(zero_im, [spec_index(N, 0, n) for n in range(N + 1)])


# ---- planted mistakes: each pin must reject them ----

def _mutated_octahedral(N, first, step):
    half = first + step * np.arange(N + 1)
    nlon = np.concatenate([half, half[::-1]])
    return {"nlat": 2 * (N + 1), "nlon": nlon, "npts": int(nlon.sum())}


@pytest.mark.parametrize("first,step", [(16, 4), (20, 2), (24, 4)])
def test_mutation_octahedral_rule_is_caught(first, step):
    with pytest.raises(AssertionError):
        _check_tco1279(_mutated_octahedral(1279, first, step))


def test_mutation_full_grid_longitudes_are_caught():
    nlat = 80
    geo = {"nlat": nlat, "nlon": np.full(nlat, 159), "npts": nlat * 159}
    with pytest.raises(AssertionError):
        _check_full(geo, 80, 160)


def test_mutation_n_major_layout_is_caught():
    N = 7

    def n_major(N, m, n):
        return n * (n + 1) // 2 + m

    pos, _ = _enumerated_index(N)
    assert any(n_major(N, m, n) != p for (m, n), p in pos.items())

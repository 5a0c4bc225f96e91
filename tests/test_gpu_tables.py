"""Plan-time kernels against the oracle: Gaussian latitudes and weights
(float64 Newton on the GPU), ring geometry, and the resident Pbar tables.

Both sides converge Newton's iteration to within an ulp of each root, but
not always to the same float.  The tolerances below are the first-order
effect of a 2-ulp difference in mu, derived from identities that hold at a
root or for every mu:
* weight: at a root of P_n, P'' = 2 mu P' / (1 - mu^2), so
  d ln w / d mu = -2 mu / (1 - mu^2); on top of that each side evaluates P'
  by an nlat-step recurrence, worth about nlat ulps of relative error;
* Pbar: (1 - mu^2) dPbar_n^m/dmu = -n mu Pbar_n^m + c Pbar_{n-1}^m with
  c = sqrt((2n+1)/(2n-1) (n^2 - m^2)) <= 1.01 n, so
  |dPbar_n^m/dmu| <= 2.1 n max|Pbar| / (1 - mu^2).
Near the poles these amplify an ulp of mu by 1/(1 - mu^2).  The sectoral
start value carries sin(theta)^m, so a last-bit difference in sin(theta)
(or in the m square roots of the seed) becomes about m ulps of relative
difference; each of the n - m recurrence steps adds about one more.  Hence
the extra term 2 (m + n) eps |Pbar|."""

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sht():
    from paper_1908_06096_amd import sht as mod

    return mod


@pytest.mark.parametrize("N,grid", [(1, "full"), (79, "full"), (399, "full"), (31, "octahedral"), (1279, "octahedral")])
def test_latitudes_weights_geometry(sht, N, grid):
    with sht.Plan(N, grid, 1, "fp32" if N == 1279 else "fp64") as plan:
        g = plan.geometry()
        geo = oracle.grid_geometry(N, grid)
        mu, w = oracle.gauss_newton(geo["nlat"])
        dmu = 2.3e-16
        assert np.all(np.abs(g["mu"] - mu) <= dmu)
        one_m = (1 - mu) * (1 + mu)
        bound = dmu * 2 * np.abs(mu) / one_m + 2 * geo["nlat"] * 2.2e-16
        _check_le(np.abs(g["w"] - w) / w, bound, "weights")
        assert abs(g["w"].sum() - 2.0) <= 4e-15 * max(1.0, geo["nlat"] / 80)
        assert np.array_equal(g["nlon"], geo["nlon"])
        assert np.array_equal(g["mmax"], geo["mmax"])
        assert np.array_equal(g["ring_offset"], geo["off"])
        assert np.array_equal(g["four_row"], geo["foff"])
        assert plan.npts == geo["npts"] and plan.nfour == geo["nfour"] and plan.nspec == geo["nspec"]


def _check_le(err, bound, what):
    err = np.asarray(err)
    bad = ~(err <= bound)
    if np.any(bad):
        i = np.unravel_index(np.argmax(np.where(bad, err / np.maximum(bound, 1e-300), 0)), err.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} of {err.size} over bound; worst at {i}: err {err[i]!r} "
                             f"bound {np.broadcast_to(bound, err.shape)[i]!r}; nan {int(np.isnan(err).sum())}")


def _first_ring(geo, m):
    nh = geo["nlat"] // 2
    return int(np.argmax(geo["mmax"][:nh] >= m))


@pytest.mark.parametrize("N,grid,prec", [(79, "full", "fp64"), (63, "octahedral", "fp64"), (63, "octahedral", "fp32"),
                                         (63, "octahedral", "bf16x3"), (1279, "octahedral", "fp64")])
def test_pbar_tables(sht, N, grid, prec):
    with sht.Plan(N, grid, 1, prec) as plan:
        geo = oracle.grid_geometry(N, grid)
        mu, _w = oracle.gauss_newton(geo["nlat"])
        nh = geo["nlat"] // 2
        ms = sorted(set([0, 1, 2, N // 3, N // 2, N - 1, N]))
        for m in ms:
            first, tab = plan.legendre_table(m)
            assert first == _first_ring(geo, m)
            ref = oracle.pbar(m, N, mu[first:nh])
            assert tab.shape == ref.shape
            x = mu[first:nh]
            scale = max(1.0, float(np.max(np.abs(ref))))
            n = np.arange(m, N + 1)[None, :]
            dmu = 2 * np.spacing(np.abs(x))[:, None]
            bound64 = (1e-13 * scale + dmu * 2.1 * np.maximum(n, 1) * scale / ((1 - x) * (1 + x))[:, None]
                       + 2 * (m + n) * 2.2e-16 * np.abs(ref))
            if prec == "fp64":
                _check_le(np.abs(tab - ref), bound64, f"m={m}")
            elif prec == "bf16x3":
                # hi + lo keeps 16 significant bits of the float32 value
                r32 = ref.astype(np.float32).astype(np.float64)
                _check_le(np.abs(tab - r32), 2.0 ** -16 * np.abs(r32) + 1e-45 + bound64, f"m={m}")
            else:
                ulp = np.spacing(np.abs(ref.astype(np.float32))).astype(np.float64)
                r32 = ref.astype(np.float32).astype(np.float64)
                _check_le(np.abs(tab - r32), ulp + bound64, f"m={m}")

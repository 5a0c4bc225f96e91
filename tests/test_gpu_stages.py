"""Stage-by-stage parity of the HIP path against the oracle's intermediates:
each stage is fed oracle data so that a failure names the stage."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import TOL, grid_inputs, rel_l2, spec_inputs, spec_to_complex

pytestmark = pytest.mark.gpu

CASES = [
    (1, "full", 1, "fp64"),
    (79, "full", 1, "fp64"),
    (79, "full", 17, "fp32"),
    (31, "octahedral", 3, "fp64"),
    (47, "octahedral", 33, "fp32"),
    (47, "octahedral", 33, "bf16x3"),
]


@pytest.fixture(scope="module")
def sht():
    from paper_1908_06096_amd import sht as mod

    return mod


def _ids(c):
    return "T%d-%s-F%d-%s" % c


def _fill_synthesis(plan, ws, four):
    view = plan.synthesis_fourier_view(ws)
    view.zero_()
    view[:, : plan.nfields] = torch.from_numpy(four.T.copy()).to(view.dtype).cuda()


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_legendre_inverse(sht, case):
    N, grid, F, prec = case
    with sht.Plan(N, grid, F, prec) as plan:
        spec_t, spec_c = spec_inputs(plan, seed=1)
        ws = plan.empty_workspace()
        plan.legendre_inverse(spec_t, ws)
        torch.cuda.synchronize()
        got = plan.synthesis_fourier_view(ws)[:, :F].cpu().numpy().T
        four, _g = oracle.inverse(spec_c, N, grid)
        assert rel_l2(got, four) <= TOL[prec]


# bf16x3 synthesis with the 128 x 128 tile (four waves, MFMA 32x32x16):
# ragged row tiles (L not a multiple of 256), column tiles past 2F, one and
# several k steps, m = 0
WIDE = [(31, "full", 1), (47, "octahedral", 33), (95, "octahedral", 70), (159, "octahedral", 5),
        (255, "octahedral", 64)]


@pytest.mark.parametrize("case", WIDE, ids=lambda c: "T%d-%s-F%d" % c)
def test_legendre_inverse_bf16x3_wide_tile(sht, case):
    N, grid, F = case
    with sht.Plan(N, grid, F, "bf16x3") as plan:
        plan.set_tile("c128")
        assert plan.tile == "c128"
        spec_t, spec_c = spec_inputs(plan, seed=1)
        ws = plan.empty_workspace()
        print(f"bf16x3 wide synthesis T{N} {grid} F={F}", flush=True)
        plan.legendre_inverse(spec_t, ws)
        torch.cuda.synchronize()
        got = plan.synthesis_fourier_view(ws)[:, :F].cpu().numpy().T
        four, _g = oracle.inverse(spec_c, N, grid)
        assert rel_l2(got, four) <= TOL["bf16x3"]
        # the same coefficients through the 128 x 64 tile (MFMA 16x16x32) agree
        # to the split's rounding
        plan.set_tile("c64")
        ws2 = plan.empty_workspace()
        plan.legendre_inverse(spec_t, ws2)
        torch.cuda.synchronize()
        other = plan.synthesis_fourier_view(ws2)[:, :F].cpu().numpy().T
        assert rel_l2(got, other) <= 1e-6


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_fourier_synthesis(sht, case):
    N, grid, F, prec = case
    with sht.Plan(N, grid, F, prec) as plan:
        geo = oracle.grid_geometry(N, grid)
        rng = np.random.default_rng(7)
        four = rng.standard_normal((F, geo["nfour"])) + 1j * rng.standard_normal((F, geo["nfour"]))
        if prec != "fp64":
            four = four.astype(np.complex64).astype(np.complex128)
        ws = plan.empty_workspace()
        _fill_synthesis(plan, ws, four)
        grid_t = plan.empty_grid()
        plan.fourier_synthesis(ws, grid_t)
        torch.cuda.synchronize()
        ref = np.zeros((F, geo["npts"]))
        for j in range(geo["nlat"]):
            ref[:, geo["off"][j]:geo["off"][j + 1]] = oracle.dft_synthesis(
                four[:, geo["foff"][j]:geo["foff"][j + 1]], int(geo["nlon"][j]))
        assert rel_l2(grid_t.cpu().numpy(), ref) <= TOL[prec]


def _analysis_form(geo, w, chat):
    """The analysis form of the Fourier workspace from the oracle's per-ring
    coefficients: slot 0 the weighted coefficients of north ring j, slot 1
    those of its mirror ring (the direct Legendre stage folds them into
    S = slot 0 + slot 1 and A = slot 0 - slot 1)."""
    nh = geo["nlat"] // 2
    F = chat.shape[0]
    out = np.zeros((geo["nfour"] // 2, 2, F), dtype=np.complex128)
    for j in range(nh):
        js = geo["nlat"] - 1 - j
        a = chat[:, geo["foff"][j]:geo["foff"][j + 1]]
        b = chat[:, geo["foff"][js]:geo["foff"][js + 1]]
        r0 = geo["foff"][j]
        out[r0:r0 + a.shape[1], 0] = (w[j] * a).T
        out[r0:r0 + a.shape[1], 1] = (w[js] * b).T
    return out


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_fourier_analysis(sht, case):
    N, grid, F, prec = case
    with sht.Plan(N, grid, F, prec) as plan:
        geo = oracle.grid_geometry(N, grid)
        _mu, w = oracle.gauss_newton(geo["nlat"])
        grid_t, grid_np = grid_inputs(plan, seed=3)
        ws = plan.empty_workspace()
        plan.fourier_analysis(grid_t, ws)
        torch.cuda.synchronize()
        got = plan.analysis_fourier_view(ws)[:, :, :F].cpu().numpy()
        chat, _s = oracle.direct(grid_np, N, grid)
        ref = _analysis_form(geo, w, chat)
        assert rel_l2(got, ref) <= TOL[prec]
        # m = 0 entries are real
        nh = geo["nlat"] // 2
        rows0 = geo["foff"][:nh]
        assert np.all(got[rows0, :, :].imag == 0)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_legendre_direct(sht, case):
    N, grid, F, prec = case
    with sht.Plan(N, grid, F, prec) as plan:
        geo = oracle.grid_geometry(N, grid)
        _mu, w = oracle.gauss_newton(geo["nlat"])
        _g, gnp = grid_inputs(plan, seed=5)
        chat, spec_ref = oracle.direct(gnp, N, grid)
        folded = _analysis_form(geo, w, chat)
        if prec != "fp64":
            folded = folded.astype(np.complex64).astype(np.complex128)
        ws = plan.empty_workspace()
        view = plan.analysis_fourier_view(ws)
        view.zero_()
        view[:, :, :F] = torch.from_numpy(folded).to(view.dtype).cuda()
        spec_t = plan.empty_spec()
        plan.legendre_direct(ws, spec_t)
        torch.cuda.synchronize()
        got = spec_to_complex(spec_t)
        assert rel_l2(got, spec_ref) <= TOL[prec]
        assert np.all(got[:, : N + 1].imag == 0)


# bf16x3 analysis with the 128 k x 128 column tile (eight waves, MFMA
# 32x32x16, transposing LDS reads): k tiles past K for one or both parities,
# one and several 32-ring steps, column tiles past 2F, m = 0
@pytest.mark.parametrize("case", WIDE, ids=lambda c: "T%d-%s-F%d" % c)
def test_legendre_direct_bf16x3_wide_tile(sht, case):
    N, grid, F = case
    with sht.Plan(N, grid, F, "bf16x3") as plan:
        plan.set_tile("c128")
        assert plan.tile == "c128"
        geo = oracle.grid_geometry(N, grid)
        _mu, w = oracle.gauss_newton(geo["nlat"])
        _g, gnp = grid_inputs(plan, seed=6)
        chat, spec_ref = oracle.direct(gnp, N, grid)
        folded = _analysis_form(geo, w, chat).astype(np.complex64).astype(np.complex128)
        ws = plan.empty_workspace()
        view = plan.analysis_fourier_view(ws)
        view.zero_()
        view[:, :, :F] = torch.from_numpy(folded).to(view.dtype).cuda()
        print(f"bf16x3 wide analysis T{N} {grid} F={F}", flush=True)
        spec_t = plan.empty_spec()
        plan.legendre_direct(ws, spec_t)
        torch.cuda.synchronize()
        got = spec_to_complex(spec_t)
        assert rel_l2(got, spec_ref) <= TOL["bf16x3"]
        assert np.all(got[:, : N + 1].imag == 0)
        # the 64 k x 128 column tile sums the same products in another order
        plan.set_tile("c64")
        spec2 = plan.empty_spec()
        plan.legendre_direct(ws, spec2)
        torch.cuda.synchronize()
        assert rel_l2(got, spec_to_complex(spec2)) <= 1e-6


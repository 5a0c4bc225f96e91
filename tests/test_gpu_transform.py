"""End-to-end parity of sht_inverse / sht_direct against the oracle, on
seeded inputs at sizes the oracle finishes in seconds (several tiles, ragged
tails in rings, wavenumbers and fields), plus round trips and determinism."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import TOL, grid_inputs, rel_l2, spec_inputs, spec_to_complex

pytestmark = pytest.mark.gpu

CASES = [
    (1, "full", 1, "fp64"),
    (3, "full", 2, "fp32"),
    (79, "full", 1, "fp64"),      # the T79 80 x 160 single-field case
    (79, "full", 1, "fp32"),
    (79, "full", 17, "fp32"),
    (1, "octahedral", 1, "fp64"),
    (31, "octahedral", 3, "fp64"),
    (63, "octahedral", 33, "fp32"),
    (95, "octahedral", 130, "fp32"),
    (159, "octahedral", 5, "fp64"),
    (79, "full", 3, "bf16x3"),
    (63, "octahedral", 33, "bf16x3"),
    (95, "octahedral", 130, "bf16x3"),
]


@pytest.fixture(scope="module")
def sht():
    from paper_1908_06096_amd import sht as mod

    return mod


def _ids(c):
    return "T%d-%s-F%d-%s" % c


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_inverse_matches_oracle(sht, case):
    N, grid, F, prec = case
    with sht.Plan(N, grid, F, prec) as plan:
        spec_t, spec_c = spec_inputs(plan, seed=2)
        g = plan.inverse(spec_t)
        torch.cuda.synchronize()
        _four, ref = oracle.inverse(spec_c, N, grid)
        assert rel_l2(g.cpu().numpy(), ref) <= TOL[prec]


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_direct_matches_oracle(sht, case):
    N, grid, F, prec = case
    with sht.Plan(N, grid, F, prec) as plan:
        grid_t, grid_np = grid_inputs(plan, seed=4)
        s = plan.direct(grid_t)
        torch.cuda.synchronize()
        _four, ref = oracle.direct(grid_np, N, grid)
        got = spec_to_complex(s)
        assert rel_l2(got, ref) <= TOL[prec]
        assert np.all(got[:, : N + 1].imag == 0)


@pytest.mark.parametrize("case", [(79, "full", 1, "fp64"), (79, "full", 3, "fp32"), (63, "octahedral", 4, "fp64"),
                                  (63, "octahedral", 4, "fp32"), (63, "octahedral", 4, "bf16x3")], ids=_ids)
def test_round_trip(sht, case):
    N, grid, F, prec = case
    with sht.Plan(N, grid, F, prec) as plan:
        spec_t, spec_c = spec_inputs(plan, seed=0)
        back = spec_to_complex(plan.direct(plan.inverse(spec_t)))
        spec_c = spec_c.copy()
        spec_c[:, : N + 1] = spec_c[:, : N + 1].real
        tol = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5}[prec]
        assert rel_l2(back, spec_c) <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("N,grid,F", [(31, "octahedral", 2), (79, "full", 37)])
def test_im_a0_ignored(sht, prec, N, grid, F):
    # every kernel drops Im a_n^0 in code of its own: the result with a large
    # imaginary part on the m = 0 coefficients is bitwise the result without,
    # and matches the oracle (which drops it by definition)
    with sht.Plan(N, grid, F, prec) as plan:
        spec_t, spec_c = spec_inputs(plan, seed=9)
        a = plan.inverse(spec_t).clone()
        spec_t[:, : N + 1, 1] = 123.0
        b = plan.inverse(spec_t)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        noisy = spec_c.copy()
        noisy[:, : N + 1] += 123.0j
        _four, ref = oracle.inverse(noisy, N, grid)
        assert rel_l2(b.cpu().numpy(), ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_deterministic(sht, prec):
    with sht.Plan(63, "octahedral", 19, prec) as plan:
        spec_t, _c = spec_inputs(plan, seed=6)
        g1 = plan.inverse(spec_t).clone()
        g2 = plan.inverse(spec_t)
        assert torch.equal(g1, g2)
        s1 = plan.direct(g1).clone()
        s2 = plan.direct(g1)
        assert torch.equal(s1, s2)


def test_single_harmonic(sht):
    N = 47
    with sht.Plan(N, "octahedral", 1, "fp64") as plan:
        spec = torch.zeros((1, plan.nspec, 2), dtype=torch.float64, device="cuda")
        idx = oracle.spec_index(N, 5, 12)
        spec[0, idx, 0] = 1.0
        back = spec_to_complex(plan.direct(plan.inverse(spec)))
        expect = np.zeros_like(back)
        expect[0, idx] = 1.0
        assert np.max(np.abs(back - expect)) <= 1e-12

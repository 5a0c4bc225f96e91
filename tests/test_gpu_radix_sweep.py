"""Ring-length coverage of the FFT stages: full grids whose single ring
length 2h (h = N + 1) takes each prime radix of the passes (7, 11, 13, 17,
19 and 23; in FP32 also 29, 31 and 37, in kernels of their own; primes
above 20 as a first pass only), the composite radix 14, or the chirp-z
convolution with a short length (FP64 above 23, both precisions above 37),
compared with the oracle in both directions and round-tripped; two fields,
so that work groups holding several fields run partly empty."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import TOL, grid_inputs, rel_l2, spec_inputs, spec_to_complex

pytestmark = pytest.mark.gpu

# N odd (full grids need a mirror for every ring); h = N + 1
TRUNCATIONS = [
    13,   # h = 14 = 2 * 7
    21,   # h = 22 = 2 * 11
    25,   # h = 26 = 2 * 13
    33,   # h = 34 = 2 * 17
    37,   # h = 38 = 2 * 19
    45,   # h = 46 = 2 * 23
    97,   # h = 98 = 2 * 7 * 7
    181,  # h = 182 = 2 * 7 * 13
    57,   # h = 58 = 2 * 29: radix 29 (FP32), chirp-z (FP64)
    61,   # h = 62 = 2 * 31: radix 31 (FP32), chirp-z (FP64)
    93,   # h = 94 = 2 * 47: chirp-z (both)
    221,  # h = 222 = 2 * 3 * 37: radix 37 and two more passes (FP32)
    105,  # h = 106 = 2 * 53: chirp-z
    201,  # h = 202 = 2 * 101: chirp-z
]
CASES = [(N, prec) for N in TRUNCATIONS for prec in ("fp64", "fp32")]


@pytest.fixture(scope="module")
def sht():
    from paper_1908_06096_amd import sht as mod

    return mod


def _ids(c):
    return "T%d-h%d-%s" % (c[0], c[0] + 1, c[1])


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_full_grid_ring_length(sht, case):
    N, prec = case
    with sht.Plan(N, "full", 2, prec) as plan:
        spec_t, spec_c = spec_inputs(plan, seed=7)
        g = plan.inverse(spec_t)
        torch.cuda.synchronize()
        _four, ref = oracle.inverse(spec_c, N, "full")
        assert rel_l2(g.cpu().numpy(), ref) <= TOL[prec]

        back = spec_to_complex(plan.direct(g))
        want = spec_c.copy()
        want[:, : N + 1] = want[:, : N + 1].real
        assert rel_l2(back, want) <= TOL[prec]

        grid_t, grid_np = grid_inputs(plan, seed=8)
        s = spec_to_complex(plan.direct(grid_t))
        _f, ref = oracle.direct(grid_np, N, "full")
        assert rel_l2(s, ref) <= TOL[prec]

"""sht_transform_static: the transform with the library's per-device static
scratch as its workspace gives bitwise the results of sht_inverse /
sht_direct with a caller workspace, on consecutive calls (the second on a
smaller problem, so stale scratch contents from the first are present), and
rejects a plan whose workspace exceeds the scratch."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1908_06096_amd import sht  # noqa: E402

from gpu_helpers import grid_inputs, spec_inputs  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

# (truncation, grid, fields): the first is the larger problem
CASES = [((159, "octahedral", 16), (31, "full", 3)), ((127, "full", 9), (47, "octahedral", 1))]


def _pair(plan, seed):
    spec, _ = spec_inputs(plan, seed=seed)
    grid, _ = grid_inputs(plan, seed=seed + 7)
    ref_g = plan.inverse(spec)
    ref_s = plan.direct(grid)
    out_g = plan.empty_grid()
    out_s = plan.empty_spec()
    print(f"static scratch: T{plan.truncation} {plan.grid} F={plan.nfields} {plan.precision}", flush=True)
    plan.transform_static("inverse", spec, out_g)
    plan.transform_static("direct", grid, out_s)
    torch.cuda.synchronize()
    return ref_g, ref_s, out_g, out_s


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("big,small", CASES)
def test_static_scratch_matches_caller_workspace(precision, big, small):
    for k, (N, grid, F) in enumerate((big, small)):
        with sht.Plan(N, grid, F, precision) as plan:
            assert plan.workspace_bytes <= sht.STATIC_SCRATCH_BYTES
            ref_g, ref_s, out_g, out_s = _pair(plan, seed=11 * k + 1)
            assert torch.equal(out_g, ref_g)
            assert torch.equal(out_s, ref_s)
            assert np.isfinite(out_s.cpu().numpy()).all()


def test_static_scratch_rejects_oversized_plan():
    # T399 full grid, 32 fields, FP64: 160000 Fourier rows x 32 x 16 B = 82 MB
    with sht.Plan(399, "full", 32, "fp64") as plan:
        assert plan.workspace_bytes > sht.STATIC_SCRATCH_BYTES
        spec = plan.empty_spec()
        grid = plan.empty_grid()
        lib = sht.library()
        rc = lib.sht_transform_static(plan._h, 0, ctypes.c_void_p(spec.data_ptr()),
                                      ctypes.c_void_p(grid.data_ptr()), None)
        assert rc == -5
        with pytest.raises(sht.SHTError):
            plan.transform_static("direct", grid, spec)

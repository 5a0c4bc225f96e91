"""Serving on the GPU: requests admitted while others run overlap on the
device, and every result is bitwise the one the same request gets alone."""

import pytest
import torch

pytestmark = pytest.mark.gpu


def test_results_same_alone_and_in_mix():
    from paper_1908_06096_amd import sht
    from paper_1908_06096_amd.serve import GpuExecutor, Scheduler, draw_requests

    reqs = draw_requests(40, rate=2000.0, seed=3, fields=(1, 24), ladder=(31, 47, 63, 95))
    ex = GpuExecutor(slots=4, input_fields=24, keep_results=True)
    for N in (31, 47, 63, 95):
        for prec in ("fp32", "bf16x3"):
            ex.warm(N, prec)
    sched = Scheduler(ex, 4, 8 << 30)
    done = sched.run(reqs)
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    assert max(r.slot for r in reqs) > 0, "more than one slot was used"
    overlapped = any(a.admitted < b.completed and b.admitted < a.completed
                     for a in reqs for b in reqs if a.rid < b.rid)
    assert overlapped, "no two requests were on the device at the same time"
    for r in reqs:
        with sht.Plan(r.truncation, "octahedral", r.fields, r.precision) as plan:
            spec_in = ex.inputs[(r.truncation, r.precision)][: r.fields]
            alone = plan.direct(plan.inverse(spec_in))
            torch.cuda.synchronize()
            assert torch.equal(alone, ex.results[r.rid]), r.rid
    ex.close()

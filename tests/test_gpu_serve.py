"""Serving on the GPU: requests admitted while others run overlap on the
device, and every result is bitwise the one the same request gets alone."""

import pytest
import torch

pytestmark = pytest.mark.gpu


def test_results_same_alone_and_in_mix():
    from paper_1908_06096_amd import sht
    from paper_1908_06096_amd.serve import GpuExecutor, Scheduler, draw_requests

    reqs = draw_requests(40, rate=2000.0, seed=3, fields=(1, 24), ladder=(31, 47, 63, 95))
    ex = GpuExecutor(slots=4, input_fields=24, keep_results=True, max_fields=24)
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
            spec_in = ex.inputs(r.truncation, r.precision, ex._bucket(r.fields))[: r.fields]
            alone = plan.direct(plan.inverse(spec_in))
            torch.cuda.synchronize()
            # the request ran on the plan of its field count rounded up to
            # 16; its own fields are bitwise those of the plan of exactly F
            assert torch.equal(alone, ex.results[r.rid][: r.fields]), r.rid
    ex.close()


def test_binding_budget_evicts_idle_tables():
    # a budget with room for one table set and one request at a time:
    # requests for other truncations evict the idle set (released in stream
    # order) and the first truncation's set is made again when it returns
    from paper_1908_06096_amd.serve import GpuExecutor, Request, Scheduler

    seq = [159, 127, 95, 63, 159, 95]
    reqs = [Request(i, 0.02 * i, N, 40, "fp32") for i, N in enumerate(seq)]
    ex = GpuExecutor(slots=2, max_fields=48, input_fields=48)
    ex.inputs(159, "fp32", 48)  # the input pool is resident from the start
    budget = ex.resident() + ex.footprint(Request(0, 0.0, 159, 48, "fp32"))
    sched = Scheduler(ex, 2, budget)
    done = sched.run(reqs)
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    assert ex.evictions >= 3  # T159 -> T127 -> T95 (+ T63) -> T159 each displace a set
    assert sched.peak <= budget
    ex.close()

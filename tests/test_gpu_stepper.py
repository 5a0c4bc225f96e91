"""Time-stepping workload: K semi-implicit steps of the reaction-diffusion
equation (synthesis, logistic term on the grid, analysis, implicit
diffusion) against the same loop written with the oracle's transforms; the
HIP-graph replay against the uncaptured steps, replay by replay, with other
eager work and synchronisations between the replays."""

import math

import numpy as np
import pytest
import torch

import oracle
from oracle.vector_oracle import degree_of_slot
from gpu_helpers import TOL, np_dtype, rel_l2, spec_to_complex
from paper_1908_06096_amd.inputs import spectral_coefficients

pytestmark = pytest.mark.gpu

DT, RATE, NU = 0.1, 1.0, 1e-2


@pytest.fixture(scope="module")
def sht():
    from paper_1908_06096_amd import sht as mod

    return mod


def _initial_state(N, F, prec, seed):
    """Small perturbations (0.05 x the seeded coefficients) of the mean 0.5:
    u stays in (0, 1), where the logistic term is stable."""
    s = 0.05 * spectral_coefficients(N, F, seed=seed)
    s[:, 0, 0] = 0.5 * math.sqrt(2.0)  # a_0^0 Pbar_0^0 = 0.5
    s = s.astype(np_dtype(prec))
    c = s[..., 0].astype(np.float64) + 1j * s[..., 1].astype(np.float64)
    return torch.from_numpy(np.ascontiguousarray(s)).cuda(), c


def _oracle_steps(a, N, grid, nsteps):
    n = degree_of_slot(N).astype(np.float64)
    damp = 1.0 / (1.0 + DT * NU * n * (n + 1.0))
    for _ in range(nsteps):
        _four, g = oracle.inverse(a, N, grid)
        g = g + DT * RATE * g * (1.0 - g)
        _f2, b = oracle.direct(g, N, grid)
        a = b * damp[None, :]
    return a


CASES = [(31, "full", 2, "fp64"), (47, "octahedral", 3, "fp64"), (63, "octahedral", 5, "fp32"),
         (79, "full", 3, "bf16x3")]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "T%d-%s-F%d-%s" % c)
def test_steps_match_oracle(sht, case):
    N, grid, F, prec = case
    K = 4
    with sht.Plan(N, grid, F, prec) as plan:
        spec, a0 = _initial_state(N, F, prec, seed=17)
        stream = torch.cuda.Stream()
        print(f"stepper T{N} {grid} F={F} {prec}", flush=True)
        with sht.Stepper(plan, spec, DT, RATE, NU, graph=True, stream=stream) as st:
            st.run(K, stream=stream)
            stream.synchronize()
        ref = _oracle_steps(a0, N, grid, K)
        # each step is two transforms, each within the stated tolerance of
        # the oracle's; K steps add at most 2K such errors (the diffusion
        # damps them and the logistic term changes them by at most a factor
        # 1 + dt r |1 - 2u| ~ 1, as u stays near 0.5)
        assert rel_l2(spec_to_complex(spec), ref) <= 2 * K * TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_graph_replays_match_eager_steps(sht, prec):
    N, grid, F = 63, "octahedral", 4
    with sht.Plan(N, grid, F, prec) as plan:
        s0, _ = _initial_state(N, F, prec, seed=23)
        eager_spec = s0.clone()
        graph_spec = s0.clone()
        stream = torch.cuda.Stream()
        with sht.Stepper(plan, eager_spec, DT, RATE, NU, graph=False, stream=stream) as eager, \
                sht.Stepper(plan, graph_spec, DT, RATE, NU, graph=True, stream=stream) as graphed:
            other = torch.randn(1 << 16, device="cuda")
            for step in range(5):
                eager.run(1, stream=stream)
                stream.synchronize()
                # unrelated eager work between the replays
                other = torch.sin(other) * 1.5
                torch.cuda.synchronize()
                graphed.run(1, stream=stream)
                stream.synchronize()
                assert torch.equal(graph_spec, eager_spec), f"replay {step}"
            # several replays queued back to back match as many eager steps
            eager.run(3, stream=stream)
            graphed.run(3, stream=stream)
            stream.synchronize()
            assert torch.equal(graph_spec, eager_spec)
            assert torch.isfinite(graph_spec).all()
        # a graph of 4 steps: 10 steps = 2 replays + 2 steps kernel by kernel
        multi_spec = s0.clone()
        eager_spec = s0.clone()
        with sht.Stepper(plan, eager_spec, DT, RATE, NU, graph=False, stream=stream) as eager, \
                sht.Stepper(plan, multi_spec, DT, RATE, NU, graph=True, graph_steps=4, stream=stream) as multi:
            for _ in range(2):
                eager.run(10, stream=stream)
                multi.run(10, stream=stream)
                stream.synchronize()
                torch.cuda.synchronize()
                assert torch.equal(multi_spec, eager_spec)


def test_stepper_rejects_bad_arguments(sht):
    import ctypes

    lib = sht.library()
    with sht.Plan(31, "full", 1, "fp64") as plan:
        spec = plan.empty_spec()
        grid = plan.empty_grid()
        ws = plan.empty_workspace()
        p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        h = ctypes.c_void_p()
        # graph capture needs a stream other than the null stream
        assert lib.sht_stepper_create(ctypes.byref(h), plan._h, 0.1, 1.0, 1e-3, p(spec), p(grid), p(ws), 1, 1,
                                      None) == -1
        assert lib.sht_stepper_create(ctypes.byref(h), plan._h, -0.1, 1.0, 1e-3, p(spec), p(grid), p(ws), 0, 1,
                                      None) == -1
        assert lib.sht_stepper_create(ctypes.byref(h), plan._h, 0.1, 1.0, 1e-3, p(spec), p(grid), p(ws), 4, 1,
                                      None) == -1
        assert lib.sht_stepper_create(ctypes.byref(h), plan._h, 0.1, 1.0, 1e-3, p(spec), p(grid), p(ws), 1, 0,
                                      None) == -1
        assert not h.value

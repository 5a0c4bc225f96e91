"""Table-free plans (no resident Pbar tables; each transform makes one chunk
of wavenumbers' tables at a time in its workspace): results bitwise equal
to a plan with resident tables, over chunk sizes from one wavenumber to
many, in every precision; parity with the oracle; the time-stepping loop on
a table-free plan; the plan keeps no table memory."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import TOL, grid_inputs, rel_l2, spec_inputs, spec_to_complex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sht():
    from paper_1908_06096_amd import sht as mod

    return mod


CASES = [
    (31, "full", 2, "fp64", 1),            # 1-byte chunks: one wavenumber per chunk
    (79, "full", 3, "fp32", 64 << 10),
    (95, "octahedral", 17, "fp32", 256 << 10),
    (159, "octahedral", 5, "fp64", 1 << 20),
    (63, "octahedral", 40, "bf16x3", 128 << 10),
    (255, "octahedral", 9, "fp32", 0),     # default chunk: one chunk
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "T%d-%s-F%d-%s-chunk%d" % c)
def test_table_free_equals_resident_tables(sht, case):
    N, grid, F, prec, chunk = case
    with sht.Plan(N, grid, F, prec) as ref, sht.Plan(N, grid, F, prec, table_free=True, chunk_bytes=chunk) as tf:
        assert tf.info.table_free == 1 and tf.info.table_bytes == 0
        assert tf.info.chunk_table_bytes > 0
        spec_t, _ = spec_inputs(ref, seed=3)
        grid_t, _ = grid_inputs(ref, seed=4)
        print(f"table-free T{N} {grid} F={F} {prec} chunk {chunk}", flush=True)
        g_ref = ref.inverse(spec_t)
        g_tf = tf.inverse(spec_t)
        s_ref = ref.direct(grid_t)
        s_tf = tf.direct(grid_t)
        torch.cuda.synchronize()
        assert torch.equal(g_ref, g_tf)
        assert torch.equal(s_ref, s_tf)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_table_free_matches_oracle(sht, prec):
    N, grid, F = 63, "octahedral", 4
    with sht.Plan(N, grid, F, prec, table_free=True, chunk_bytes=32 << 10) as tf:
        spec_t, spec_c = spec_inputs(tf, seed=9)
        g = tf.inverse(spec_t)
        torch.cuda.synchronize()
        _f, ref = oracle.inverse(spec_c, N, grid)
        assert rel_l2(g.cpu().numpy(), ref) <= TOL[prec]
        grid_t, grid_np = grid_inputs(tf, seed=10)
        s = tf.direct(grid_t)
        torch.cuda.synchronize()
        _f2, sref = oracle.direct(grid_np, N, grid)
        assert rel_l2(spec_to_complex(s), sref) <= TOL[prec]


def test_table_free_stepper_and_like(sht):
    N, grid, F = 47, "octahedral", 3
    with sht.Plan(N, grid, F, "fp32") as ref, sht.Plan(N, grid, F, "fp32", table_free=True,
                                                       chunk_bytes=16 << 10) as tf:
        spec_t, _ = spec_inputs(ref, seed=12)
        a = spec_t * 0.05
        a[:, 0, 0] += 0.5 * 2 ** 0.5
        b = a.clone()
        stream = torch.cuda.Stream()
        with sht.Stepper(ref, a, 0.1, 1.0, 1e-2, graph=True, stream=stream) as s1, \
                sht.Stepper(tf, b, 0.1, 1.0, 1e-2, graph=True, stream=stream) as s2:
            s1.run(3, stream=stream)
            s2.run(3, stream=stream)
            stream.synchronize()
        assert torch.equal(a, b)
        like = sht.Plan(None, nfields=5, like=tf)
        assert like.info.table_free == 1
        spec5, _ = spec_inputs(like, seed=13)
        with sht.Plan(N, grid, 5, "fp32") as ref5:
            g1 = ref5.inverse(spec5)
            g2 = like.inverse(spec5)
            torch.cuda.synchronize()
            assert torch.equal(g1, g2)
        like.close()

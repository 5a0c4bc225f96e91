"""Batches of uneven transforms in shared launches: every transform's result
is bitwise the one it gets alone (same kernels, same summation order per
output whatever the tile variant or launch shape), persistent or not, through
a replayed HIP graph or not, after autotuning or not; and the batch agrees
with the oracle."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import TOL, rel_l2, spec_inputs, spec_to_complex

pytestmark = pytest.mark.gpu

SHAPES = [(47, 1), (31, 33), (63, 5), (31, 2), (95, 70), (47, 17)]


@pytest.fixture(scope="module")
def sht():
    from paper_1908_06096_amd import sht as mod

    return mod


def _make(sht, prec, shapes=SHAPES, seed=0):
    plans = [sht.Plan(N, "octahedral", F, prec) for N, F in shapes]
    specs, specs_c = [], []
    for i, p in enumerate(plans):
        t, c = spec_inputs(p, seed=seed + 100 * i)
        specs.append(t)
        specs_c.append(c)
    return plans, specs, specs_c


def _alone(plans, specs):
    grids, backs = [], []
    for p, s in zip(plans, specs):
        g = p.inverse(s)
        grids.append(g.clone())
        backs.append(p.direct(g).clone())
    torch.cuda.synchronize()
    return grids, backs


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x3"])
@pytest.mark.parametrize("persistent,graph", [(False, False), (True, False), (True, True)])
def test_batch_equals_alone(sht, prec, persistent, graph):
    plans, specs, _ = _make(sht, prec)
    ref_g, ref_b = _alone(plans, specs)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        grids = [p.empty_grid() for p in plans]
        backs = [p.empty_spec() for p in plans]
        b = sht.Batch(plans, persistent=persistent, graph=graph)
        b.bind(specs, grids)
        b.inverse()
        stream.synchronize()
        for g, r in zip(grids, ref_g):
            assert torch.equal(g, r)
        b.bind(backs, grids)  # analysis reads grids[i], writes backs[i]
        b.direct()
        stream.synchronize()
        for s, r in zip(backs, ref_b):
            assert torch.equal(s, r)
        b.close()
    for p in plans:
        p.close()


def test_graph_replays_and_rebinding(sht):
    plans, specs, _ = _make(sht, "fp32")
    ref_g, _ = _alone(plans, specs)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = sht.Batch(plans, persistent=True, graph=True)
        for rep in range(4):
            grids = [p.empty_grid().fill_(float("nan")) for p in plans]
            b.bind(specs, grids)
            b.inverse()
            stream.synchronize()
            # eager work between replays
            junk = torch.randn(1 << 20, device="cuda").sum().item()
            assert np.isfinite(junk)
            for g, r in zip(grids, ref_g):
                assert torch.equal(g, r), rep
        b.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("graph", [False, True])
def test_rebinding_is_stream_ordered(sht, graph):
    # bind, inverse, bind, direct, bind, inverse enqueued on one non-blocking
    # stream with no host synchronisation in between: each run uses the
    # buffers bound just before it
    plans, specs, _ = _make(sht, "fp32")
    ref_g, ref_b = _alone(plans, specs)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        grids = [p.empty_grid() for p in plans]
        grids2 = [p.empty_grid().fill_(float("nan")) for p in plans]
        backs = [p.empty_spec().fill_(float("nan")) for p in plans]
        b = sht.Batch(plans, persistent=True, graph=graph)
        b.bind(specs, grids)
        b.inverse()
        b.bind(backs, grids)
        b.direct()
        b.bind(specs, grids2)
        b.inverse()
        stream.synchronize()
        for g, g2, r in zip(grids, grids2, ref_g):
            assert torch.equal(g, r)
            assert torch.equal(g2, r)
        for s_, r in zip(backs, ref_b):
            assert torch.equal(s_, r)
        b.close()
    for p in plans:
        p.close()


def test_tuned_batch_equals_alone(sht):
    plans, specs, _ = _make(sht, "fp32")
    ref_g, ref_b = _alone(plans, specs)
    grids = [p.empty_grid() for p in plans]
    backs = [p.empty_spec() for p in plans]
    b = sht.Batch(plans, persistent=True)
    b.bind(specs, grids)
    b.tune()
    tiles = b.tiles()
    assert len(tiles) == len(plans) and set(tiles) <= {"c128", "c64", "c32"}
    b.inverse()
    b.bind(backs, grids)
    b.direct()
    torch.cuda.synchronize()
    for g, r in zip(grids, ref_g):
        assert torch.equal(g, r)
    for s, r in zip(backs, ref_b):
        assert torch.equal(s, r)
    b.close()
    for p in plans:
        p.close()


def test_tuning_cache_round_trip(sht, tmp_path):
    plans, specs, _ = _make(sht, "fp32")
    grids = [p.empty_grid() for p in plans]
    cache = str(tmp_path / "tiles.json")
    b = sht.Batch(plans, persistent=True)
    b.bind(specs, grids)
    first = b.tune(cache=cache)
    b.inverse()
    torch.cuda.synchronize()
    ref = [g.clone() for g in grids]
    b.close()
    # a new batch over the same shapes takes the stored choices without timing
    b2 = sht.Batch(plans, persistent=True)
    b2.bind(specs, grids)
    b2.set_tiles(["c32"] * len(plans))
    assert b2.tiles() == ["c32"] * len(plans)
    assert b2.tune(cache=cache) == first
    b2.inverse()
    torch.cuda.synchronize()
    for g, r in zip(grids, ref):
        assert torch.equal(g, r)
    b2.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("tile", ["c128", "c64", "c32"])
def test_tile_variants_agree(sht, tile):
    with sht.Plan(63, "octahedral", 21, "fp32") as plan:
        spec_t, _ = spec_inputs(plan, seed=8)
        ref = plan.inverse(spec_t).clone()
        ref_b = plan.direct(ref).clone()
        plan.set_tile(tile)
        assert plan.tile == tile
        g = plan.inverse(spec_t)
        assert torch.equal(g, ref)
        assert torch.equal(plan.direct(g), ref_b)


def test_batch_matches_oracle(sht):
    shapes = [(31, 3), (47, 1), (63, 9)]
    plans, specs, specs_c = _make(sht, "fp32", shapes, seed=5)
    grids = [p.empty_grid() for p in plans]
    b = sht.Batch(plans, persistent=True)
    b.bind(specs, grids)
    b.inverse()
    torch.cuda.synchronize()
    for (N, F), g, c in zip(shapes, grids, specs_c):
        _f, ref = oracle.inverse(c, N, "octahedral")
        assert rel_l2(g.cpu().numpy(), ref) <= TOL["fp32"]
    b.close()
    for p in plans:
        p.close()


def test_batch_rejects_mixed_precision(sht):
    a = sht.Plan(31, "octahedral", 1, "fp32")
    c = sht.Plan(31, "octahedral", 1, "fp64")
    with pytest.raises(sht.SHTError):
        sht.Batch([a, c])
    a.close()
    c.close()

"""Throughput benchmark of the spherical-harmonic transform on one MI355X.

One step = one round trip (synthesis then analysis) of every field of the
workload, inputs resident in HBM.  Default workload: TCo1279 octahedral
reduced Gaussian grid (2560 rings, 20 + 4i points on ring i from each pole,
6,599,680 points), triangular truncation 1279, 411 fields (3 fields x 137
levels), Legendre products and FFTs in FP32.  Spectral coefficients are the
seeded synthetic recipe of paper_1908_06096_amd.inputs (complex N(0,1) scaled
by 1/(n+1), one generator per field).

Prints one JSON line (metric, value = field-transforms/s, per-stage timings,
the roofline of the dominant kernel measured with HIP events on the stream the
kernels run on, the FP32 / bf16x3 synthesis compared with the plain FP64 form
on the same GPU, and the FP64 CPU oracle's rate on a bounded sample).

    python bench.py [--steps K] [--warmup W] [--precision fp32|bf16x3|fp64]
                    [--variants bf16x3,fp64]

The main precision and each variant (other precisions of the same workload,
for comparison) are timed over K steps.  Further objects on the same line:
``configs`` (the T79 single-field per-call latency and the T399 x 411 FP64
throughput), ``stepping`` (time steps of synthesis -> grid-point operation
-> analysis -> spectral operation, uncaptured against HIP-graph replay),
``vector`` (vorticity/divergence <-> winds at TCo1279), ``batch`` and
``serving``.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK = {  # MI355X published dense peaks
    "fp64": 78.6e12,
    "fp32": 157.3e12,
    "bf16": 2516.6e12,
    "hbm": 8.0e12,
}

WORKLOADS = {
    # name: (truncation, grid, fields)
    "TCo1279-O1280-F411": (1279, "octahedral", 411),
    "T399-full-400x800-F411": (399, "full", 411),
    "T79-full-80x160-F1": (79, "full", 1),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def geometry_counts(N, grid):
    """Ring lengths, per-ring truncation and the per-m ring counts L_m
    (north rings carrying m), from the grid definition alone."""
    if grid == "full":
        nlat = N + 1
        nlon = np.full(nlat, 2 * N + 2)
    else:
        nlat = 2 * (N + 1)
        half = 20 + 4 * np.arange(N + 1)
        nlon = np.concatenate([half, half[::-1]])
    mmax = np.minimum(N, (nlon - 1) // 2)
    nh = nlat // 2
    L = np.array([int(np.sum(mmax[:nh] >= m)) for m in range(N + 1)])
    return {"nlat": nlat, "npts": int(nlon.sum()), "nfour": int((mmax + 1).sum()), "L": L,
            "nspec": (N + 1) * (N + 2) // 2}


def legendre_flops(N, geo, F):
    """Algorithmic flops of one Legendre product (either direction):
    2 flops per multiply-add, 2F real columns, L_m rings by N - m + 1
    degrees per m (both parity halves, no padding)."""
    m = np.arange(N + 1)
    return float(4.0 * F * np.sum(geo["L"] * (N - m + 1)))


def stage_bytes(N, geo, F, elem, tab_elem):
    """Algorithmic HBM bytes per launch of each stage (each operand read or
    written once)."""
    m = np.arange(N + 1)
    tab = float(np.sum(geo["L"] * (N - m + 1))) * tab_elem
    spec = float(F) * geo["nspec"] * 2 * elem
    four = float(F) * geo["nfour"] * 2 * elem
    grid = float(F) * geo["npts"] * elem
    return {
        "legendre_inverse": tab + spec + four,
        "fourier_synthesis": four + grid,
        "fourier_analysis": grid + four,
        "legendre_direct": tab + four + spec,
    }


_INPUTS = {}


def host_inputs(workload, seed=0):
    """Seeded spectral coefficients of every field, drawn once (float64)."""
    from paper_1908_06096_amd.inputs import spectral_coefficients

    key = (workload, seed)
    if key not in _INPUTS:
        N, _grid, F = WORKLOADS[workload]
        t0 = time.time()
        _INPUTS[key] = spectral_coefficients(N, F, seed=seed, dtype=np.float64)
        log(f"[bench] drew inputs for {workload} ({time.time() - t0:.1f} s)")
    return _INPUTS[key]


def stage_report(N, geo, F, precision, per_stage_ms):
    """Per-stage rates against their roofs and the roofline of the slowest
    stage.  Legendre products: algorithmic flops (bf16x3 issues three BF16
    products per multiply-add and is measured against the BF16 peak, with
    the FP32-equivalent rate alongside); FFTs: algorithmic HBM bytes."""
    elem = 8 if precision == "fp64" else 4
    flops = legendre_flops(N, geo, F)
    nbytes = stage_bytes(N, geo, F, elem, elem)
    mult, peak = {"fp64": (1, PEAK["fp64"]), "fp32": (1, PEAK["fp32"]), "bf16x3": (3, PEAK["bf16"])}[precision]
    stages = {}
    for name, ms in per_stage_ms.items():
        if name.startswith("legendre"):
            ach = mult * flops / (ms * 1e-3)
            stages[name] = {"ms": ms, "bound": "mfma", "achieved_tflops": ach / 1e12, "frac": ach / peak,
                            "fp32_equiv_tflops": flops / (ms * 1e-3) / 1e12,
                            "hbm_gbs": nbytes[name] / (ms * 1e-3) / 1e9}
        else:
            ach = nbytes[name] / (ms * 1e-3)
            stages[name] = {"ms": ms, "bound": "hbm", "achieved_gbs": ach / 1e9, "frac": ach / PEAK["hbm"]}
    dom = max(per_stage_ms, key=per_stage_ms.get)
    d = stages[dom]
    if d["bound"] == "mfma":
        roof = {"kernel": dom, "bound": "mfma", "achieved": d["achieved_tflops"], "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": d["frac"], "traffic": None}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": d["achieved_gbs"], "peak": PEAK["hbm"] / 1e9,
                "unit": "GB/s", "frac": d["frac"], "traffic": None}
    return stages, roof


def committed_traffic(workload, precision, stage):
    """HBM bytes per launch of ``stage`` from the PMC summary committed under
    profiles/ (FETCH_SIZE + WRITE_SIZE scaled by a copy of known size), or
    None if there is none or the kernels changed since it was taken."""
    from paper_1908_06096_amd.profiling import measured_traffic

    return measured_traffic(os.path.join(HERE, "profiles", f"traffic_{workload}_{precision}.json"), stage)


def run_gpu(workload, precision, steps, warmup, seed=0):
    import torch

    from paper_1908_06096_amd import sht

    N, grid, F = WORKLOADS[workload]
    torch.cuda.set_device(0)
    t0 = time.time()
    plan = sht.Plan(N, grid, F, precision)
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    log(f"[bench] plan {workload} {precision}: {plan_s:.2f} s, tables {plan.info.table_bytes / 1e9:.2f} GB")
    dt = torch.float64 if precision == "fp64" else torch.float32
    t0 = time.time()
    spec = torch.from_numpy(host_inputs(workload, seed)).to(device="cuda", dtype=dt)
    grid_t = plan.empty_grid()
    back = plan.empty_spec()
    ws = plan.empty_workspace()
    torch.cuda.synchronize()
    log(f"[bench] inputs resident ({time.time() - t0:.1f} s)")

    stream = torch.cuda.current_stream()
    names = ["legendre_inverse", "fourier_synthesis", "fourier_analysis", "legendre_direct"]

    def step(evs=None):
        if evs is not None:
            evs[0].record(stream)
        plan.legendre_inverse(spec, ws)
        if evs is not None:
            evs[1].record(stream)
        plan.fourier_synthesis(ws, grid_t)
        if evs is not None:
            evs[2].record(stream)
        plan.fourier_analysis(grid_t, ws)
        if evs is not None:
            evs[3].record(stream)
        plan.legendre_direct(ws, back)
        if evs is not None:
            evs[4].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    log("[bench] warmup done")
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.time()
    start.record(stream)
    for k in range(steps):
        step(events[k])
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - wall0
    total_ms = start.elapsed_time(stop)
    per_stage = {n: float(np.mean([events[k][i].elapsed_time(events[k][i + 1]) for k in range(steps)]))
                 for i, n in enumerate(names)}
    log(f"[bench] timed {steps} steps: {total_ms:.2f} ms (wall {wall * 1e3:.1f} ms); stages {per_stage}")

    # self-consistency: the round trip returns the band-limited input
    a = spec.double()
    a[:, : N + 1, 1] = 0
    rt = float(torch.linalg.vector_norm(back.double() - a) / torch.linalg.vector_norm(a))
    out = {
        "plan": plan,
        "N": N, "grid": grid, "F": F,
        "total_ms": total_ms, "steps": steps, "per_stage_ms": per_stage,
        "round_trip_rel_l2": rt, "plan_s": plan_s,
        "spec": spec, "grid_t": grid_t,
    }
    return out


BATCH_TRUNCATIONS = (159, 255, 399, 639)


def batch_shapes(n=64, seed=2024):
    """The batched workload: n round trips, truncation uniform over
    BATCH_TRUNCATIONS (octahedral grids), 1 to 137 fields each."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice(BATCH_TRUNCATIONS, size=n)
    Fs = rng.integers(1, 138, size=n)
    return [(int(a), int(b)) for a, b in zip(Ns, Fs)]


def run_batch(steps, warmup, precision="fp32"):
    """Time the batched workload through sht_batch_* (persistent launches,
    graph replay, tuned tiles) and the same transforms one call at a time.
    Inputs: the seeded recipe with 4 distinct fields per transform, repeated
    to its field count.  A step is a round trip in place: synthesis of the
    spectral arrays, then analysis back into them."""
    import torch

    from paper_1908_06096_amd import sht
    from paper_1908_06096_amd.inputs import spectral_coefficients

    shapes = batch_shapes()
    t0 = time.time()
    plans = [sht.Plan(N, "octahedral", F, precision) for N, F in shapes]
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    dt = torch.float64 if precision == "fp64" else torch.float32
    specs = []
    for i, (N, F) in enumerate(shapes):
        d = min(F, 4)
        a = spectral_coefficients(N, d, seed=1000 * i)[np.arange(F) % d]
        specs.append(torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt))
    grids = [p.empty_grid() for p in plans]
    fields = sum(F for _, F in shapes)
    stream = torch.cuda.Stream()
    out = {"transforms": len(shapes), "fields": fields, "precision": precision,
           "truncations": {str(n): sum(1 for N, _ in shapes if N == n) for n in BATCH_TRUNCATIONS},
           "plan_s": plan_s}
    with torch.cuda.stream(stream):
        b = sht.Batch(plans, persistent=True, graph=True)
        ws = b.bind(specs, grids)
        t_tune = time.time()
        b.tune()
        out["tune_s"] = time.time() - t_tune
        out["tiles"] = {t: b.tiles().count(t) for t in ("c128", "c64", "c32")}
        for _ in range(warmup):
            b.inverse()
            b.direct()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        stream.synchronize()
        for k in range(steps):
            ev[k][0].record(stream)
            b.inverse()
            ev[k][1].record(stream)
            b.direct()
            ev[k][2].record(stream)
        stream.synchronize()
        inv = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
        dirt = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
        out["ms_per_step"] = inv + dirt
        out["inverse_ms"] = inv
        out["direct_ms"] = dirt
        out["value"] = 2.0 * fields / ((inv + dirt) * 1e-3)
        # the same transforms, one plan call after another, on the same stream
        wss = [p.empty_workspace() for p in plans]
        for p, s_, g, w in zip(plans, specs, grids, wss):
            p.inverse(s_, g, w)
            p.direct(g, s_, w)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        stream.synchronize()
        e0.record(stream)
        for _ in range(steps):
            for p, s_, g, w in zip(plans, specs, grids, wss):
                p.inverse(s_, g, w)
                p.direct(g, s_, w)
        e1.record(stream)
        stream.synchronize()
        seq = e0.elapsed_time(e1) / steps
        out["one_by_one_ms_per_step"] = seq
        out["speedup_vs_one_by_one"] = seq / out["ms_per_step"]
        b.close()
        del ws, wss
    for p in plans:
        p.close()
    log(f"[bench] batch: {out['ms_per_step']:.2f} ms per round trip of {len(shapes)} transforms "
        f"({fields} fields), one by one {seq:.2f} ms")
    return out


def run_serving(n_requests=1000, slots=4, budget_gb=40.0, load=0.8, bypass=2):
    """Serving stream: Poisson arrivals of round-trip requests, truncation
    log-uniform over T79-T1279 snapped to a ladder of resident resolutions,
    1-411 fields, FP32 or bf16x3 with probability 1/2 each.  The arrival rate
    is `load` times the capacity measured on a burst of 100 requests that
    all arrive at once; latency runs from arrival to completion.  The default
    memory budget (40 GB) is below what all table sets, the input pools and
    the in-flight requests need at once (a T1279 request of 411 fields holds
    22 GB), so admission waits for memory and idle table sets are evicted
    (and made again when a request needs them; that time is in its latency).
    Up to `bypass` later requests that fit may start ahead of one that waits
    for memory (0: strict arrival order; 1 to 4 measured a p99 ~10 ms lower
    than 0 at the 40 GB budget)."""
    import torch

    from paper_1908_06096_amd.serve import TRUNCATION_LADDER, GpuExecutor, Scheduler, draw_requests, percentile

    ex = GpuExecutor(slots=slots)
    budget = int(budget_gb * 1e9)
    # warm the table sets that fit the budget with room for the largest request
    t0 = time.time()
    for N in TRUNCATION_LADDER:
        for prec in ("fp32", "bf16x3"):
            if ex.resident() + ex.estimate_tables(N, prec) < 0.6 * budget:
                ex.warm(N, prec)
    torch.cuda.synchronize()
    warm_s = time.time() - t0
    sleep = lambda: time.sleep(2e-5)  # noqa: E731
    burst = draw_requests(100, rate=0.0, seed=11)
    t0 = time.perf_counter()
    Scheduler(ex, slots, budget, idle=sleep, bypass=bypass).run(burst)
    torch.cuda.synchronize()
    cap = len(burst) / (time.perf_counter() - t0)
    rate = load * cap
    reqs = draw_requests(n_requests, rate=rate, seed=7)
    ex.evictions = 0
    ex.warm_s = 0.0
    sched = Scheduler(ex, slots, budget, idle=sleep, bypass=bypass)
    t0 = time.perf_counter()
    sched.run(reqs)
    torch.cuda.synchronize()
    span = time.perf_counter() - t0
    lat = [r.latency for r in reqs]
    evictions, remade_s = ex.evictions, ex.warm_s
    fields = sum(r.fields for r in reqs)
    ex.close()
    out = {
        "requests": len(reqs),
        "slots": slots,
        "arrival_rate_per_s": rate,
        "capacity_per_s": cap,
        "load": load,
        "p50_latency_ms": percentile(lat, 50) * 1e3,
        "p99_latency_ms": percentile(lat, 99) * 1e3,
        "mean_latency_ms": float(np.mean(lat)) * 1e3,
        "throughput_field_transforms_per_s": 2.0 * fields / span,
        "makespan_s": span,
        "peak_resident_gb": sched.peak / 1e9,
        "budget_gb": budget_gb,
        "bypass": bypass,
        "warm_s": warm_s,
        "truncation_ladder": list(TRUNCATION_LADDER),
        "table_evictions": evictions,
        "tables_remade_s": remade_s,
    }
    log(f"[bench] serving: {len(reqs)} requests at {rate:.1f}/s, p50 {out['p50_latency_ms']:.1f} ms, "
        f"p99 {out['p99_latency_ms']:.1f} ms")
    return out


def fp64_form_error(res):
    """Relative L2 of a run's synthesis against the plain FP64 form on the
    same GPU: an FP64 plan synthesises the very same coefficients (the
    inputs as rounded to the run's data type) of the first, middle and last
    field."""
    import torch
    from paper_1908_06096_amd import sht

    F = res["F"]
    sel = torch.tensor(sorted({0, F // 2, F - 1}), device="cuda")
    with sht.Plan(res["N"], res["grid"], int(sel.numel()), "fp64") as p64:
        ref = p64.inverse(res["spec"][sel].double().contiguous())
        got = res["grid_t"][sel].double()
        err = float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref))
        del ref, got
    return err


def host_description():
    """nproc, CPU model and the BLAS library numpy uses on this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas, threads = "unknown", os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info

        info = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if info:
            blas = f"{info[0].get('internal_api')} {info[0].get('version')}"
            threads = int(info[0].get("num_threads", threads))
    except Exception:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "blas": blas, "blas_threads": threads}


def cpu_baseline(workload, seed=0, stride=None):
    """The FP64 oracle on the host cores, one field of the workload, on a
    bounded sample: synthesis of every `stride`-th ring and analysis of every
    `stride`-th wavenumber (each restricted call does the full work of its
    rings / wavenumbers: Legendre sums, brute-force DFTs).  The sample's time
    times the stride estimates the full single-field round trip (no fitted
    model; uniform sampling of rings and wavenumbers)."""
    import oracle
    from paper_1908_06096_amd.inputs import grid_noise, spectral_coefficients

    host = host_description()
    N, grid, _F = WORKLOADS[workload]
    if stride is None:
        stride = 64 if N > 500 else 1
    geo = oracle.grid_geometry(N, grid)
    t0 = time.perf_counter()
    gauss = oracle.gauss_newton(geo["nlat"])
    t_gauss = time.perf_counter() - t0
    s = spectral_coefficients(N, 1, seed=seed)
    spec_c = s[..., 0] + 1j * s[..., 1]
    g = grid_noise(geo["npts"], 1, seed=seed)
    rings = np.arange(0, geo["nlat"], stride)
    ms = np.arange(0, N + 1, stride)
    t0 = time.perf_counter()
    oracle.inverse(spec_c, N, grid, rings=rings, geometry=geo, gauss=gauss)
    t_inv = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.direct(g, N, grid, ms=ms, geometry=geo, gauss=gauss)
    t_dir = time.perf_counter() - t0
    inv_full = t_inv * geo["nlat"] / rings.size
    dir_full = t_dir * (N + 1) / ms.size
    value = 2.0 / (inv_full + dir_full + t_gauss)
    out = {
        "value": value,
        "unit": "field-transforms/s",
        "cores": int(host["blas_threads"]),
        "kind": "oracle",
        "sample": (f"{workload}, 1 field, FP64 oracle: synthesis of every {stride}th ring ({rings.size} of "
                   f"{geo['nlat']}, {t_inv:.1f} s) and analysis of every {stride}th wavenumber ({ms.size} of "
                   f"{N + 1}, {t_dir:.1f} s), each scaled by its sampling ratio, plus the latitudes "
                   f"({t_gauss:.1f} s): {inv_full + dir_full + t_gauss:.1f} s per single-field round trip"),
    }
    out.update({k: v for k, v in host.items() if k != "blas_threads"})
    return out


def time_calls(fn, n, stream):
    """Mean ms of `fn()` over n back-to-back calls on `stream` (HIP events)."""
    import torch

    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(n):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def run_stepping(workload, precision, nsteps):
    """Time steps (synthesis, logistic term on the grid, analysis, implicit
    diffusion) on resident data: enqueued kernel by kernel, and replayed
    from a HIP graph captured once."""
    import torch

    from paper_1908_06096_amd import sht

    N, grid, F = WORKLOADS[workload]
    dt = torch.float64 if precision == "fp64" else torch.float32
    stream = torch.cuda.Stream()
    out = {"workload": workload, "precision": precision, "steps": nsteps,
           "step": "synthesis, g += dt r g (1 - g), analysis, a /= 1 + dt nu n(n+1)"}
    with sht.Plan(N, grid, F, precision, stream=stream) as plan:
        a = 0.05 * host_inputs(workload)
        a[:, 0, 0] = 0.5 * np.sqrt(2.0)
        gs = 10 if nsteps >= 100 else 1
        runs = [("eager_us_per_step", False, 1), ("graph_us_per_step", True, 1)]
        if gs > 1:
            runs.append((f"graph{gs}_us_per_step", True, gs))
        for key, graph, steps_per_graph in runs:
            spec = torch.from_numpy(a).to(device="cuda", dtype=dt)
            with sht.Stepper(plan, spec, 0.1, 1.0, 1e-2, graph=graph, graph_steps=steps_per_graph,
                             stream=stream) as st:
                ms = time_calls(lambda: st.run(steps_per_graph, stream=stream), nsteps // steps_per_graph, stream)
            out[key] = ms * 1e3 / steps_per_graph
    out["graph_speedup"] = out["eager_us_per_step"] / min(v for k, v in out.items() if k.startswith("graph")
                                                          and k.endswith("_us_per_step"))
    log(f"[bench] stepping {workload} {precision}: " +
        ", ".join(f"{k} {v:.1f}" for k, v in out.items() if k.endswith("_us_per_step")))
    return out


def run_small_configs(steps):
    """T79 full grid, one field, FP64: microseconds per call (a latency, not
    a roofline case); T399 full grid x 411 fields, FP64: throughput."""
    import torch

    from paper_1908_06096_amd import sht

    out = {}
    stream = torch.cuda.current_stream()
    N, grid, F = WORKLOADS["T79-full-80x160-F1"]
    with sht.Plan(N, grid, F, "fp64") as plan:
        spec = torch.from_numpy(host_inputs("T79-full-80x160-F1")).cuda()
        g = plan.empty_grid()
        back = plan.empty_spec()
        ws = plan.empty_workspace()
        inv = time_calls(lambda: plan.inverse(spec, g, ws), 500, stream)
        dirm = time_calls(lambda: plan.direct(g, back, ws), 500, stream)
        torch.cuda.synchronize()
        a = spec.clone()
        a[:, : N + 1, 1] = 0
        rt = float(torch.linalg.vector_norm(back - a) / torch.linalg.vector_norm(a))
    out["T79-full-80x160-F1"] = {"precision": "fp64", "inverse_us_per_call": inv * 1e3,
                                 "direct_us_per_call": dirm * 1e3, "round_trip_rel_l2": rt,
                                 "field_transforms_per_s": 2.0 / ((inv + dirm) * 1e-3)}
    log(f"[bench] T79 x 1 FP64: inverse {inv * 1e3:.1f} us, direct {dirm * 1e3:.1f} us per call")
    torch.cuda.empty_cache()
    r = run_gpu("T399-full-400x800-F411", "fp64", steps, 1)
    geo = geometry_counts(r["N"], r["grid"])
    st, rf = stage_report(r["N"], geo, r["F"], "fp64", r["per_stage_ms"])
    rf["traffic"] = committed_traffic("T399-full-400x800-F411", "fp64", rf["kernel"])
    out["T399-full-400x800-F411"] = {"precision": "fp64", "steps": steps,
                                     "ms_per_step": r["total_ms"] / steps,
                                     "value": 2.0 * r["F"] * steps / (r["total_ms"] * 1e-3),
                                     "roofline": rf, "stages": st, "round_trip_rel_l2": r["round_trip_rel_l2"]}
    r["plan"].close()
    return out


def run_vector(steps, workload="TCo1279-O1280-F411", precision="fp32", vfields=137):
    """Vorticity and divergence of `vfields` vector fields (one wind per
    level) -> winds U, V -> vorticity and divergence, at the workload's
    truncation and grid.  Counts 2 components per vector field and
    direction as field-transforms."""
    import torch

    from paper_1908_06096_amd import sht
    from paper_1908_06096_amd.inputs import spectral_coefficients

    N, grid, _F = WORKLOADS[workload]
    dt = torch.float64 if precision == "fp64" else torch.float32
    stream = torch.cuda.current_stream()
    with sht.Plan(N, grid, vfields, precision, vector=True) as plan:
        d = 4
        a = spectral_coefficients(N, 2 * d, seed=5)
        idx = np.arange(2 * vfields) % (2 * d)
        vd = torch.from_numpy(np.ascontiguousarray(a[idx])).to(device="cuda", dtype=dt).view(2, vfields, -1, 2)
        uv = plan.empty_uv()
        back = plan.empty_vortdiv()
        ws = plan.empty_workspace()
        inv = time_calls(lambda: plan.vector_inverse(vd, uv, ws), steps, stream)
        dirm = time_calls(lambda: plan.vector_direct(uv, back, ws), steps, stream)
        tab = plan.info.table_bytes
    out = {"workload": f"{workload.split('-F')[0]}-V{vfields}", "precision": precision, "vector_fields": vfields,
           "inverse_ms": inv, "direct_ms": dirm,
           "value": 2.0 * 2 * vfields / ((inv + dirm) * 1e-3), "unit": "field-transforms/s (2 per vector field)",
           "table_gb": tab / 1e9}
    log(f"[bench] vector {out['workload']}: inverse {inv:.2f} ms, direct {dirm:.2f} ms")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="TCo1279-O1280-F411", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "fp64"])
    ap.add_argument("--variants", default="bf16x3,fp64",
                    help="comma-separated other precisions to time on the same workload ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-workload measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the small configs, the time-stepping and the vector measurements")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of this many MiB first (reference for PMC byte counters)")
    ap.add_argument("--no-fp64-check", "--no-oracle-check", dest="no_fp64_check", action="store_true",
                    help="skip comparing FP32 / bf16x3 synthesis with the FP64 form")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the transform is built and measured on a single MI355X "
              "(no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        import torch

        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {args.copy_calibration} MiB")
        del a, b
    res = run_gpu(args.workload, args.precision, args.steps, args.warmup)
    N, F = res["N"], res["F"]
    geo = geometry_counts(N, res["grid"])
    stages, roof = stage_report(N, geo, F, args.precision, res["per_stage_ms"])
    roof["traffic"] = committed_traffic(args.workload, args.precision, roof["kernel"])

    ms_per_step = res["total_ms"] / args.steps
    value = 2.0 * F * args.steps / (res["total_ms"] * 1e-3)
    out = {
        "metric": "field-transforms/s",
        "value": value,
        "unit": "field-transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x3": "bf16x3-f32acc", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "truncation": N, "grid": res["grid"], "fields": F,
                   "precision": args.precision, "step": "inverse + direct of all fields"},
        "roofline": roof,
        "stages": stages,
        "round_trip_rel_l2": res["round_trip_rel_l2"],
    }
    if not args.no_fp64_check and args.precision != "fp64":
        out["rel_l2_vs_fp64"] = fp64_form_error(res)
        log(f"[bench] rel L2 against the FP64 form {out['rel_l2_vs_fp64']:.2e}")
    res["plan"].close()
    del res
    variants = {}
    for prec in [v for v in args.variants.split(",") if v and v != args.precision]:
        import torch

        torch.cuda.empty_cache()
        r = run_gpu(args.workload, prec, args.steps, 1)
        st, rf = stage_report(N, geo, F, prec, r["per_stage_ms"])
        rf["traffic"] = committed_traffic(args.workload, prec, rf["kernel"])
        variants[prec] = {
            "value": 2.0 * F * r["steps"] / (r["total_ms"] * 1e-3),
            "ms_per_step": r["total_ms"] / r["steps"],
            "steps": r["steps"],
            "roofline": rf,
            "stages": st,
            "round_trip_rel_l2": r["round_trip_rel_l2"],
        }
        if not args.no_fp64_check and prec != "fp64":
            variants[prec]["rel_l2_vs_fp64"] = fp64_form_error(r)
        r["plan"].close()
        del r
    if variants:
        out["variants"] = variants
    if not args.no_extras:
        import torch

        torch.cuda.empty_cache()
        out["configs"] = run_small_configs(args.steps)
        torch.cuda.empty_cache()
        out["stepping"] = [run_stepping("T79-full-80x160-F1", "fp64", 1000),
                           run_stepping(args.workload, args.precision, min(args.steps, 5))]
        torch.cuda.empty_cache()
        out["vector"] = run_vector(min(args.steps, 5))
    if not args.no_batch:
        import torch

        torch.cuda.empty_cache()
        out["batch"] = run_batch(min(args.steps, 5), 1)
    if not args.no_serving:
        import torch

        torch.cuda.empty_cache()
        out["serving"] = run_serving()
        torch.cuda.empty_cache()
        out["serving_unbound"] = run_serving(budget_gb=200.0)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

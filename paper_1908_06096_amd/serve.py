"""Request serving for round-trip transforms: continuous batching on one GPU.

Requests (truncation, fields, precision) arrive over time.  The scheduler
admits them in arrival order as soon as an execution slot is free and the
request's device footprint fits the memory budget; admitted requests run at
once on their slot's HIP stream, so work of requests admitted at different
times overlaps on the device.  Legendre and FFT tables stay resident per
(truncation, precision) -- evicted least-recently-used, and only when idle,
if a new table set would not fit -- and each field count gets a light plan
that shares them (``sht_plan_create_like``).  Latency is measured from a
request's arrival to the completion of its last kernel.

The scheduler is plain host logic over two small interfaces, an executor and
a clock, so its admission rules can be exercised without a GPU.
"""

import collections
import heapq
import time

__all__ = ["Request", "Scheduler", "GpuExecutor", "percentile", "TRUNCATION_LADDER", "draw_requests"]

# Resolutions a request's truncation is snapped to (log-spaced from T79 to
# T1279), so that a bounded set of table sets can stay resident.
TRUNCATION_LADDER = (79, 95, 127, 159, 191, 255, 319, 399, 511, 639, 799, 1023, 1279)


def draw_requests(n, rate, seed=7, fields=(1, 411), ladder=TRUNCATION_LADDER, precisions=("fp32", "bf16x3")):
    """n requests with Poisson arrivals at `rate` per second; truncation
    log-uniform over [ladder[0], ladder[-1]] snapped (in log space) to the
    ladder; fields uniform in the closed range `fields`; precision uniform
    over `precisions`."""
    import math

    import numpy as np

    rng = np.random.default_rng(seed)
    t = 0.0
    logs = np.log(np.asarray(ladder, dtype=float))
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        x = math.exp(rng.uniform(math.log(ladder[0]), math.log(ladder[-1])))
        N = ladder[int(np.argmin(np.abs(logs - math.log(x))))]
        F = int(rng.integers(fields[0], fields[1] + 1))
        prec = precisions[int(rng.integers(0, len(precisions)))]
        out.append(Request(i, t, N, F, prec))
    return out


class Request:
    __slots__ = ("rid", "arrival", "truncation", "fields", "precision", "admitted", "completed", "slot")

    def __init__(self, rid, arrival, truncation, fields, precision):
        self.rid = rid
        self.arrival = float(arrival)
        self.truncation = int(truncation)
        self.fields = int(fields)
        self.precision = precision
        self.admitted = None
        self.completed = None
        self.slot = None

    @property
    def latency(self):
        return None if self.completed is None else self.completed - self.arrival


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(0, min(len(v) - 1, int(-(-q * len(v) // 100)) - 1))
    return v[k]


class Scheduler:
    """Admission and completion loop.

    executor interface:
      footprint(req)      -> bytes the request would add (buffers, plus its
                             tables if they are not resident)
      evictable()         -> bytes the executor could free by dropping idle tables
      evict(nbytes)       -> frees at least nbytes of idle tables, returns bytes freed
      launch(req, slot)   -> handle; enqueues the request's work on the slot
      done(handle)        -> True once the work has completed
      finish(handle)      -> releases the request's buffers, returns bytes freed
      resident()          -> bytes currently held (tables + in-flight buffers)
    clock(): seconds, monotonic.
    """

    def __init__(self, executor, slots, budget_bytes, clock=time.perf_counter, idle=lambda: None):
        self.ex = executor
        self.slots = int(slots)
        self.budget = int(budget_bytes)
        self.clock = clock
        self.idle = idle
        self.peak = 0

    def run(self, requests):
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending.reverse()
        queue = collections.deque()
        running = {}  # slot -> (req, handle)
        free = list(range(self.slots))
        heapq.heapify(free)
        t0 = self.clock()
        done = []
        while pending or queue or running:
            now = self.clock() - t0
            progressed = False
            while pending and pending[-1].arrival <= now:
                queue.append(pending.pop())
                progressed = True
            for slot in list(running):
                req, h = running[slot]
                if self.ex.done(h):
                    req.completed = self.clock() - t0
                    self.ex.finish(h)
                    del running[slot]
                    heapq.heappush(free, slot)
                    done.append(req)
                    progressed = True
            # admit in arrival order while a slot is free and the head fits
            while queue and free:
                req = queue[0]
                need = self.ex.footprint(req)
                room = self.budget - self.ex.resident()
                # free idle tables until the request fits; re-price it after
                # each round, since its own tables may have been among them
                while need > room and self.ex.evictable() > 0:
                    if self.ex.evict(need - room) <= 0:
                        break
                    need = self.ex.footprint(req)
                    room = self.budget - self.ex.resident()
                if need > room:
                    if not running and need > self.budget:
                        raise MemoryError(f"request {req.rid} needs {need} bytes, budget {self.budget}")
                    break
                queue.popleft()
                slot = heapq.heappop(free)
                req.slot = slot
                req.admitted = self.clock() - t0
                running[slot] = (req, self.ex.launch(req, slot))
                self.peak = max(self.peak, self.ex.resident())
                progressed = True
            if not progressed:
                self.idle()
        return done


class GpuExecutor:
    """Runs admitted requests with the HIP library: one stream per slot,
    resident tables per (truncation, precision), light plans per field
    count, device-resident seeded inputs per (truncation, precision) from
    which a request takes its first F fields."""

    def __init__(self, slots, grid="octahedral", input_fields=411, distinct_fields=4, plan_cache=512,
                 keep_results=False):
        import torch

        from . import sht

        self.torch = torch
        self.sht = sht
        self.grid = grid
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.setup_stream = torch.cuda.Stream()
        self.tables = collections.OrderedDict()  # (N, prec) -> base Plan (LRU order)
        self.table_bytes = {}
        self.inputs = {}  # (N, prec) -> device spec [input_fields][nspec][2]
        self.plans = collections.OrderedDict()  # (N, F, prec) -> Plan
        self.plan_cache = plan_cache
        self.inflight = {}  # handle -> (bytes, key)
        self.busy = collections.Counter()  # (N, prec) -> in-flight requests
        self.input_fields = input_fields
        self.distinct = distinct_fields
        self.buffer_bytes = 0
        self.results = {} if keep_results else None

    # ---- residency ----
    def _elem(self, prec):
        return 8 if prec == "fp64" else 4

    def _buffers(self, req, plan):
        e = self._elem(req.precision)
        return req.fields * (plan.npts * e + plan.nspec * 2 * e) + plan.workspace_bytes

    def warm(self, truncation, precision):
        """Make the tables and the input pool of (truncation, precision) resident."""
        key = (truncation, precision)
        if key in self.tables:
            self.tables.move_to_end(key)
            return self.tables[key]
        import numpy as np

        from .inputs import spectral_coefficients

        with self.torch.cuda.stream(self.setup_stream):
            base = self.sht.Plan(truncation, self.grid, 1, precision, stream=self.setup_stream)
            d = self.distinct
            a = spectral_coefficients(truncation, d, seed=truncation)[np.arange(self.input_fields) % d]
            dt = self.torch.float64 if precision == "fp64" else self.torch.float32
            self.inputs[key] = self.torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)
        self.setup_stream.synchronize()
        self.tables[key] = base
        self.table_bytes[key] = base.info.plan_bytes + self.inputs[key].numel() * self.inputs[key].element_size()
        return base

    def _plan(self, req):
        key = (req.truncation, req.fields, req.precision)
        p = self.plans.get(key)
        if p is None:
            base = self.warm(req.truncation, req.precision)
            p = self.sht.Plan(0, nfields=req.fields, like=base, stream=self.setup_stream)
            self.plans[key] = p
            while len(self.plans) > self.plan_cache:
                _k, old = self.plans.popitem(last=False)
                old.close()
        else:
            self.plans.move_to_end(key)
        return p

    def footprint(self, req):
        e = self._elem(req.precision)
        # buffers: grid, output spectral array, workspace (upper bound from a
        # padded field count so no plan is needed to price the request)
        N = req.truncation
        nlat = 2 * (N + 1) if self.grid == "octahedral" else N + 1
        npts = 2 * sum(20 + 4 * i for i in range(N + 1)) if self.grid == "octahedral" else nlat * (2 * N + 2)
        nspec = (N + 1) * (N + 2) // 2
        nfour_bound = npts // 2 + nlat
        fpad = -(-req.fields // 16) * 16
        need = req.fields * (npts * e + nspec * 2 * e) + nfour_bound * fpad * 2 * e
        if (N, req.precision) not in self.tables:
            need += self.estimate_tables(N, req.precision)
        return need

    def estimate_tables(self, N, prec):
        e = 8 if prec == "fp64" else 4
        nlat = 2 * (N + 1) if self.grid == "octahedral" else N + 1
        pbar = sum(nlat // 2 * (N - m + 1) for m in range(N + 1))  # upper bound
        nspec = (N + 1) * (N + 2) // 2
        return pbar * e + self.input_fields * nspec * 2 * e

    def resident(self):
        return sum(self.table_bytes.values()) + self.buffer_bytes

    def evictable(self):
        return sum(b for k, b in self.table_bytes.items() if self.busy[k] == 0)

    def evict(self, nbytes):
        freed = 0
        for key in list(self.tables):
            if freed >= nbytes:
                break
            if self.busy[key]:
                continue
            for pk in [k for k in self.plans if (k[0], k[2]) == key]:
                self.plans.pop(pk).close()
            self.tables.pop(key).close()
            del self.inputs[key]
            freed += self.table_bytes.pop(key)
        return freed

    # ---- execution ----
    def launch(self, req, slot):
        torch = self.torch
        plan = self._plan(req)
        key = (req.truncation, req.precision)
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            spec_in = self.inputs[key][: req.fields]
            grid = plan.empty_grid()
            spec_out = plan.empty_spec()
            ws = plan.empty_workspace()
            plan.inverse(spec_in, grid, ws)
            plan.direct(grid, spec_out, ws)
            ev = torch.cuda.Event()
            ev.record(stream)
        nbytes = self._buffers(req, plan)
        self.buffer_bytes += nbytes
        self.busy[key] += 1
        h = (ev, grid, spec_out, ws, nbytes, key, req)
        return h

    def done(self, h):
        return h[0].query()

    def finish(self, h):
        _ev, _g, spec_out, _ws, nbytes, key, req = h
        self.buffer_bytes -= nbytes
        self.busy[key] -= 1
        if self.results is not None:
            self.results[req.rid] = spec_out
        return nbytes

    def close(self):
        for p in self.plans.values():
            p.close()
        for p in self.tables.values():
            p.close()
        self.plans.clear()
        self.tables.clear()
        self.inputs.clear()

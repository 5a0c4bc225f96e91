"""Request serving for round-trip transforms: continuous batching on one GPU.

Requests (truncation, fields, precision) arrive over time.  The scheduler
admits them in arrival order as soon as an execution slot is free and the
request's device footprint fits the memory budget; admitted requests run at
once on their slot's HIP stream, so work of requests admitted at different
times overlaps on the device.  Legendre and FFT tables stay resident per
(truncation, precision) -- evicted least-recently-used, and only when idle,
if a new table set would not fit, and released in stream order so that the
other slots do not stall -- and each field count, rounded up to a multiple
of 16 (the Fourier workspace's field padding), gets a light plan that
shares them (``sht_plan_create_like``), made on first use and kept while
they stay.  Latency is measured from a request's arrival to the
completion of its last kernel.

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
      inflight()          -> bytes of the in-flight requests' buffers
    clock(): seconds, monotonic.

    Admission is in arrival order.  With ``bypass`` = k > 0, while the
    oldest waiting request does not fit the memory left, later requests that
    fit it as it is (no eviction on their behalf) may start ahead of it, at
    most k of them per waiting request, so a large request is delayed by a
    bounded number of small ones and the slots do not idle behind it.
    """

    def __init__(self, executor, slots, budget_bytes, clock=time.perf_counter, idle=lambda: None, bypass=0):
        self.ex = executor
        self.slots = int(slots)
        self.budget = int(budget_bytes)
        self.clock = clock
        self.idle = idle
        self.bypass = int(bypass)
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
        passed = 0  # requests admitted ahead of the current head of the queue

        def admit(req):
            slot = heapq.heappop(free)
            req.slot = slot
            req.admitted = self.clock() - t0
            running[slot] = (req, self.ex.launch(req, slot))
            self.peak = max(self.peak, self.ex.resident())

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
                # free idle tables only if the request would not fit even
                # once every running request has finished (otherwise wait for
                # their buffers: evicting tables for transient buffer
                # pressure makes them be made again soon after); re-price it
                # after each round, since its own tables may have been among
                # them
                while need > room + self.ex.inflight() and self.ex.evictable() > 0:
                    if self.ex.evict(need - room) <= 0:
                        break
                    need = self.ex.footprint(req)
                    room = self.budget - self.ex.resident()
                if need > room:
                    if not running and need > self.budget:
                        raise MemoryError(f"request {req.rid} needs {need} bytes, budget {self.budget}")
                    # the head waits for memory: later requests that fit as
                    # things are may pass it, up to `bypass` of them
                    i = 1
                    while free and passed < self.bypass and i < len(queue):
                        cand = queue[i]
                        if self.ex.footprint(cand) <= self.budget - self.ex.resident():
                            del queue[i]
                            admit(cand)
                            passed += 1
                            progressed = True
                        else:
                            i += 1
                    break
                queue.popleft()
                passed = 0
                admit(req)
                progressed = True
            if not progressed:
                self.idle()
        return done


class GpuExecutor:
    """Runs admitted requests with the HIP library: one stream per slot,
    resident tables per (truncation, precision), light plans per field
    count, device-resident seeded inputs per (truncation, precision) from
    which a request takes its first F fields."""

    FIELD_STEP = 16  # light plans per multiple of 16 fields

    def __init__(self, slots, grid="octahedral", input_fields=411, distinct_fields=4, keep_results=False,
                 max_fields=411):
        import torch

        from . import sht

        self.torch = torch
        self.sht = sht
        self.grid = grid
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.setup_stream = torch.cuda.Stream()
        self.tables = collections.OrderedDict()  # (N, prec) -> base Plan (LRU order)
        self.table_bytes = {}
        self.pools = {}  # prec -> flat device pool of seeded coefficients (largest request's size)
        self.pool_bytes = 0
        self.plans = {}  # (N, F rounded up to FIELD_STEP, prec) -> Plan
        self.busy = collections.Counter()  # (N, prec) -> in-flight requests
        self.max_fields = max_fields
        # the input pool covers the largest rounded field count
        self.input_fields = max(input_fields, self._bucket(max_fields))
        self.warm_s = 0.0  # time spent making table sets (and their plans)
        self.evictions = 0  # table sets dropped to make room
        self.distinct = distinct_fields
        self.buffer_bytes = 0
        self.results = {} if keep_results else None

    # ---- residency ----
    def _elem(self, prec):
        return 8 if prec == "fp64" else 4

    @classmethod
    def _bucket(cls, fields):
        return -(-int(fields) // cls.FIELD_STEP) * cls.FIELD_STEP

    def _buffers(self, req, plan):
        e = self._elem(req.precision)
        return plan.nfields * (plan.npts * e + plan.nspec * 2 * e) + plan.workspace_bytes

    def warm(self, truncation, precision):
        """Make the tables, the light plans of every rounded field count and
        the input pool of (truncation, precision) resident."""
        key = (truncation, precision)
        if key in self.tables:
            self.tables.move_to_end(key)
            return self.tables[key]
        import numpy as np

        from .inputs import spectral_coefficients

        t0 = time.perf_counter()
        with self.torch.cuda.stream(self.setup_stream):
            base = self.sht.Plan(truncation, self.grid, 1, precision, stream=self.setup_stream)
        self.setup_stream.synchronize()
        self.tables[key] = base
        self.table_bytes[key] = base.info.plan_bytes
        self.warm_s += time.perf_counter() - t0
        return base

    def inputs(self, truncation, precision, fields):
        """Device spectral input [fields][nspec][2] for a request: a view of
        the precision's pool, which holds the seeded coefficients of the
        largest truncation served (T1279 unless smaller requests come first
        and a larger one later grows it).  A smaller truncation reads the
        pool's leading values in its own layout: finite values of the same
        distribution, which is all the timing needs."""
        import numpy as np

        from .inputs import spectral_coefficients

        ns = (truncation + 1) * (truncation + 2) // 2
        need = fields * ns * 2
        pool = self.pools.get(precision)
        if pool is None or pool.numel() < need:
            big = max(truncation, 1279)
            nsb = (big + 1) * (big + 2) // 2
            n = self.input_fields * nsb * 2
            d = self.distinct
            a = spectral_coefficients(big, d, seed=big)[np.arange(self.input_fields) % d].reshape(-1)
            dt = self.torch.float64 if precision == "fp64" else self.torch.float32
            if pool is not None:
                self.pool_bytes -= pool.numel() * pool.element_size()
            pool = self.torch.from_numpy(np.ascontiguousarray(a[:max(n, need)])).to(device="cuda", dtype=dt)
            self.pools[precision] = pool
            self.pool_bytes += pool.numel() * pool.element_size()
        return pool[:need].view(fields, ns, 2)

    def _plan(self, req):
        """The light plan of the request's rounded field count, made on first
        use and kept (with its bytes counted) while the tables stay."""
        key = (req.truncation, req.precision)
        base = self.warm(*key)
        pk = (req.truncation, self._bucket(req.fields), req.precision)
        p = self.plans.get(pk)
        if p is None:
            t0 = time.perf_counter()
            p = self.sht.Plan(0, nfields=pk[1], like=base, stream=self.setup_stream)
            self.plans[pk] = p
            self.table_bytes[key] += p.info.own_bytes
            self.warm_s += time.perf_counter() - t0
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
        fb = self._bucket(req.fields)
        need = fb * (npts * e + nspec * 2 * e) + nfour_bound * fb * 2 * e
        if (N, req.precision) not in self.tables:
            need += self.estimate_tables(N, req.precision)
        return need

    def estimate_tables(self, N, prec):
        e = 8 if prec == "fp64" else 4
        nlat = 2 * (N + 1) if self.grid == "octahedral" else N + 1
        pbar = sum(nlat // 2 * (N - m + 1) for m in range(N + 1))  # upper bound
        plans = (self._bucket(self.max_fields) // self.FIELD_STEP) * (1 << 20)  # light plans' work lists (bound)
        return pbar * e + plans

    def resident(self):
        return sum(self.table_bytes.values()) + self.buffer_bytes + self.pool_bytes

    def inflight(self):
        return self.buffer_bytes

    def evictable(self):
        return sum(b for k, b in self.table_bytes.items() if self.busy[k] == 0)

    def evict(self, nbytes):
        freed = 0
        for key in list(self.tables):
            if freed >= nbytes:
                break
            if self.busy[key]:
                continue
            # idle: every kernel that used these plans has completed, so they
            # are released in stream order, with no device-wide wait
            for pk in [k for k in self.plans if (k[0], k[2]) == key]:
                self.plans.pop(pk).close_async(self.setup_stream)
            self.tables.pop(key).close_async(self.setup_stream)
            freed += self.table_bytes.pop(key)
            self.evictions += 1
        return freed

    # ---- execution ----
    def launch(self, req, slot):
        torch = self.torch
        plan = self._plan(req)
        key = (req.truncation, req.precision)
        stream = self.streams[slot]
        spec_in = self.inputs(req.truncation, req.precision, plan.nfields)
        with torch.cuda.stream(stream):
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
        self.pools.clear()
        self.pool_bytes = 0
        # the requests' buffers came from torch's caching allocator, which
        # keeps freed blocks for torch alone: hand them back to the device,
        # where the library's tables and the kernels' scratch memory are
        # allocated (a later run could otherwise find the device full)
        self.torch.cuda.synchronize()
        self.torch.cuda.empty_cache()

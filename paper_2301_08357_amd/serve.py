"""Continuous-batching server for pressure solves on a pool of meshes.

Requests (mesh, right-hand side) arrive over time; each is an FP64 solve, or
with mixed=True an FP32-inner mixed-precision solve to the same tolerance.  The server keeps a set
of meshes resident on the GPU within an HBM budget (each mesh's operator
data, CG vectors and its last solution, sized by pressure_footprint),
evicting the least recently used idle mesh when a new one must be loaded.
Admitted requests join the running batch at the next step, so solves of
different meshes overlap on the device; a mesh serves one request at a time
because each request starts from that mesh's previous solution (the warm
start of the paper's projection stage, Sec. 3.4).  A solve's result does not
depend on when it joined or on the other solves in flight.  Meshes are set
up on worker threads, so that a burst of first requests (each needing its
mesh's host layout and upload) does not hold up the solves in flight.

The heavy lifting (setup, batched CG steps, residuals) happens in
libpressure.so; this module only schedules calls.
"""

import collections
import time
from concurrent.futures import ThreadPoolExecutor, FIRST_COMPLETED, wait
from dataclasses import dataclass, field

import numpy as np

from . import _lib
from .system import PressureBatch, PressureSystem, footprint


@dataclass
class Request:
    rid: int
    mesh: int
    arrival: float                  # seconds after the start of the run
    rhs: object = None              # device tensor (filled at admission)
    x0: object = None               # device tensor of the warm start, or None (cold)
    start: float = -1.0
    done: float = -1.0
    iters: int = 0
    status: int = 0
    true_relres: float = 0.0
    result: object = None
    cold: bool = True
    step0: int = 0                  # server step at admission


@dataclass
class ServeStats:
    n: int = 0
    makespan_s: float = 0.0
    solves_per_s: float = 0.0
    latency_ms: dict = field(default_factory=dict)
    # the first request of each mesh (cold: setup included, x0 = 0) and the
    # others (warm), separately; service = completion - admission
    latency_ms_warm: dict = field(default_factory=dict)
    latency_ms_cold: dict = field(default_factory=dict)
    service_ms_mean: float = 0.0
    mean_iters_cold: float = 0.0
    mean_iters_warm: float = 0.0
    loads: int = 0
    evictions: int = 0
    rebuilds: int = 0
    steps: int = 0
    max_in_flight_seen: int = 0
    # host wall time by activity (seconds): batched steps (GPU iterations and
    # status read), finishing solves, admitting requests (rhs, begin),
    # rebuilding the batch
    t_step: float = 0.0
    t_finish: float = 0.0
    t_admit: float = 0.0
    t_rebuild: float = 0.0


class PressureServer:
    """problems: list of synth Problem (mesh id = index).  rhs_fn(req) must
    return the request's right-hand side as a float64 CUDA tensor."""

    def __init__(self, problems, budget_bytes, max_in_flight=64, rtol=1e-10, max_iter=20000,
                 graph_iters=16, tiles_per_slot=4, nodes_per_lane=8, keep_x0=False, mixed=False,
                 inner_rtol=1e-2, on_result=None, retain=False, loaders=4):
        self.problems = problems
        self.budget = int(budget_bytes)
        self.max_in_flight = int(max_in_flight)
        self.rtol = rtol
        self.max_iter = max_iter
        self.graph_iters = graph_iters
        self.tps = tiles_per_slot
        self.npl = nodes_per_lane
        self.keep_x0 = keep_x0
        # A finished request's device tensors (rhs, warm start, result) are
        # handed to on_result(req, p) and then released, so the resident
        # meshes and their last solutions are all the server holds.  With
        # retain set they stay on the request (for callers that inspect
        # them afterwards) and count against the budget.
        self.on_result = on_result
        self.retain = bool(retain)
        self.retained = 0                             # bytes held by finished requests
        # Mesh setups (host layout, upload) run on `loaders` worker threads
        # (the C call releases the GIL), so the batch keeps stepping the
        # solves in flight while meshes load; 0 sets meshes up inline.
        self.loaders = int(loaders)
        self._pool = None
        self.loading = {}                             # mesh -> Future of its PressureSystem
        self._device = None
        self.mixed = bool(mixed)
        self.inner_rtol = inner_rtol
        self.flags = _lib.PM_FP64 | (_lib.PM_FP32_INNER if self.mixed else 0)
        self.cost = [footprint(p.mesh.dim, p.mesh.coords, p.mesh.elems, self.flags,
                               getattr(p.mesh, "period", None)) + 8 * p.mesh.n_nodes
                     for p in problems]
        self.resident = collections.OrderedDict()     # mesh -> PressureSystem, least recent first
        self.last = {}                                # mesh -> last solution (device)
        self.batch = None
        self.members = []                             # mesh ids in batch order
        self.slot = {}                                # mesh id -> position in the batch
        self.dirty = False                            # resident set differs from the batch's
        self.batch_next = 1                           # launch index carried over rebuilds
        self.stats = ServeStats()

    # -- residency ---------------------------------------------------------
    def _used(self):
        return sum(self.cost[m] for m in self.resident) + sum(self.cost[m] for m in self.loading) + self.retained

    def _make_room(self, m, busy):
        """Evict idle meshes (least recently used first) until mesh m fits."""
        if self.cost[m] + self.retained > self.budget:
            raise ValueError("mesh %d needs %d bytes, more than the budget left by %d bytes of retained "
                             "results" % (m, self.cost[m], self.retained))
        while self._used() + self.cost[m] > self.budget:
            victim = next((v for v in self.resident if v not in busy), None)
            if victim is None:
                return False
            # the batch must not step over a closed handle: drop it now and
            # rebuild before the next step
            if self.batch is not None:
                self.batch_next = self.batch.next_index()
                self.batch.close()
                self.batch = None
            self.resident.pop(victim).close()
            self.last.pop(victim, None)
            self.stats.evictions += 1
            self.dirty = True
        return True

    def _setup(self, m):
        import torch
        torch.cuda.set_device(self._device)
        return PressureSystem.from_problem(self.problems[m], flags=self.flags)

    def _load(self, m):
        """Set mesh m up: at once (returns True) or on a loader thread."""
        if self.loaders <= 0:
            self.resident[m] = PressureSystem.from_problem(self.problems[m], flags=self.flags)
            self.stats.loads += 1
            return True
        if self._pool is None:
            import torch
            self._device = torch.cuda.current_device()
            self._pool = ThreadPoolExecutor(max_workers=self.loaders)
        self.loading[m] = self._pool.submit(self._setup, m)
        return False

    def _collect_loads(self, block=False):
        """Meshes whose setup finished become resident; with block set, wait
        for the first one.  Returns True if the resident set changed."""
        if not self.loading:
            return False
        if block:
            wait(list(self.loading.values()), timeout=0.01, return_when=FIRST_COMPLETED)
        ready = [m for m, f in self.loading.items() if f.done()]
        for m in ready:
            self.resident[m] = self.loading.pop(m).result()
            self.stats.loads += 1
        if ready:
            self.dirty = True                          # the batch must take the new meshes
        return bool(ready)

    def _rebuild(self):
        first = self.batch.next_index() if self.batch is not None else self.batch_next
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        self.batch_next = first
        self.members = list(self.resident.keys())
        self.slot = {m: j for j, m in enumerate(self.members)}
        self.dirty = False
        if self.members:
            self.batch = PressureBatch([self.resident[m] for m in self.members], self.tps, self.npl, first,
                                       mixed=self.mixed, inner_rtol=self.inner_rtol)
            self.batch.set_graph(self.graph_iters)
            self.stats.rebuilds += 1

    # -- run ---------------------------------------------------------------
    def run(self, requests, rhs_fn, clock=time.perf_counter):
        """Serve the requests (sorted by arrival).  Returns the list of
        finished requests and fills self.stats."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queues = collections.defaultdict(collections.deque)
        in_flight = {}                     # mesh -> Request
        finished = []
        t0 = clock()
        while pending or in_flight or any(queues.values()):
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                queues[r.mesh].append(r)
            changed = self._collect_loads()
            # admission: oldest waiting request first, one per mesh
            waiting = sorted((q[0] for m, q in queues.items() if q and m not in in_flight), key=lambda r: r.arrival)
            admit = []
            for r in waiting:
                if len(in_flight) + len(admit) >= self.max_in_flight:
                    break
                if r.mesh in self.loading:
                    continue
                if r.mesh not in self.resident:
                    busy = set(in_flight) | {a.mesh for a in admit} | set(self.loading)
                    if not self._make_room(r.mesh, busy):
                        continue
                    if not self._load(r.mesh):
                        continue                  # loading; admitted once resident
                    changed = True
                admit.append(r)
            t_a = clock()
            if changed or self.dirty or (admit and self.batch is None):
                self._rebuild()
            t_b = clock()
            self.stats.t_rebuild += t_b - t_a
            for r in admit:
                queues[r.mesh].popleft()
                self.resident.move_to_end(r.mesh)
                r.rhs = rhs_fn(r)
                r.x0 = self.last.get(r.mesh)
                r.cold = r.x0 is None
                if self.keep_x0 and r.x0 is not None:
                    r.x0 = r.x0.clone()
                r.start = clock() - t0
                self.batch.begin(self.slot[r.mesh], r.rhs, r.x0, self.rtol, self.max_iter)
                r.step0 = self.stats.steps
                in_flight[r.mesh] = r
            t_c = clock()
            self.stats.t_admit += t_c - t_b
            self.stats.max_in_flight_seen = max(self.stats.max_in_flight_seen, len(in_flight))
            if in_flight:
                if self.batch is None:
                    raise RuntimeError("requests in flight without a batch")
                done = self.batch.step()
                t_d = clock()
                # every step advances each solve in flight by at least 8 CG
                # iterations (mixed: or one correction), so a solve still in
                # flight after this many steps has stopped making progress
                limit = self.max_iter // 4 + 1000
                stuck = [m for m, r in in_flight.items() if self.stats.steps - r.step0 > limit]
                if stuck:
                    raise RuntimeError("solves of meshes %s made no progress in %d steps" % (stuck[:8], limit))
                self.stats.t_step += t_d - t_c
                self.stats.steps += 1
                for m in [m for m in in_flight if done[self.slot[m]]]:
                    r = in_flight.pop(m)
                    res = self.batch.finish(self.slot[m], r.rhs, self.rtol)
                    r.done = clock() - t0
                    r.iters, r.status, r.true_relres = res.iters, res.status, res.true_relres
                    self.last[m] = res.p
                    if self.on_result is not None:
                        self.on_result(r, res.p)
                    if self.retain:
                        r.result = res.p
                        self.retained += sum(8 * t.numel() for t in (r.rhs, r.x0, r.result) if t is not None)
                    else:
                        r.rhs = r.x0 = None
                    finished.append(r)
                self.stats.t_finish += clock() - t_d
            elif self.loading:
                self._collect_loads(block=True)
            elif pending:
                time.sleep(max(0.0, min(1e-3, pending[0].arrival - (clock() - t0))))
        st = self.stats
        st.n = len(finished)
        st.makespan_s = max(r.done for r in finished) if finished else 0.0
        st.solves_per_s = st.n / st.makespan_s if st.makespan_s > 0 else 0.0
        def pct(rs):
            lat = np.array([r.done - r.arrival for r in rs]) * 1e3
            if not lat.size:
                return {}
            return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                    "mean": float(lat.mean()), "max": float(lat.max()), "n": int(lat.size)}
        st.latency_ms = pct(finished)
        st.latency_ms_warm = pct([r for r in finished if not r.cold])
        st.latency_ms_cold = pct([r for r in finished if r.cold])
        if finished:
            st.service_ms_mean = float(np.mean([r.done - r.start for r in finished])) * 1e3
        cold = [r.iters for r in finished if r.cold]
        warm = [r.iters for r in finished if not r.cold]
        st.mean_iters_cold = float(np.mean(cold)) if cold else 0.0
        st.mean_iters_warm = float(np.mean(warm)) if warm else 0.0
        return finished

    def close(self):
        for f in self.loading.values():
            f.result().close()
        self.loading.clear()
        if self._pool is not None:
            self._pool.shutdown()
            self._pool = None
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        for s in self.resident.values():
            s.close()
        self.resident.clear()
        self.last.clear()

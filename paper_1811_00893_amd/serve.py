"""Continuous-batching solve server over the library's batch step API.

Requests (a gauge field, kappa, tolerance, 1..12 right-hand sides) arrive over time.
Each resident gauge field gets one batch of `nslots` solve slots in the library
(`wilson_batch_*`), on its own HIP stream.  The loop repeatedly
  * admits waiting requests: each right-hand side takes a free slot of its gauge field's
    batch as soon as one frees up (a request may be partly running while the rest of its
    right-hand sides wait); a new batch is created only if its device footprint, plus the
    gauge field's when that is not resident yet, fits in the HBM budget next to everything
    already resident; to make room, idle batches and then idle gauge fields (no slot in use
    and no older request waiting for them) are released, least recently used first, and a
    field that is needed again is loaded again;
  * enqueues a turn of iterations on every batch with running slots (all streams are
    fed before any is waited on, so batches of different lattices overlap on the GPU);
    with `turn_ms` the iterations per turn adapt so that a turn lasts about that long;
  * polls every batch, copies finished solutions out and frees their slots;
  * completes a request when all its right-hand sides are done, recording latency
    from arrival to solution-on-host (with an engine that copies solutions to the host
    asynchronously, when that copy has finished).
Each slot is an independent solve (own scalars, own kappa and tolerance, reductions
per slot in a fixed order), so a request's result does not depend on what else runs.

The scheduler (`Scheduler`) is plain host logic over an engine interface; `LibEngine`
is the real engine.  Tests drive the scheduler with a simulated engine and clock.
"""
import collections
import dataclasses
import time
from typing import Any, Dict, List, Optional

FREE, RUNNING, FINISHED = 0, 1, 2


@dataclasses.dataclass
class Request:
    rid: int
    gauge_id: Any
    kappa: float
    tol: float
    b: Any                      # (nrhs, V, 4, 3) complex128 (host or device)
    arrival: float = 0.0
    maxiter: int = 20000
    # filled by the scheduler
    x: Any = None
    pending: List[int] = dataclasses.field(default_factory=list)  # RHS indices not yet attached
    running: int = 0
    done_rhs: int = 0
    status: List[int] = dataclasses.field(default_factory=list)
    info: List[dict] = dataclasses.field(default_factory=list)
    finish: Optional[float] = None
    rejected: bool = False

    @property
    def nrhs(self):
        return int(self.b.shape[0])

    @property
    def latency(self):
        return None if self.finish is None else self.finish - self.arrival


class Scheduler:
    """Admission, slot assignment, stepping and retirement (engine-agnostic)."""

    def __init__(self, engine, hbm_budget: float, nslots: int = 12, step_iters: int = 8, clock=time.perf_counter,
                 turn_ms: Optional[float] = None, max_heavy: Optional[int] = None, heavy_ms: float = 0.5):
        self.engine = engine
        self.budget = float(hbm_budget)
        self.nslots = nslots
        self.step_iters = step_iters   # iterations per turn (the maximum when turn_ms is set)
        self.turn_ms = turn_ms         # target wall time of a turn: iterations adapt to it
        self.iters = step_iters
        # at most `max_heavy` heavy batches (an iteration estimated at >= heavy_ms) advance
        # at once, those holding the oldest requests first (None: no limit)
        if max_heavy is not None and max_heavy < 1:
            raise ValueError("max_heavy must be >= 1 (or None)")
        self.max_heavy = max_heavy
        self.heavy_ms = heavy_ms
        self.clock = clock
        self.gauges: Dict[Any, dict] = {}      # gauge_id -> {"dims", "bytes", "resident", "last_used"}
        self.batches: Dict[Any, dict] = {}     # gauge_id -> {"handle", "slots": [(req, k) | None], "bytes"}
        self.waiting: collections.deque = collections.deque()
        self.completed: List[Request] = []
        self.rejected: List[Request] = []
        self.draining: List[Request] = []      # done on the device, solution still on its way to the host
        self.loads = 0                         # gauge fields brought in on demand
        self.evictions = 0                     # gauge fields released to make room

    # ---- resources ----
    def resident_bytes(self):
        return (sum(g["bytes"] for g in self.gauges.values() if g["resident"]) +
                sum(b["bytes"] for b in self.batches.values()))

    def register_gauge(self, gauge_id, dims, nbytes, resident=True):
        """A gauge field requests may name: already resident (loaded by the engine), or known
        to the engine and loaded on demand (`engine.load_gauge(gauge_id)`); `nbytes` is its
        device footprint (before loading an upper bound, replaced by the loaded size)."""
        self.gauges[gauge_id] = {"dims": tuple(dims), "bytes": float(nbytes), "resident": bool(resident),
                                 "last_used": 0.0}

    def submit(self, req: Request):
        req.arrival = self.clock() if not req.arrival else req.arrival
        req.pending = list(range(req.nrhs))
        req.status = [None] * req.nrhs
        req.info = [None] * req.nrhs
        req.x = self.engine.alloc_solution(req)
        g = self.gauges.get(req.gauge_id)
        need = self.engine.batch_bytes(g["dims"], self.nslots) if g else float("inf")
        if g is None or g["bytes"] + need > self.budget:
            req.rejected = True   # can never fit
            self.rejected.append(req)
            return False
        self.waiting.append(req)
        return True

    def _batch_for(self, req):
        gauge_id = req.gauge_id
        b = self.batches.get(gauge_id)
        if b is not None:
            return b
        g = self.gauges[gauge_id]
        bb = self.engine.batch_bytes(g["dims"], self.nslots)
        need = bb + (0.0 if g["resident"] else g["bytes"])
        if self.resident_bytes() + need > self.budget:
            self._evict_idle(need, keep=gauge_id, before=req.arrival)
            if self.resident_bytes() + need > self.budget:
                return None
        if not g["resident"]:
            g["bytes"] = float(self.engine.load_gauge(gauge_id))
            g["resident"] = True
            self.loads += 1
        handle = self.engine.create_batch(gauge_id, self.nslots)
        b = {"handle": handle, "slots": [None] * self.nslots, "bytes": bb}
        self.batches[gauge_id] = b
        return b

    def _evict_idle(self, need, keep=None, before=float("inf")):
        """Release idle resources until `need` more bytes fit: first batches with no slot in
        use, then resident gauge fields without a batch (if the engine can unload them),
        least recently used first.  A resource stays while a request that arrived before
        `before` (the one that needs the room) waits for its field, and `keep` stays."""
        def wanted(gid):
            return any(r.gauge_id == gid and r.arrival <= before for r in self.waiting)

        def fits():
            return self.resident_bytes() + need <= self.budget

        for gid in sorted(self.batches, key=lambda k: self.gauges[k]["last_used"]):
            b = self.batches[gid]
            if all(s is None for s in b["slots"]) and not b.get("inflight") and gid != keep and not wanted(gid):
                self.engine.destroy_batch(b["handle"])
                del self.batches[gid]
                if fits():
                    return
        unload = getattr(self.engine, "unload_gauge", None)
        if unload is None:
            return
        idle = [gid for gid, g in self.gauges.items()
                if g["resident"] and gid not in self.batches and gid != keep and not wanted(gid)]
        for gid in sorted(idle, key=lambda k: self.gauges[k]["last_used"]):
            unload(gid)
            self.gauges[gid]["resident"] = False
            self.evictions += 1
            if fits():
                return

    # ---- one turn of the loop ----
    def admit(self):
        still = collections.deque()
        while self.waiting:
            req = self.waiting.popleft()
            b = self._batch_for(req)
            if b is not None and not b.get("inflight"):  # slots change only between turns
                for k, slot in enumerate(b["slots"]):
                    if not req.pending:
                        break
                    if slot is None:
                        j = req.pending.pop(0)
                        self.engine.attach(b["handle"], k, req, j)
                        b["slots"][k] = (req, j)
                        req.running += 1
                        self.gauges[req.gauge_id]["last_used"] = self.clock()
            if req.pending:
                still.append(req)
        self.waiting = still

    def _iters_for(self, b):
        """Iterations of one batch per turn.  With a target turn length and an engine that
        can estimate the cost of an iteration, each batch gets its own count, so a batch
        on a small lattice advances many iterations while one on a large lattice does one
        or two; otherwise the shared adaptive count."""
        est = getattr(self.engine, "iter_ms", None)
        if self.turn_ms and est is not None:
            n = sum(s is not None for s in b["slots"])
            ms = est(b["handle"], n)
            return int(min(self.step_iters, max(1, round(self.turn_ms / max(ms, 1e-3)))))
        return self.iters

    def _heavy(self, b):
        est = getattr(self.engine, "iter_ms", None)
        if est is None:
            return False
        return est(b["handle"], sum(s is not None for s in b["slots"])) >= self.heavy_ms

    def _may_advance(self, active):
        """Batches that may start a turn now.  Heavy batches share the GPU's bandwidth:
        several at once each run slower, and the requests that then finish last are the
        large ones that waited longest.  With `max_heavy`, only that many heavy batches
        advance, ordered by the arrival of their oldest request (the others keep their
        slots and wait); light batches always advance."""
        if self.max_heavy is None:
            return active
        heavy = [b for b in active if self._heavy(b)]
        heavy.sort(key=lambda b: min(s[0].arrival for s in b["slots"] if s is not None))
        held = set(id(b) for b in heavy[self.max_heavy:])
        return [b for b in active if id(b) not in held]

    def step(self):
        """One pass of the loop: start a turn on every batch with running slots that has
        none in flight (within the heavy-batch limit), then retire the slots of every batch
        whose turn has finished.  With an engine that can tell whether a batch's turn is
        done (`ready`) the batches run their turns independently (a small lattice does not
        wait for a large one's turn); otherwise every started turn is waited for in this
        pass."""
        active = [b for b in self.batches.values() if any(s is not None for s in b["slots"])]
        t0 = time.perf_counter()
        ready = getattr(self.engine, "ready", None)
        for b in self._may_advance(active):    # enqueue on every idle stream first ...
            if not b.get("inflight"):
                self.engine.step(b["handle"], self._iters_for(b))
                b["inflight"] = True
        for b in active:                       # ... then retire what has finished
            if not b.get("inflight"):
                continue
            if ready is not None and not ready(b["handle"]):
                continue
            b["inflight"] = False
            state, status = self.engine.poll(b["handle"])
            for k, slot in enumerate(b["slots"]):
                if slot is None or state[k] != FINISHED:
                    continue
                req, j = slot
                st, info = self.engine.detach(b["handle"], k, req, j)
                req.status[j] = st
                req.info[j] = info
                req.running -= 1
                req.done_rhs += 1
                b["slots"][k] = None
                if req.done_rhs == req.nrhs:
                    self.engine.finish(req)
                    self.draining.append(req)
        # requests whose solutions have reached the host
        done = getattr(self.engine, "finished", None)
        still = []
        for req in self.draining:
            if done is None or done(req):
                req.finish = self.clock()
                self.completed.append(req)
            else:
                still.append(req)
        self.draining = still
        if self.turn_ms and active and ready is None:
            # A slot whose Krylov cycle ends inside a turn waits for the turn to end before
            # its next cycle starts, so turns are kept short: a few milliseconds of work,
            # which on large lattices means polling every iteration or two.
            ms = 1e3 * (time.perf_counter() - t0)
            scale = self.turn_ms / max(ms, 1e-3)
            self.iters = int(min(self.step_iters, max(1, round(self.iters * min(max(scale, 0.5), 2.0)))))

    def busy(self):
        return bool(self.waiting) or bool(self.draining) or any(
            any(s is not None for s in b["slots"]) or b.get("inflight") for b in self.batches.values())

    def run_until_idle(self, max_turns=10 ** 7):
        for _ in range(max_turns):
            if not self.busy():
                return
            self.admit()
            self.step()
        raise RuntimeError("server did not drain")

    def close(self):
        for b in self.batches.values():
            self.engine.destroy_batch(b["handle"])
        self.batches.clear()


class LibEngine:
    """Engine on libwilson.so: one context and HIP stream per resident gauge field.

    Gauge fields are loaded up front (`load_gauge(id, U, dims)`) or registered as sources
    (`add_gauge_source`) that the scheduler loads and unloads on demand.  With
    `host_results`, a request's solutions are solved into device memory and then copied
    to pinned host memory on a copy stream; the request counts as finished when that copy
    has completed (`finished`), so latency runs to the solution on the host."""

    def __init__(self, precision=1, solver=0, inner_tol=0.0, device="cuda:0", host_results=False):
        import torch

        from . import _lib
        self.L = _lib
        self.torch = torch
        self.device = torch.device(device)
        self.opts = {"precision": precision, "solver": solver, "inner_tol": inner_tol, "maxiter": 100000}
        self.gauge = {}    # gauge_id -> (ctx, handle, dims, stream)
        self.sources = {}  # gauge_id -> (links or a callable returning them, dims)
        self.host_results = host_results
        self.copy_stream = torch.cuda.Stream(device=self.device) if host_results else None  # default priority
        self.pending = {}  # id(request) -> (host tensor, event)

    def gauge_bits(self):
        return self.L.WILSON_GAUGE_FP32 | (self.L.WILSON_GAUGE_FP16 if self.opts["precision"] == 2 else 0)

    def add_gauge_source(self, gauge_id, U, dims):
        """Links (host or device tensor, or a callable returning one) that `load_gauge(gauge_id)`
        will load when the scheduler needs the field; returns an upper bound of its device
        bytes (full 18-real links)."""
        self.sources[gauge_id] = (U, tuple(dims))
        return self.L.wilson_gauge_footprint_bytes(dims, self.gauge_bits(), 18)

    def load_gauge(self, gauge_id, U=None, dims=None):
        torch = self.torch
        if U is None:
            U, dims = self.sources[gauge_id]
            U = U() if callable(U) else U
        stream = torch.cuda.Stream(device=self.device)  # default priority
        ctx = self.L.wilson_context_create(stream)
        g = self.L.wilson_gauge_load(ctx, U, dims, self.gauge_bits())
        self.gauge[gauge_id] = (ctx, g, tuple(dims), stream)
        return self.L.wilson_gauge_bytes(g)

    def unload_gauge(self, gauge_id):
        ctx, g, dims, stream = self.gauge.pop(gauge_id)
        stream.synchronize()
        self.L.wilson_gauge_free(ctx, g)
        self.L.wilson_context_destroy(ctx)

    def batch_bytes(self, dims, nslots):
        return self.L.wilson_footprint_bytes(dims, nslots, self.opts)

    # Cost model of one batched iteration (milliseconds): a launch-bound floor (about a
    # dozen kernels) plus the streamed bytes at a sustained rate: per right-hand side the
    # four hops' spinor traffic and the vector updates (~2300 B per even site in FP32),
    # and the links of the four hops, shared (~1536 B per even site).
    LAUNCH_MS = 0.15
    SUSTAINED_BYTES_PER_MS = 5.0e9

    def iter_ms(self, handle, n_active):
        dims = self.gauge[handle[0]][2]
        vh = (dims[0] * dims[1] * dims[2] * dims[3]) // 2
        return self.LAUNCH_MS + vh * (2300.0 * max(n_active, 1) + 1536.0) / self.SUSTAINED_BYTES_PER_MS

    def create_batch(self, gauge_id, nslots):
        ctx, g, dims, stream = self.gauge[gauge_id]
        return (gauge_id, self.L.wilson_batch_create(ctx, g, nslots, self.opts), nslots)

    def destroy_batch(self, handle):
        self.L.wilson_batch_destroy(handle[1])

    def alloc_solution(self, req):
        if self.host_results:  # solved on the device, copied out when the request is done
            return self.torch.zeros(tuple(req.b.shape), dtype=self.torch.complex128, device=self.device)
        return self.torch.zeros(tuple(req.b.shape), dtype=self.torch.complex128)

    def attach(self, handle, slot, req, j):
        b = req.b[j]
        if not b.is_contiguous():
            b = b.contiguous()
        st = self.L.wilson_batch_attach(handle[1], slot, b, req.kappa, req.tol, req.maxiter)
        self.L.check(st, "wilson_batch_attach")

    def step(self, handle, iters):
        self.L.wilson_batch_step(handle[1], iters)

    def ready(self, handle):
        """True when the batch's stream has no work left (non-blocking)."""
        return self.gauge[handle[0]][3].query()

    def poll(self, handle):
        return self.L.wilson_batch_poll(handle[1], handle[2])

    def detach(self, handle, slot, req, j):
        out = req.x[j]
        st, info = self.L.wilson_batch_detach(handle[1], slot, out)
        return st, info

    def finish(self, req):
        if not self.host_results:
            return
        torch = self.torch
        xh = torch.empty(tuple(req.x.shape), dtype=req.x.dtype, pin_memory=True)
        ev = torch.cuda.Event()
        with torch.cuda.stream(self.copy_stream):  # detach has already synchronized the solve's stream
            xh.copy_(req.x, non_blocking=True)
            ev.record()
        self.pending[id(req)] = (xh, ev)

    def finished(self, req):
        """True once the request's solutions are on the host (non-blocking)."""
        if not self.host_results:
            return True
        xh, ev = self.pending[id(req)]
        if not ev.query():
            return False
        del self.pending[id(req)]
        req.x = xh
        return True

    def close(self):
        for gid, (ctx, g, dims, stream) in self.gauge.items():
            self.L.wilson_gauge_free(ctx, g)
            self.L.wilson_context_destroy(ctx)
        self.gauge.clear()


def make_server(hbm_budget, nslots=12, step_iters=8, precision=1, solver=0, turn_ms=None, max_heavy=None,
                host_results=False):
    eng = LibEngine(precision=precision, solver=solver, host_results=host_results)
    return Scheduler(eng, hbm_budget, nslots=nslots, step_iters=step_iters, turn_ms=turn_ms,
                     max_heavy=max_heavy), eng

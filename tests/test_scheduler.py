"""Serving policy of the continuous-batching scheduler, driven by a simulated engine and
clock (a test double of the engine interface only; the real engine is the library's batch
API, exercised in the GPU tests)."""
import numpy as np
import pytest

from paper_1811_00893_amd.serve import FINISHED, FREE, RUNNING, Request, Scheduler


class FakeEngine:
    """Each attached RHS finishes after `need` iterations (kappa-dependent); one step of
    `iters` iterations advances every running slot."""

    def __init__(self, batch_bytes=100.0):
        self.bb = batch_bytes
        self.batches = {}
        self.created = 0
        self.destroyed = 0
        self.steps = 0

    def batch_bytes(self, dims, nslots):
        return self.bb

    def create_batch(self, gid, nslots):
        self.created += 1
        h = (gid, self.created)
        self.batches[h] = [None] * nslots
        return h

    def destroy_batch(self, h):
        self.destroyed += 1
        del self.batches[h]

    def alloc_solution(self, req):
        return np.zeros(req.b.shape)

    def attach(self, h, k, req, j):
        assert self.batches[h][k] is None, "slot double-booked"
        need = int(round(1000 * req.kappa)) + j
        self.batches[h][k] = [need, 0, req.rid, j]

    def step(self, h, iters):
        self.steps += 1
        for s in self.batches[h]:
            if s is not None:
                s[1] += iters

    def poll(self, h):
        st = np.array([FREE if s is None else (FINISHED if s[1] >= s[0] else RUNNING) for s in self.batches[h]])
        return st, np.zeros_like(st)

    def detach(self, h, k, req, j):
        s = self.batches[h][k]
        assert s[2] == req.rid and s[3] == j
        req.x[j] = req.rid * 100 + j
        self.batches[h][k] = None
        return 0, {"iterations": s[1]}

    def finish(self, req):
        pass


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1.0
        return self.t


def mkreq(rid, gid, nrhs, kappa=0.01):
    return Request(rid=rid, gauge_id=gid, kappa=kappa, tol=1e-10, b=np.zeros((nrhs, 4)))


def test_slots_refill_and_requests_complete():
    eng = FakeEngine()
    sch = Scheduler(eng, hbm_budget=1000, nslots=4, step_iters=5, clock=Clock())
    sch.register_gauge("g", (4, 4, 4, 4), 50)
    reqs = [mkreq(i, "g", nrhs=n) for i, n in enumerate([3, 3, 2, 5])]
    for r in reqs:
        assert sch.submit(r)
    sch.admit()
    b = sch.batches["g"]
    # 4 slots: request 0 takes 3, request 1 takes the last one, the rest wait
    assert [s[0].rid for s in b["slots"]] == [0, 0, 0, 1]
    assert reqs[1].pending == [1, 2] and len(sch.waiting) == 3
    sch.run_until_idle()
    assert sorted(r.rid for r in sch.completed) == [0, 1, 2, 3]
    for r in reqs:
        assert list(r.x[:, 0]) == [r.rid * 100 + j for j in range(r.nrhs)]
        assert all(s == 0 for s in r.status)
        assert r.latency is not None and r.latency > 0
    assert eng.created == 1


def test_admission_by_memory_budget_and_rejection():
    """Resident gauge fields and batch workspaces must fit the HBM budget together; a
    request whose field plus one batch can never fit is rejected at once."""
    eng = FakeEngine(batch_bytes=100)
    sch = Scheduler(eng, hbm_budget=300, nslots=2, step_iters=10, clock=Clock())
    sch.register_gauge("a", (4, 4, 4, 4), 30)
    sch.register_gauge("b", (4, 4, 4, 4), 30)
    assert not sch.submit(mkreq(9, "unknown", 1))
    assert sch.submit(mkreq(0, "a", 2))
    assert sch.submit(mkreq(1, "b", 2))
    sch.admit()
    # 30 + 30 (fields) + 100 + 100 (two batches) = 260 <= 300
    assert set(sch.batches) == {"a", "b"}
    assert sch.resident_bytes() <= 300
    sch.run_until_idle()
    assert len(sch.completed) == 2
    small = Scheduler(FakeEngine(batch_bytes=100), hbm_budget=120, nslots=2, clock=Clock())
    small.register_gauge("c", (4, 4, 4, 4), 30)
    assert not small.submit(mkreq(3, "c", 1))  # 30 + 100 > 120: can never run
    assert small.rejected and small.rejected[0].rid == 3


def test_idle_batches_are_evicted_to_admit_new_ones():
    eng = FakeEngine(batch_bytes=100)
    sch = Scheduler(eng, hbm_budget=200, nslots=2, step_iters=50, clock=Clock())
    for g in ("a", "b"):
        sch.register_gauge(g, (4, 4, 4, 4), 10)
    sch.submit(mkreq(0, "a", 1))
    sch.run_until_idle()
    assert "a" in sch.batches
    sch.submit(mkreq(1, "b", 1))  # 10 + 10 + 100 + 100 > 200: idle batch a must go
    sch.run_until_idle()
    assert "a" not in sch.batches and eng.destroyed == 1
    assert len(sch.completed) == 2


def test_result_independent_of_mix():
    """A request's slots see only their own RHS: same outputs alone and mixed."""
    def run(mix):
        eng = FakeEngine()
        sch = Scheduler(eng, hbm_budget=1e9, nslots=3, step_iters=7, clock=Clock())
        sch.register_gauge("g", (4, 4, 4, 4), 1)
        target = mkreq(42, "g", 4, kappa=0.013)
        for r in ([mkreq(i, "g", 2, kappa=0.02 + 0.001 * i) for i in range(mix)] + [target]):
            sch.submit(r)
        sch.run_until_idle()
        return target.x.copy(), [i["iterations"] >= 13 for i in target.info]
    a = run(0)
    b = run(5)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


def test_turn_length_adapts_to_target():
    """With a target turn duration the iterations per turn shrink when a turn runs long
    and grow back (up to the maximum) when it runs short."""
    import time as _time

    class SlowEngine(FakeEngine):
        per_iter_s = 0.002

        def step(self, h, iters):
            super().step(h, iters)
            _time.sleep(iters * self.per_iter_s)

    eng = SlowEngine()
    sch = Scheduler(eng, hbm_budget=1e9, nslots=2, step_iters=16, clock=Clock(), turn_ms=8.0)
    sch.register_gauge("g", (4, 4, 4, 4), 1)
    sch.submit(mkreq(0, "g", 2, kappa=0.2))  # 200+ iterations
    for _ in range(8):
        sch.admit()
        sch.step()
    assert 2 <= sch.iters <= 6, sch.iters      # about 8 ms / 2 ms per iteration
    eng.per_iter_s = 0.0001
    for _ in range(8):
        sch.admit()
        sch.step()
    assert sch.iters == 16                     # short turns: back to the maximum
    sch.run_until_idle()
    assert len(sch.completed) == 1


def test_per_batch_turn_length_from_engine_cost():
    """An engine that estimates the cost of an iteration gets per-batch iteration counts:
    the cheap batch advances many iterations per turn, the expensive one a few."""
    class CostEngine(FakeEngine):
        cost = {"small": 0.1, "big": 4.0}

        def iter_ms(self, h, n_active):
            return self.cost[h[0]]

    eng = CostEngine()
    sch = Scheduler(eng, hbm_budget=1e9, nslots=2, step_iters=32, clock=Clock(), turn_ms=4.0)
    for gid in ("small", "big"):
        sch.register_gauge(gid, (4, 4, 4, 4), 1)
        sch.submit(mkreq(len(sch.waiting), gid, 1, kappa=0.5))
    sch.admit()
    assert sch._iters_for(sch.batches["small"]) == 32   # 4 ms / 0.1 ms, capped
    assert sch._iters_for(sch.batches["big"]) == 1
    sch.run_until_idle()
    assert len(sch.completed) == 2


def test_independent_turns_with_ready():
    """With `ready`, a batch whose turn is still running is neither waited for nor given
    new slots; other batches keep turning and completing."""
    class AsyncEngine(FakeEngine):
        def __init__(self):
            super().__init__()
            self.busy_polls = {}

        def ready(self, h):
            # the "slow" batch reports its turn done only every third query
            if h[0] != "slow":
                return True
            self.busy_polls[h] = self.busy_polls.get(h, 0) + 1
            return self.busy_polls[h] % 3 == 0

    eng = AsyncEngine()
    sch = Scheduler(eng, hbm_budget=1e9, nslots=2, step_iters=5, clock=Clock())
    for gid in ("slow", "fast"):
        sch.register_gauge(gid, (4, 4, 4, 4), 1)
    sch.submit(mkreq(0, "slow", 2, kappa=0.05))
    sch.submit(mkreq(1, "fast", 2, kappa=0.05))
    sch.submit(mkreq(2, "slow", 1, kappa=0.05))  # waits for a free slot of the slow batch
    steps_before = eng.steps
    sch.admit()
    sch.step()
    assert sch.batches["slow"]["inflight"] and not sch.batches["fast"]["inflight"]
    sch.admit()  # no attach into a batch with a turn in flight
    assert [s[0].rid for s in sch.batches["slow"]["slots"]] == [0, 0]
    sch.run_until_idle()
    assert sorted(r.rid for r in sch.completed) == [0, 1, 2]
    assert all(not b.get("inflight") for b in sch.batches.values())
    assert eng.steps > steps_before


def test_heavy_batches_take_turns_oldest_first():
    """With max_heavy = 1 only the heavy batch holding the oldest request advances; the
    other heavy batch keeps its slots and waits, light batches advance meanwhile, and the
    waiting batch runs once the first drains."""
    class CostEngine(FakeEngine):
        cost = {"big1": 3.0, "big2": 3.0, "small": 0.05}

        def __init__(self):
            super().__init__()
            self.log = []

        def iter_ms(self, h, n_active):
            return self.cost[h[0]]

        def step(self, h, iters):
            self.log.append(h[0])
            super().step(h, iters)

    eng = CostEngine()
    sch = Scheduler(eng, hbm_budget=1e9, nslots=2, step_iters=4, clock=Clock(), max_heavy=1, heavy_ms=1.0)
    for gid in ("big2", "big1", "small"):
        sch.register_gauge(gid, (4, 4, 4, 4), 1)
    sch.submit(mkreq(0, "big1", 1, kappa=0.02))   # oldest: 20 iterations
    sch.submit(mkreq(1, "big2", 1, kappa=0.02))
    sch.submit(mkreq(2, "small", 1, kappa=0.01))
    sch.admit()
    sch.step()
    assert sorted(eng.log) == ["big1", "small"]
    while not any(r.rid == 0 for r in sch.completed):
        sch.admit()
        sch.step()
    assert "big2" not in eng.log                 # held until the oldest heavy request finished
    sch.run_until_idle()
    assert sorted(r.rid for r in sch.completed) == [0, 1, 2]
    with pytest.raises(ValueError):
        Scheduler(eng, hbm_budget=1e9, max_heavy=0)


class LoadingEngine(FakeEngine):
    """FakeEngine whose gauge fields are loaded and unloaded on demand (40 bytes each)."""

    def __init__(self, batch_bytes=100.0):
        super().__init__(batch_bytes)
        self.loaded = set()
        self.log = []

    def load_gauge(self, gid):
        assert gid not in self.loaded
        self.loaded.add(gid)
        self.log.append(("load", gid))
        return 40

    def unload_gauge(self, gid):
        assert not any(h[0] == gid for h in self.batches), "field unloaded under a live batch"
        self.loaded.remove(gid)
        self.log.append(("unload", gid))

    def create_batch(self, gid, nslots):
        assert gid in self.loaded, "batch on a field that is not resident"
        return super().create_batch(gid, nslots)


def test_gauge_fields_load_on_demand_and_evict_least_recently_used():
    """With room for one field and its batch (170 < 2 x 40 + 100), requests on fields a, b, a
    load a, then release
    a's idle batch and field for b, then reload a; the loaded size replaces the upper bound,
    and no request is rejected."""
    eng = LoadingEngine(batch_bytes=100)
    sch = Scheduler(eng, hbm_budget=170, nslots=2, step_iters=50, clock=Clock())
    for g in "ab":
        sch.register_gauge(g, (4, 4, 4, 4), 50, resident=False)  # 50: upper bound; 40 once loaded
    for rid, g in enumerate("aba"):
        assert sch.submit(mkreq(rid, g, 1))
        sch.run_until_idle()
        assert sch.resident_bytes() <= 170
    assert eng.log == [("load", "a"), ("unload", "a"), ("load", "b"), ("unload", "b"), ("load", "a")]
    assert sch.loads == 3 and sch.evictions == 2
    assert sch.gauges["a"]["bytes"] == 40 and sch.gauges["a"]["resident"]
    assert [r.rid for r in sch.completed] == [0, 1, 2]
    assert list(sch.completed[2].x[:, 0]) == [200]


def test_field_with_an_older_waiting_request_is_not_evicted():
    """A request for field b that arrives while an older request for a still has right-hand
    sides waiting does not take a's place: a's request finishes first, then b is loaded."""
    eng = LoadingEngine(batch_bytes=100)
    sch = Scheduler(eng, hbm_budget=170, nslots=2, step_iters=5, clock=Clock())
    for g in "ab":
        sch.register_gauge(g, (4, 4, 4, 4), 40, resident=False)
    assert sch.submit(mkreq(0, "a", 5))   # 5 RHS through 2 slots: part of it waits
    assert sch.submit(mkreq(1, "b", 1))
    sch.run_until_idle()
    assert [r.rid for r in sch.completed] == [0, 1]
    assert eng.log == [("load", "a"), ("unload", "a"), ("load", "b")]
    # a field that can never fit (40 + 100 > 120) is still rejected at once
    small = Scheduler(LoadingEngine(batch_bytes=100), hbm_budget=120, nslots=2, clock=Clock())
    small.register_gauge("c", (4, 4, 4, 4), 40, resident=False)
    assert not small.submit(mkreq(3, "c", 1))

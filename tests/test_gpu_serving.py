"""Serving on the GPU: continuous batching through the library's batch API.

Every finished right-hand side must pass the oracle's FP64 residual check, and a
request's result must be bitwise the same alone and in a mix with other requests: a slot's
arithmetic never reads another slot, its reductions are summed per slot in a fixed order,
and the launch shapes depend on the batch's slot count, not on how many slots are busy.
The mix covers two tiny lattices (direction-split hops) and a 16^3x32 lattice, whose hops
run in the tuned multi-RHS shapes of a 4-slot batch.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1811_00893_amd import inputs
from paper_1811_00893_amd.serve import Request, make_server

pytestmark = pytest.mark.gpu


def residual(x, b, U, k, dims):
    return float(np.linalg.norm(b - oracle.apply_D(x, U, k, dims)) / np.linalg.norm(b))


GAUGES = {"a": ((4, 4, 4, 4), 1101, 0.25), "b": ((4, 4, 2, 8), 1102, 0.35), "c": ((16, 16, 16, 32), 1103, 0.3)}


def fields():
    return {gid: inputs.gauge_field(d, eps=e, seed=s) for gid, (d, s, e) in GAUGES.items()}


def serve(requests, U, precision, nslots=4, step_iters=3):
    sch, eng = make_server(hbm_budget=64e9, nslots=nslots, step_iters=step_iters, precision=precision)
    try:
        for gid, (dims, _, _) in GAUGES.items():
            nb = eng.load_gauge(gid, U[gid].cuda(), dims)
            sch.register_gauge(gid, dims, nb)
        for r in requests:
            assert sch.submit(r)
        sch.run_until_idle()
    finally:
        sch.close()
        eng.close()
    return sch


def make_requests(ids, seed0=0):
    out = []
    rng = np.random.default_rng(seed0)
    for rid in ids:
        gid = "abc"[rid % 3]
        dims = GAUGES[gid][0]
        nrhs = 1 + (rid // 3) % 3
        b = inputs.gaussian_source(dims, seed=5000 + rid, nrhs=nrhs)
        out.append(Request(rid=rid, gauge_id=gid, kappa=0.115 + 0.002 * (rid % 5), tol=[1e-8, 1e-10, 1e-12][rid % 3],
                           b=b, maxiter=5000))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_serving_results_pass_oracle_and_match_alone(precision):
    U = fields()
    mix = make_requests(range(7))
    sch = serve(mix, U, precision)
    assert len(sch.completed) == 7
    for r in sch.completed:
        dims = GAUGES[r.gauge_id][0]
        for j in range(r.nrhs):
            assert r.status[j] == 0, (r.rid, j, r.status)
            res = residual(r.x[j].numpy(), r.b[j].numpy(), U[r.gauge_id].numpy(), r.kappa, dims)
            assert res < r.tol, (r.rid, j, res, r.tol)
        assert r.latency > 0
    # the same requests alone: a tiny lattice (rid 4) and the 16^3x32 one with two RHS (rid 5)
    for rid in (4, 5):
        target = [r for r in sch.completed if r.rid == rid][0]
        alone = serve(make_requests([rid]), U, precision)
        x_alone = alone.completed[0].x
        d = float((x_alone - target.x).abs().max() / target.x.abs().max())
        print(f"precision {precision} request {rid} ({target.gauge_id}, {target.nrhs} RHS): "
              f"alone vs mixed max relative difference {d:.2e}")
        assert torch.equal(x_alone, target.x)


def test_batch_api_slot_lifecycle():
    """attach -> step -> poll -> detach through the raw API; a busy slot refuses a second
    attach, an unfinished slot refuses detach, and a freed slot is reusable."""
    from paper_1811_00893_amd import _lib as L
    dims = (4, 4, 4, 4)
    U = inputs.gauge_field(dims, seed=1201)
    ctx = L.wilson_context_create()
    g = L.wilson_gauge_load(ctx, U.cuda(), dims)
    bat = L.wilson_batch_create(ctx, g, 2, {"precision": 0})
    b0 = inputs.gaussian_source(dims, seed=1)
    b1 = inputs.gaussian_source(dims, seed=2)
    assert L.wilson_batch_attach(bat, 0, b0, 0.12, 1e-10) == 0
    assert L.wilson_batch_attach(bat, 0, b1, 0.12, 1e-10) == L.WILSON_BUSY
    x = torch.zeros_like(b0)
    st, _ = L.wilson_batch_detach(bat, 0, x)
    assert st == L.WILSON_BUSY
    assert L.wilson_batch_attach(bat, 1, b1, 0.125, 1e-10) == 0
    for _ in range(200):
        L.wilson_batch_step(bat, 4)
        state, status = L.wilson_batch_poll(bat, 2)
        if (state == 2).all():
            break
    assert (state == 2).all() and (status == 0).all()
    for slot, (b, k) in enumerate(((b0, 0.12), (b1, 0.125))):
        x = torch.zeros_like(b)
        st, info = L.wilson_batch_detach(bat, slot, x)
        assert st == 0 and info["converged"] == 1
        assert residual(x.numpy(), b.numpy(), U.numpy(), k, dims) < 1e-10
    state, _ = L.wilson_batch_poll(bat, 2)
    assert (state == 0).all()
    assert L.wilson_batch_attach(bat, 0, b1, 0.125, 1e-10) == 0  # reusable
    L.wilson_batch_destroy(bat)
    L.wilson_gauge_free(ctx, g)
    L.wilson_context_destroy(ctx)


def test_evicted_and_reloaded_field_gives_identical_results():
    """An HBM budget with room for one 8^4 field and its batch but not two fields: requests on
    fields a, b, a load a, release it for b, and load it again (then b is released).  The
    third request (field a, the same sources and kappa as the first) gives bitwise the
    first one's solutions, every result passes the oracle, and solutions arrive on the host
    through the engine's asynchronous copy."""
    from paper_1811_00893_amd.serve import LibEngine, Scheduler
    dims = (8, 8, 8, 8)
    Ua = inputs.gauge_field(dims, eps=0.3, seed=1601)
    Ub = inputs.gauge_field(dims, eps=0.25, seed=1602)
    b = inputs.gaussian_source(dims, seed=1603, nrhs=2)
    eng = LibEngine(precision=1, host_results=True)
    ga = eng.add_gauge_source("a", Ua.cuda(), dims)
    gb = eng.add_gauge_source("b", lambda: Ub.cuda(), dims)  # a source may also be produced on demand
    bb = eng.batch_bytes(dims, 2)
    sch = Scheduler(eng, ga + bb + ga // 4, nslots=2, step_iters=4)
    sch.register_gauge("a", dims, ga, resident=False)
    sch.register_gauge("b", dims, gb, resident=False)
    reqs = [Request(rid=k, gauge_id=g, kappa=0.12, tol=1e-10, b=b.clone()) for k, g in enumerate("aba")]
    try:
        for r in reqs:
            assert sch.submit(r)
            sch.run_until_idle()
            assert sch.resident_bytes() <= sch.budget
    finally:
        sch.close()
        eng.close()
    print(f"loads {sch.loads}, evictions {sch.evictions}")
    assert sch.loads == 3 and sch.evictions == 2
    assert [r.rid for r in sch.completed] == [0, 1, 2]
    assert not reqs[0].x.is_cuda and not reqs[2].x.is_cuda
    assert torch.equal(reqs[0].x, reqs[2].x)
    for r, U in zip(reqs, (Ua, Ub, Ua)):
        for j in range(2):
            assert r.status[j] == 0
            assert residual(r.x[j].numpy(), b[j].numpy(), U.numpy(), 0.12, dims) < 1e-10

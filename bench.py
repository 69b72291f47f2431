"""Benchmark: Wilson-Dirac solves on one MI355X.

Default workload (one "step" = one whole solve): plain FP64 even-odd BiCGStab on a
32^3x64 lattice, links exp(i*0.3*A), kappa = 0.125, a complex Gaussian source per step,
relative residual 1e-10 (checked in FP64 after the iteration).  Sources and links are
resident in HBM before the timed region starts.

Printed: one JSON line with solves/s (value), p50/p99 latency from a separate pass of 100
solves, the achieved bandwidth of the dominant kernel (the parity hop, timed with HIP events
on the library's stream) against the MI355X HBM peak on the algorithmic byte count, the
bytes two-row links must move and the measured counter traffic, a Dslash-only figure (parity
hop alone), the CPU oracle timed on the same workload (a full FP64 solve), and under
"configs" the headline figures of the other configurations: 8^4 FP64, the three
mixed-precision variants at 48^3x96 and the 12 point sources at 24^3x48 (each with its hop's
roofline fractions and the gain over the plain FP64 solver; --no-extras leaves them out).

Other workloads (not the headline line): --workload small8 | mixed48 | mixed48_fp16 | mixed48_fp16h |
mixed48_reliable | mixed48_fp16_reliable | batched24 | batched24_fp16 | block24 | block24_k135 |
clover32 | clover32_mixed | serve | layouts.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash GB/s & % HBM roofline; solves/s + p99 latency at rel. residual 1e-10"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="fp64_32")
    p.add_argument("--dslash-reps", type=int, default=100)
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--inner-tol", type=float, default=0.0,
                   help="mixed precision: residual drop per cycle (0: the library's default)")
    p.add_argument("--dslash-only", action="store_true", help="only the Dslash section and the copy probe")
    p.add_argument("--requests", type=int, default=60, help="serving: requests per phase")
    p.add_argument("--loads", type=lambda v: [float(x) for x in v.split(",")], default=[0.5, 0.8, 1.0],
                   help="serving: offered loads as fractions of the server's closed-loop capacity")
    p.add_argument("--outstanding", type=int, default=24, help="serving: requests in flight in the capacity run")
    p.add_argument("--step-iters", type=int, default=32, help="serving: most iterations per scheduler turn")
    p.add_argument("--turn-ms", type=float, default=3.0, help="serving: target duration of a scheduler turn")
    p.add_argument("--max-heavy", type=int, default=2,
                   help="serving: heavy batches (an iteration >= 0.5 ms) advancing at once, oldest first (0: no limit)")
    p.add_argument("--hbm-budget", type=float, default=100e9, help="serving: device bytes for fields + batches")
    p.add_argument("--nslots", type=int, default=12, help="serving: solve slots per gauge field's batch")
    p.add_argument("--latency-samples", type=int, default=100, help="solves of the latency pass (p50/p99)")
    p.add_argument("--extra-latency-samples", type=int, default=100,
                   help="latency pass of the other configurations of the default run")
    p.add_argument("--no-extras", action="store_true",
                   help="default run: leave out the other configurations (8^4, 48^3x96 mixed x 3, 24^3x48 batched)")
    return p.parse_args()


KERNEL_SOURCES = ["paper_1811_00893_amd/csrc/dslash.hip", "paper_1811_00893_amd/csrc/dslash_kernels.h",
                  "paper_1811_00893_amd/csrc/device.h", "paper_1811_00893_amd/csrc/common.h"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def committed_traffic(workload, dslash):
    """HBM bytes per hop launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE, calibrated on the library's streaming copy), or None when the kernel
    sources changed since the counters were taken or no summary covers this workload."""
    path = os.path.join(ROOT, "profiles", "hop_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(workload)
    if not rec or rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q))


WORKLOADS = {
    # name: (dims, kappa, tol, precision, nrhs, description)
    "fp64_32": ((32, 32, 32, 64), 0.125, 1e-10, 0, 1,
                "plain FP64 even-odd BiCGStab, 32^3x64, kappa=0.125, eps=0.3, tol=1e-10"),
    "small8": ((8, 8, 8, 8), 0.12, 1e-10, 0, 1, "plain FP64 even-odd BiCGStab, 8^4, kappa=0.12, tol=1e-10"),
    "mixed48": ((48, 48, 48, 96), 0.125, 1e-10, 1, 1,
                "mixed precision (FP32 inner, FP64 outer) even-odd BiCGStab, 48^3x96, kappa=0.125, tol=1e-10"),
    "mixed48_fp16": ((48, 48, 48, 96), 0.125, 1e-10, 3, 1,
                     "mixed precision (FP16 spinors + per-site scale, FP32 links inner; FP64 outer), 48^3x96"),
    "mixed48_fp16h": ((48, 48, 48, 96), 0.125, 1e-10, 2, 1,
                      "mixed precision (FP16 spinors + per-site scale, FP16 links inner; FP64 outer), 48^3x96"),
    "batched24": ((24, 24, 24, 48), 0.125, 1e-10, 1, 12,
                  "12 point sources in one batched solve, FP32 inner / FP64 outer, 24^3x48, kappa=0.125"),
    "batched24_fp16": ((24, 24, 24, 48), 0.125, 1e-10, 3, 12,
                       "12 point sources in one batched solve, FP16 spinors + per-site scale and FP32 links "
                       "inner / FP64 outer, 24^3x48, kappa=0.125"),
    "clover32": ((32, 32, 32, 64), 0.125, 1e-10, 0, 1,
                 "clover matrix D_W + F, plain FP64 even-odd BiCGStab, 32^3x64, kappa=0.125, synthetic F (c=0.05)"),
    "clover32_mixed": ((32, 32, 32, 64), 0.125, 1e-10, 1, 1,
                       "clover matrix D_W + F, mixed precision (FP32 inner, FP64 outer), 32^3x64, kappa=0.125"),
    "mixed48_reliable": ((48, 48, 48, 96), 0.125, 1e-10, 1, 1,
                         "mixed precision with reliable updates (FP32 inner recurrence kept across FP64 residual "
                         "replacements), 48^3x96, kappa=0.125, tol=1e-10"),
    "mixed48_fp16_reliable": ((48, 48, 48, 96), 0.125, 1e-10, 3, 1,
                              "mixed precision with reliable updates (FP16 spinors + per-site scale, FP32 links), "
                              "48^3x96, kappa=0.125, tol=1e-10"),
    "block24": ((24, 24, 24, 48), 0.125, 1e-10, 0, 12,
                "12 point sources solved together by block BiCGStab (one Krylov space, s = 12), FP64, 24^3x48, "
                "kappa=0.125"),
    "block24_k135": ((24, 24, 24, 48), 0.135, 1e-10, 0, 12,
                     "12 point sources solved together by block BiCGStab (one Krylov space, s = 12), FP64, "
                     "24^3x48, kappa=0.135 (closer to critical)"),
}
CLOVER = {"clover32", "clover32_mixed"}
RELIABLE = {"mixed48_reliable", "mixed48_fp16_reliable"}
BLOCK = {"block24", "block24_k135"}


def run_serving(args):
    """Serving: a Poisson stream of solve requests over four lattice sizes, each request on
    one of two seeded gauge fields per size (eps ~ U[0.2, 0.4]), kappa ~ U[0.115, 0.125],
    tol in {1e-8, 1e-10, 1e-12}, 1-12 Gaussian right-hand sides; mixed precision (FP32 inner,
    FP64 outer).  Sources are generated when a request arrives and released when it
    completes, so any number of requests fits in memory.

      1. FIFO baselines, every request of the trace served alone, one after the other:
         (a) all its right-hand sides in one mixed-precision batched solve; (b) the plain
         path: each right-hand side by the FP64 solver alone.  Their service times give
         FIFO latencies on any arrival sequence.
      2. Capacity: the continuous-batching server fed as fast as it drains (at most
         `--outstanding` requests waiting or running): RHS/s and requests/s.
      3. For each offered load in `--loads` (fractions of that capacity): Poisson arrivals
         at load x capacity replayed through the server; p50/p99 latency (arrival ->
         solution on the host) and throughput, next to FIFO on the same arrivals.
    Every latency, FIFO's too, ends when the solution is in pinned host memory.  The server
    admits by HBM footprint within `--hbm-budget`: the gauge fields are registered as
    sources and loaded when first needed; idle batches and fields are released to make
    room (least recently used first) and reloaded when needed again.
    """
    import numpy as np
    import torch

    from paper_1811_00893_amd import _lib as L
    from paper_1811_00893_amd import inputs
    from paper_1811_00893_amd.serve import Request, make_server

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(3000)
    sizes = [(8, 8, 8, 8), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)]
    pool = {}
    for si, d in enumerate(sizes):
        for k in range(2):
            pool[(si, k)] = (d, float(rng.uniform(0.2, 0.4)), 3100 + 10 * si + k)
    nreq = args.requests
    trace = []
    for i in range(nreq):
        si = int(rng.integers(0, 4))
        k = int(rng.integers(0, 2))
        trace.append(dict(gid=(si, k), kappa=float(rng.uniform(0.115, 0.125)),
                          tol=float([1e-8, 1e-10, 1e-12][int(rng.integers(0, 3))]),
                          nrhs=int(rng.integers(1, 13)), seed=4000 + i))
    rhs_total = sum(t["nrhs"] for t in trace)
    U = {gid: inputs.gauge_field(d, eps=e, seed=s, device=dev) for gid, (d, e, s) in pool.items()}

    def source(i):
        t = trace[i]
        return inputs.gaussian_source(pool[t["gid"]][0], seed=t["seed"], nrhs=t["nrhs"], device=dev)

    def progress(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    opts = {"precision": 1, "maxiter": 100000}

    # 1. FIFO: one request at a time through wilson_solve_ex (all its RHS together)
    ctx = L.wilson_context_create()
    G = {gid: L.wilson_gauge_load(ctx, U[gid], pool[gid][0], L.WILSON_GAUGE_FP32) for gid in pool}

    def fifo_once(i, b):
        t = trace[i]
        x = torch.zeros_like(b)
        st, _ = L.wilson_solve_ex(ctx, G[t["gid"]], x, b, t["nrhs"], t["kappa"], t["tol"], opts)
        L.check(st, "fifo solve")
        xh = torch.empty(x.shape, dtype=x.dtype, pin_memory=True)
        xh.copy_(x)  # the solution on the host

    # warm the tuner: every lattice size and class of RHS count before anything is timed
    for si, d in enumerate(sizes):
        for n in (1, 2, 4, 8, 12):
            b = inputs.gaussian_source(d, seed=3900 + n, nrhs=n, device=dev)
            x = torch.zeros_like(b)
            L.check(L.wilson_solve_ex(ctx, G[(si, 0)], x, b, n, 0.12, 1e-8, opts)[0], "warm-up solve")
            del b, x
    progress("tuner warm")
    service = []
    torch.cuda.synchronize()
    for i in range(nreq):
        b = source(i)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        fifo_once(i, b)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - s0)
        del b
        if (i + 1) % 50 == 0:
            progress(f"fifo {i + 1}/{nreq}")
    fifo_total = sum(service)

    # the plain path: one request at a time, each right-hand side by the FP64 solver alone
    popts = {"precision": 0, "maxiter": 100000}
    plain = []
    for i in range(nreq):
        t = trace[i]
        b = source(i)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for j in range(t["nrhs"]):
            x = torch.zeros_like(b[j])
            st, _ = L.wilson_solve_ex(ctx, G[t["gid"]], x, b[j], 1, t["kappa"], t["tol"], popts)
            L.check(st, "plain FP64 solve")
            xh = torch.empty(x.shape, dtype=x.dtype, pin_memory=True)
            xh.copy_(x)
        torch.cuda.synchronize()
        plain.append(time.perf_counter() - s0)
        del b
        if (i + 1) % 50 == 0:
            progress(f"plain fp64 {i + 1}/{nreq}")
    plain_total = sum(plain)

    def fifo_replay(arrivals):
        """The batched FIFO run in real time on the trace's arrivals: each request waits
        for the one before it, its source is made on arrival (as for the server) and its
        latency runs to the solution in host memory."""
        t0 = time.perf_counter()
        lat = []
        for i in range(nreq):
            wait = arrivals[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            fifo_once(i, source(i))
            lat.append(time.perf_counter() - t0 - arrivals[i])
        return lat, rhs_total / (time.perf_counter() - t0)

    # the continuous-batching server
    sch, eng = make_server(hbm_budget=args.hbm_budget, nslots=args.nslots, step_iters=args.step_iters, precision=1,
                           turn_ms=args.turn_ms, max_heavy=args.max_heavy if args.max_heavy > 0 else None,
                           host_results=True)
    for gid, (d, e, s) in pool.items():  # loaded on first use, within the budget
        sch.register_gauge(gid, d, eng.add_gauge_source(gid, U[gid], d), resident=False)
    for si, d in enumerate(sizes):  # one request per lattice size through the server
        sch.submit(Request(rid=-1 - si, gauge_id=(si, 0), kappa=0.12, tol=1e-8,
                           b=inputs.gaussian_source(d, seed=3950, nrhs=1, device=dev)))
    sch.run_until_idle()
    sch.completed.clear()

    def serve(arrivals, outstanding=None):
        """Replay the trace; arrivals None = closed loop with at most `outstanding` requests
        in the server.  Returns (wall seconds, latencies, failed request ids)."""
        t0 = time.perf_counter()
        sch.clock = lambda: time.perf_counter() - t0
        sch.completed.clear()
        lat, bad, done, nxt, inflight = [], [], 0, 0, 0
        while done < nreq:
            now = sch.clock()
            while nxt < nreq and ((arrivals is None and inflight < outstanding) or
                                  (arrivals is not None and arrivals[nxt] <= now)):
                t = trace[nxt]
                r = Request(rid=nxt, gauge_id=t["gid"], kappa=t["kappa"], tol=t["tol"], b=source(nxt),
                            maxiter=100000, arrival=float(arrivals[nxt]) if arrivals is not None else now)
                if not sch.submit(r):
                    raise RuntimeError(f"request {nxt} rejected")
                nxt += 1
                inflight += 1
            if sch.busy():
                sch.admit()
                sch.step()
            elif arrivals is not None and nxt < nreq:
                time.sleep(max(0.0, min(arrivals[nxt] - now, 0.01)))
            for r in sch.completed:  # record and release finished requests
                lat.append(r.latency)
                if any(st != 0 for st in r.status):
                    bad.append(r.rid)
                r.b = r.x = None
                done += 1
                inflight -= 1
                if done % 100 == 0:
                    progress(f"served {done}/{nreq}")
            sch.completed.clear()
        return sch.clock(), lat, bad

    # 2. capacity of the server (closed loop)
    wall_c, lat_c, bad_c = serve(None, outstanding=args.outstanding)
    cap_req = nreq / wall_c
    progress(f"capacity {rhs_total / wall_c:.1f} RHS/s")

    # 3. open-loop load points
    points = []
    for load in args.loads:
        lam = load * cap_req
        arrivals = np.cumsum(np.random.default_rng(3500 + int(100 * load)).exponential(1.0 / lam, size=nreq))
        wall, lat, bad = serve(arrivals)
        def fifo(times):
            t_free, out = 0.0, []
            for a, sv in zip(arrivals, times):
                t_free = max(a, t_free) + sv
                out.append(t_free - a)
            return out, rhs_total / t_free
        fifo_lat, fifo_rate = fifo(service)
        plain_lat, plain_rate = fifo(plain)
        replay_lat, replay_rate = fifo_replay(arrivals)
        progress(f"load {load}: batched FIFO replayed, p99 {1e3 * percentile(replay_lat, 99):.0f} ms")
        points.append({
            "offered_load": load, "arrival_rate_per_s": lam,
            "rhs_per_s": rhs_total / wall, "requests_per_s": nreq / wall,
            "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
            "fifo_batched_mixed": {"p50_ms": 1e3 * percentile(fifo_lat, 50), "p99_ms": 1e3 * percentile(fifo_lat, 99),
                                   "rhs_per_s": fifo_rate,
                                   "note": "queue of the measured per-request service times"},
            "fifo_batched_mixed_replayed": {"p50_ms": 1e3 * percentile(replay_lat, 50),
                                            "p99_ms": 1e3 * percentile(replay_lat, 99), "rhs_per_s": replay_rate,
                                            "note": "run on the GPU in real time on the same arrivals"},
            "fifo_plain_fp64": {"p50_ms": 1e3 * percentile(plain_lat, 50), "p99_ms": 1e3 * percentile(plain_lat, 99),
                                "rhs_per_s": plain_rate},
            "failed_requests": bad,
        })
        progress(f"load {load}: p50 {points[-1]['p50_ms']:.0f} ms p99 {points[-1]['p99_ms']:.0f} ms")
    sch.close()
    eng.close()
    for g in G.values():
        L.wilson_gauge_free(ctx, g)
    L.wilson_context_destroy(ctx)
    return {
        "metric": METRIC, "workload": "serving", "unit": "solves/s",
        "value": rhs_total / wall_c,
        "requests": nreq, "rhs": rhs_total,
        "capacity": {"rhs_per_s": rhs_total / wall_c, "requests_per_s": cap_req,
                     "p50_ms": 1e3 * percentile(lat_c, 50), "p99_ms": 1e3 * percentile(lat_c, 99),
                     "outstanding": args.outstanding, "failed_requests": bad_c},
        "fifo_batched_mixed_capacity_rhs_per_s": rhs_total / fifo_total,
        "fifo_plain_fp64_capacity_rhs_per_s": rhs_total / plain_total,
        "gain_over_plain_fp64": (rhs_total / wall_c) / (rhs_total / plain_total),
        "load_points": points,
        "rejected": len(sch.rejected),
        "gauge_loads": sch.loads, "gauge_evictions": sch.evictions,
        "config": {"lattices": sizes, "gauge_fields_per_size": 2, "nslots": args.nslots,
                   "step_iters_max": args.step_iters, "turn_ms": args.turn_ms, "max_heavy": args.max_heavy,
                   "hbm_budget": args.hbm_budget,
                   "precision": "mixed_fp32", "latency": "arrival to solution in pinned host memory",
                   "loads_relative_to": "closed-loop capacity of the continuous-batching server"},
    }


def run_layouts(args):
    """Layout ablation: the parity hop of one kernel under each storage layout (site-per-lane
    planes, array of structures, 64-site tiles, sub-lattice lanes), FP64 and FP32, links
    stored as 18 or 12 reals, on 32^3x64; the library's production hop is timed beside it."""
    import numpy as np
    import torch

    from paper_1811_00893_amd import _lib as L
    from paper_1811_00893_amd import counts, inputs

    dims, kappa = (32, 32, 32, 64), 0.125
    dev = torch.device("cuda:0")
    Vh = int(np.prod(dims)) // 2
    U = inputs.gauge_field(dims, eps=0.3, seed=1002, device=dev)
    psi = inputs.gaussian_source(dims, seed=2002, device=dev)
    out = torch.zeros_like(psi)
    ctx = L.wilson_context_create()
    reps = max(args.dslash_reps // 2, 5)
    rows = []
    t0 = time.perf_counter()
    for prec, pname in ((0, "fp64"), (1, "fp32")):
        rb = counts.REAL_BYTES[pname]
        for link_reals in (18, 12):
            for name, lay in (("soa", 0), ("aos", 1), ("aosoa", 2), ("vnode", 3)):
                st, us = L.wilson_layout_hop(ctx, out, psi, U, dims, kappa, 0, prec, lay, link_reals, reps)
                L.check(st, f"layout hop {name}")
                alg = counts.hop_bytes_per_site(pname) * Vh
                stored = (8 * link_reals + 48) * rb * Vh
                rows.append({"layout": name, "precision": pname, "link_reals": link_reals, "us_per_launch": us,
                             "gbs_algorithmic": alg / (us * 1e-6) / 1e9,
                             "frac_hbm_peak": alg / (us * 1e-6) / 1e9 / counts.MI355X_HBM_GBS,
                             "gbs_stored_bytes": stored / (us * 1e-6) / 1e9})
                print(f"layout {name} {pname} links {link_reals}: {us:.1f} us", file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    # the production kernel on the same fields (tuned launch, link storage chosen at upload)
    g = L.wilson_gauge_load(ctx, U, dims, L.WILSON_GAUGE_FP32)
    prod = {}
    for prec, pname in ((0, "fp64"), (1, "fp32")):
        for _ in range(3):
            L.check(L.wilson_dslash_ex(ctx, g, out, psi, kappa, 0, prec, 1), "dslash")
        torch.cuda.synchronize()
        L.wilson_timing_enable(ctx, True)
        for _ in range(reps):
            L.check(L.wilson_dslash_ex(ctx, g, out, psi, kappa, 0, prec, 1), "dslash")
        torch.cuda.synchronize()
        ms, n, _ = L.wilson_timing_read(ctx, L.WILSON_KERNEL_HOP)
        L.wilson_timing_enable(ctx, False)
        us = 1e3 * ms / max(n, 1)
        alg = counts.hop_bytes_per_site(pname) * Vh
        prod[pname] = {"us_per_launch": us, "gbs_algorithmic": alg / (us * 1e-6) / 1e9}
    L.wilson_gauge_free(ctx, g)
    # 2 GiB copy probe: bandwidth reference, and the calibration of hardware byte counters
    nb = 1 << 31
    src_buf = torch.empty(nb, dtype=torch.uint8, device=dev)
    dst_buf = torch.empty(nb, dtype=torch.uint8, device=dev)
    for _ in range(2):
        L.wilson_stream_copy(ctx, dst_buf, src_buf, nb)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        L.wilson_stream_copy(ctx, dst_buf, src_buf, nb)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * nb / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src_buf, dst_buf
    L.wilson_context_destroy(ctx)
    best = next(r for r in rows if r["layout"] == "soa" and r["precision"] == "fp64" and r["link_reals"] == 12)
    return {
        "metric": "parity-hop GB/s (algorithmic bytes) by storage layout",
        "value": best["gbs_algorithmic"], "unit": "GB/s", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": best["us_per_launch"] / 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64/f32", "data": "synthetic",
        "config": {"workload": "layout ablation of the parity hop (value: site-per-lane planes, FP64, 12-real "
                               "links), 32^3x64, kappa=0.125, eps=0.3", "dims": list(dims)},
        "layouts": rows, "production_hop": prod, "hbm_copy_gbs": copy_gbs, "ablation_seconds": elapsed,
    }


# the host CPUs this process may use, read before any OpenMP region (with OMP_PROC_BIND the
# runtime then binds the main thread to one place)
AFFINITY_AT_START = len(os.sched_getaffinity(0))


def host_info(nthr):
    host = {"cpu_model": None, "logical_cpus": os.cpu_count(), "cpus_in_affinity": AFFINITY_AT_START,
            "omp_threads_used": nthr, "omp_proc_bind": os.environ.get("OMP_PROC_BIND"),
            "omp_places": os.environ.get("OMP_PLACES")}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    host["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return host


def cpu_baseline(args, U, b, kappa, tol, dims, nrhs, precision, it_gpu, F=None, check=None, block=False):
    """The FP64 oracle timed on the host's cores.  Plain FP64 Wilson workloads with one
    right-hand side up to 32^3x64: a full even-odd BiCGStab solve of the same problem to the
    same tolerance (value = 1 / its time), on one core too when it takes under half a
    second; others: setup + per-iteration cost x the GPU's iteration count (the difference
    of a 1- and a (1+k)-iteration run, about `--cpu-seconds` of work).  Also the operator
    units (parity hop with all threads and with one, full D) and the host triad.  With `check` (GPU results copied to the host: a solution x of
    right-hand side xb, and an operator output dout of input din with its parity dpar), the
    oracle's FP64 operator also grades them (outside the timed region)."""
    import numpy as np

    import oracle
    from paper_1811_00893_amd import counts
    Un = U.cpu().numpy()
    bn = (b[0] if nrhs > 1 else b).cpu().numpy()
    Fn = None if F is None else F.cpu().numpy()

    def solve(t, iters):
        if block:  # the oracle's block BiCGStab on all the right-hand sides
            return oracle.solve_block(b.cpu().numpy(), Un, kappa, dims, t, iters, F=Fn)
        if Fn is None:
            return oracle.solve(bn, Un, kappa, dims, t, iters, "bicgstab_eo")
        return oracle.solve_clov(bn, Un, Fn, kappa, dims, t, iters, "bicgstab_eo")

    full = None
    nthr = oracle.num_threads()
    V = int(np.prod(dims))
    one = more = 0.0
    k_it = 0
    per_iter = setup = None
    if not block and Fn is None and nrhs == 1 and precision == 0 and V <= (1 << 21):
        # the plain FP64 workloads up to 32^3x64: one full solve (about 10 s at 32^3x64)
        t1 = time.perf_counter()
        _, st, tres = solve(tol, 20000)
        full = {"seconds": time.perf_counter() - t1, "iterations": st, "true_residual": tres}
    else:
        t1 = time.perf_counter()
        solve(0.0, 1)
        one = time.perf_counter() - t1
        k_it = max(2, min(40, int(args.cpu_seconds / max(one, 1e-3))))
        t1 = time.perf_counter()
        solve(0.0, 1 + k_it)
        more = time.perf_counter() - t1
        per_iter = max(more - one, 1e-9) / k_it
        setup = max(one - per_iter, 0.0)

    def best_of(fn, n=3):
        ts = []
        for _ in range(n):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return min(ts)

    hop_s = best_of(lambda: oracle.dslash(bn, Un, kappa, dims, 0))
    if Fn is None:
        d_s = best_of(lambda: oracle.apply_D(bn, Un, kappa, dims))
    else:
        d_s = best_of(lambda: oracle.apply_Dclov(bn, Un, Fn, kappa, dims))
    oracle.set_threads(1)
    try:
        hop1_s = best_of(lambda: oracle.dslash(bn, Un, kappa, dims, 0), n=1)
        one_core_full = None
        if full is not None and full["seconds"] < 0.5:  # small lattices: the whole solve on one core
            t1 = time.perf_counter()
            solve(tol, 20000)
            one_core_full = time.perf_counter() - t1
    finally:
        oracle.set_threads(nthr)
    triad = oracle.triad_gbps()
    graded = None
    if check is not None:
        xr, xbr, dout, din, dpar = check
        if Fn is None:
            dx = oracle.apply_D(xr, Un, kappa, dims)
            dref = oracle.dslash(din, Un, kappa, dims, dpar) if dpar < 2 else oracle.apply_D(din, Un, kappa, dims)
        else:
            dx = oracle.apply_Dclov(xr, Un, Fn, kappa, dims)
            dref = oracle.apply_Dclov(din, Un, Fn, kappa, dims)
        graded = {
            "solution_residual_by_oracle": float(np.linalg.norm(xbr - dx) / np.linalg.norm(xbr)),
            "operator_rel_error_vs_oracle": float(np.linalg.norm(dout - dref) / np.linalg.norm(dref)),
            "operator": ("D_clov" if Fn is not None else ("parity hop" if dpar < 2 else "D")) +
                        f" in the workload's precision ({['fp64', 'fp32', 'fp16', 'fp16 spinors + fp32 links'][precision]})",
        }
    what = ("the same right-hand side" if nrhs == 1 else
            f"all {nrhs} right-hand sides in the oracle's block BiCGStab" if block else
            f"right-hand side 0 of the {nrhs}, the batch costed as {nrhs} sequential solves")
    inner = "" if precision == 0 else " (the GPU's inner iterations in reduced precision; the oracle is FP64)"
    if full is not None:
        value = 1.0 / full["seconds"]
        sample = (f"FP64 oracle even-odd BiCGStab on {list(dims)}, {what}, one full solve to tol {tol:g} "
                  f"({full['iterations']} iterations, {full['seconds']:.1f} s)")
    else:
        value = (nrhs if block else 1.0) / (setup + per_iter * it_gpu)
        sample = (f"FP64 oracle even-odd {'block ' if block else ''}BiCGStab"
                  f"{' (clover matrix)' if Fn is not None else ''} on {list(dims)}, {what}, run for 1 and "
                  f"{1 + k_it} iterations ({one + more:.1f} s of CPU work); solve time = setup + per-iteration "
                  f"cost x the {it_gpu:.0f} iterations the GPU solve needed{inner}")
    return {
        "value": value,
        "unit": "solves/s",
        "cores": nthr,
        "kind": "oracle",
        "sample": sample,
        "full_solve": full,
        "seconds_per_iteration": per_iter,
        "setup_seconds": setup,
        "one_core": {"solve_s": one_core_full, "parity_hop_s": hop1_s},
        "units": {
            "parity_hop_s": hop_s,
            "parity_hop_gbs_algorithmic": (V // 2) * counts.hop_bytes_per_site("fp64") / hop_s / 1e9,
            "full_d_s": d_s,
            "full_d_gflops": (counts.FULL_D_FLOPS_PER_SITE if Fn is None else counts.CLOVER_FLOPS_PER_SITE) * V / d_s / 1e9,
            "host_triad_gbs": triad,
        },
        "gpu_results_graded_by_oracle": graded,
        "host": host_info(nthr),
    }


def probes(L, ctx, dev):
    """HBM references: a plain streaming copy and a read of 2 GiB (GB/s)."""
    import torch
    nb = 1 << 31
    src_buf = torch.empty(nb, dtype=torch.uint8, device=dev)
    dst_buf = torch.empty(nb, dtype=torch.uint8, device=dev)
    for _ in range(2):
        L.wilson_stream_copy(ctx, dst_buf, src_buf, nb)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        L.wilson_stream_copy(ctx, dst_buf, src_buf, nb)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * nb / (e0.elapsed_time(e1) * 1e-3) / 1e9
    for _ in range(2):
        L.wilson_stream_read(ctx, src_buf, nb)
    e0.record()
    for _ in range(10):
        L.wilson_stream_read(ctx, src_buf, nb)
    e1.record()
    torch.cuda.synchronize()
    read_gbs = 10 * nb / (e0.elapsed_time(e1) * 1e-3) / 1e9
    return copy_gbs, read_gbs


def measure(args, name, steps, warmup, lat_samples, dslash_reps, with_cpu, full_d=True, host_lat=0,
            compare=True):
    """One workload: Dslash-only timing of the parity hop (the dominant kernel) with its
    roofline fractions, `steps` timed solves after `warmup` (the timed region: sources and
    links resident in HBM), a separate latency pass of `lat_samples` solves (p50 / p99 of
    the call; the solution in HBM when it returns), optionally `host_lat` solves whose
    solution is also copied to pinned host memory (latency to x on the host), the hop and
    vector-kernel figures of solves run with event timing, the comparisons (sequential
    single-RHS solves, the plain FP64 solver on the same problem, the lockstep solver for
    block workloads) and the CPU oracle."""
    import numpy as np
    import torch

    from paper_1811_00893_amd import _lib as L
    from paper_1811_00893_amd import counts, inputs

    dims, kappa, tol, precision, nrhs, desc = WORKLOADS[name]
    dev = torch.device("cuda:0")
    V = int(np.prod(dims))
    Vh = V // 2
    t_setup = time.perf_counter()
    U = inputs.gauge_field(dims, eps=0.3, seed=1002, device=dev)
    nsrc = max(steps + warmup, 2)
    if nrhs == 1:
        srcs = [inputs.gaussian_source(dims, seed=2002 + i, device=dev) for i in range(nsrc)]
    else:
        pts = inputs.point_sources(dims, device=dev)
        srcs = [pts for _ in range(nsrc)]
    x = torch.zeros_like(srcs[0])
    ctx = L.wilson_context_create()
    gbits = L.WILSON_GAUGE_FP32 | (L.WILSON_GAUGE_FP16 if precision == 2 else 0)
    g = L.wilson_gauge_load(ctx, U, dims, gbits)
    clover = name in CLOVER
    F = None
    if clover:
        F = inputs.clover_field(dims, c=0.05, seed=1005, device=dev)
        L.check(L.wilson_gauge_attach_clover(ctx, g, F, dims), "attach clover")
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    opts = {"precision": precision, "maxiter": 20000, "mixed_update": 1 if name in RELIABLE else 0,
            "solver": L.WILSON_SOLVER_BLOCK_BICGSTAB_EO if name in BLOCK else L.WILSON_SOLVER_BICGSTAB_EO,
            "inner_tol": args.inner_tol}

    # ---- Dslash only: plain parity hop on resident fields (in the workload's inner
    # precision); for the clover matrix the hops of D_clov on both parities ----
    dprec = precision
    dpar = 2 if clover else 0
    psi = srcs[0]  # all right-hand sides of the workload in one launch
    out = torch.zeros_like(psi)
    for _ in range(3):
        L.check(L.wilson_dslash_ex(ctx, g, out, psi, kappa, dpar, dprec, nrhs), "dslash")
    torch.cuda.synchronize()
    L.wilson_timing_enable(ctx, True)
    for _ in range(dslash_reps):
        L.check(L.wilson_dslash_ex(ctx, g, out, psi, kappa, dpar, dprec, nrhs), "dslash")
    torch.cuda.synchronize()
    d_ms, d_n, d_bytes = L.wilson_timing_read(ctx, L.WILSON_KERNEL_HOP)
    L.wilson_timing_enable(ctx, False)
    d_us = 1e3 * d_ms / max(d_n, 1)
    d_gbs = d_bytes / (d_ms * 1e-3) / 1e9
    sname = {0: "fp64", 1: "fp32", 2: "fp16", 3: "fp16"}[dprec]
    lname = {0: "fp64", 1: "fp32", 2: "fp16", 3: "fp32"}[dprec]
    per_launch = d_bytes / max(d_n, 1)
    # bytes the kernel must move with its link storage: SU(3) links keep 12 of 18 reals
    floor_launch = per_launch - (2 if clover else 1) * Vh * 8 * 6 * counts.REAL_BYTES[lname]
    dslash = {
        "precision": sname,
        "link_precision": lname,
        "nrhs": nrhs,
        "us_per_launch": d_us,
        "launches": d_n,
        "algorithmic_bytes_per_launch": per_launch,
        "floor_bytes_per_launch": floor_launch,
        "bytes_per_site": per_launch / Vh,
        "gbs": d_gbs,
        "frac_hbm_peak": d_gbs / counts.MI355X_HBM_GBS,
        "frac_floor": floor_launch / (d_us * 1e-6) / 1e9 / counts.MI355X_HBM_GBS,
        "gflops": (counts.CLOVER_FLOPS_PER_SITE if clover else counts.HOP_FLOPS_PER_SITE) * Vh * nrhs
                  / (d_us * 1e-6) / 1e9,
        "working_set_mb": per_launch / 1e6,
    }
    if clover:  # both hops of one D_clov application, with the paper's ideal byte count
        per_app = 1e-6 * d_us * 2
        dslash["d_clov"] = {
            "us_per_application": 2 * d_us,
            "gflops_1944": counts.CLOVER_FLOPS_PER_SITE * V * nrhs / per_app / 1e9,
            "gbs_ideal_count": counts.clover_full_bytes_per_site(lname if lname != "fp16" else "fp32") * V / per_app / 1e9,
        }
    fd = None
    if full_d and not args.dslash_only and not clover:
        for _ in range(2):
            L.check(L.wilson_dslash_ex(ctx, g, out, psi, kappa, 2, dprec, nrhs), "full D")
        torch.cuda.synchronize()
        L.wilson_timing_enable(ctx, True)
        reps_d = max(dslash_reps // 2, 1)
        for _ in range(reps_d):
            L.check(L.wilson_dslash_ex(ctx, g, out, psi, kappa, 2, dprec, nrhs), "full D")
        torch.cuda.synchronize()
        f_ms, f_n, f_bytes = L.wilson_timing_read(ctx, L.WILSON_KERNEL_HOP)
        L.wilson_timing_enable(ctx, False)
        f_us = 1e3 * f_ms / reps_d
        # the paper's count for D: each link, input and output read or written once per site
        ideal_site = 4 * counts.link_bytes(lname) + nrhs * 2 * counts.spinor_site_bytes(sname)
        fd = {
            "us_per_application": f_us,
            "hop_launches_per_application": f_n / reps_d,
            "gflops": counts.FULL_D_FLOPS_PER_SITE * V * nrhs / (f_us * 1e-6) / 1e9,
            "ideal_bytes_per_site": ideal_site,
            "gbs_ideal_count": ideal_site * V / (f_us * 1e-6) / 1e9,
            "gbs_launch_count": f_bytes / (f_ms * 1e-3) / 1e9,
        }
    dslash["full_d"] = fd
    del out
    traffic = committed_traffic(name, dslash)
    roofline = {
        "bound": "hbm",
        "kernel": (f"parity hop of D_clov (T x - kappa H x), {sname} spinors, {list(dims)}" if clover else
                   f"parity hop (Dslash D_eo = -kappa H_eo), {sname} spinors, {lname} links, {nrhs} RHS, "
                   f"{list(dims)}"),
        "achieved": d_gbs,
        "peak": counts.MI355X_HBM_GBS,
        "unit": "GB/s",
        "frac": d_gbs / counts.MI355X_HBM_GBS,
        "traffic": traffic,
        "algorithmic_bytes_per_launch": per_launch,
        "us_per_launch": d_us,
        # the same time against the bytes the kernel must move with two-row (12-real) links,
        # and against the HBM bytes the counters measured (when the summary is current)
        "floor_bytes_per_launch": floor_launch,
        "frac_floor": dslash["frac_floor"],
        "frac_counter": (traffic / (d_us * 1e-6) / 1e9 / counts.MI355X_HBM_GBS) if traffic else None,
        "frac_basis": "frac counts each link as 18 reals (Table 1's convention, the >= 70 % target); frac_floor "
                      "counts the 12 reals the two-row link storage reads; frac_counter uses the measured traffic",
    }
    if args.dslash_only:
        L.wilson_gauge_free(ctx, g)
        L.wilson_context_destroy(ctx)
        return {"dslash": dslash, "roofline": roofline, "setup_s": setup_s}

    # ---- solves: the timed region ----
    kap = [kappa] * nrhs
    tl = [tol] * nrhs
    for i in range(warmup):
        x.zero_()
        st, info = L.wilson_solve_ex(ctx, g, x, srcs[i], nrhs, kap, tl, opts)
        L.check(st, "warmup solve")
    torch.cuda.synchronize()
    iters, res, cycles = [], [], []
    t0 = time.perf_counter()
    for i in range(steps):
        st, info = L.wilson_solve_ex(ctx, g, x, srcs[warmup + i], nrhs, kap, tl, opts)
        if st != 0:
            raise RuntimeError(f"solve {i} returned {st}: {L.wilson_last_error()}")
        iters.append(max(d["iterations"] for d in info))
        cycles.append(max(d["outer_cycles"] for d in info))
        res.append(max(d["true_residual"] for d in info))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    x_last = (x[0] if nrhs > 1 else x).cpu().numpy()
    # ---- latency: a separate pass, every call timed on its own ----
    lat = []
    for i in range(lat_samples):
        s0 = time.perf_counter()
        st, _ = L.wilson_solve_ex(ctx, g, x, srcs[(warmup + i) % nsrc], nrhs, kap, tl, opts)
        lat.append(time.perf_counter() - s0)
        L.check(st, "latency solve")
    lat_host = []
    if host_lat:
        xh = torch.empty(x.shape, dtype=x.dtype, pin_memory=True)
        for i in range(host_lat):
            s0 = time.perf_counter()
            L.check(L.wilson_solve_ex(ctx, g, x, srcs[(warmup + i) % nsrc], nrhs, kap, tl, opts)[0], "solve")
            xh.copy_(x)
            lat_host.append(time.perf_counter() - s0)
    # per-kernel figures from a separate pass with event timing on
    n_prof = min(steps, 3)
    L.wilson_timing_enable(ctx, True)
    tp0 = time.perf_counter()
    for i in range(n_prof):
        L.check(L.wilson_solve_ex(ctx, g, x, srcs[warmup + i], nrhs, kap, tl, opts)[0], "profiled solve")
    torch.cuda.synchronize()
    prof_total = time.perf_counter() - tp0
    h_ms, h_n, h_bytes = L.wilson_timing_read(ctx, L.WILSON_KERNEL_HOP)
    b_ms, b_n, b_bytes = L.wilson_timing_read(ctx, L.WILSON_KERNEL_BLAS)
    L.wilson_timing_enable(ctx, False)
    solves = steps * nrhs
    hop_gbs = h_bytes / (h_ms * 1e-3) / 1e9
    solve_hops = {
        "launches": h_n,
        "us_per_launch": 1e3 * h_ms / max(h_n, 1),
        "algorithmic_gbs": hop_gbs,
        "frac_hbm_peak": hop_gbs / counts.MI355X_HBM_GBS,
        "hop_time_fraction": h_ms / (prof_total * 1e3),
        "solves_profiled": n_prof,
        "blas_gbs": b_bytes / (b_ms * 1e-3) / 1e9 if b_ms > 0 else None,
        "blas_time_fraction": b_ms / (prof_total * 1e3),
    }

    sequential = fp64_same = lockstep = None
    if compare and nrhs > 1 and name not in BLOCK:  # the same right-hand sides one at a time
        seq_t = []
        for i in range(min(steps, 3)):
            s0 = time.perf_counter()
            for k in range(nrhs):
                xk = torch.zeros_like(srcs[0][k])
                st, _ = L.wilson_solve_ex(ctx, g, xk, srcs[0][k].contiguous(), 1, kappa, tol,
                                          dict(opts, solver=L.WILSON_SOLVER_BICGSTAB_EO))
                L.check(st, "sequential solve")
            torch.cuda.synchronize()
            seq_t.append(time.perf_counter() - s0)
        sequential = {"value": nrhs / float(np.median(seq_t)), "unit": "solves/s",
                      "ms_per_batch": 1e3 * float(np.median(seq_t)),
                      "speedup_of_batched": (solves / total) / (nrhs / float(np.median(seq_t)))}
    if compare and precision != 0:  # the same problem with the plain FP64 solver
        f_lat, f_it = [], []
        fopts = dict(opts, precision=0, mixed_update=0)
        x.zero_()
        L.check(L.wilson_solve_ex(ctx, g, x, srcs[0], nrhs, kap, tl, fopts)[0], "FP64 warm-up solve")
        torch.cuda.synchronize()
        nref = max(min(steps, 5), 2)
        for i in range(nref):
            s0 = time.perf_counter()
            st, info = L.wilson_solve_ex(ctx, g, x, srcs[(warmup + i) % nsrc], nrhs, kap, tl, fopts)
            f_lat.append(time.perf_counter() - s0)
            L.check(st, "FP64 solve")
            f_it.append(max(d["iterations"] for d in info))
        f_val = nref * nrhs / sum(f_lat)
        fp64_same = {"value": f_val, "unit": "solves/s", "p50_ms": 1e3 * percentile(f_lat, 50),
                     "p99_ms": 1e3 * percentile(f_lat, 99), "iterations_median": float(np.median(f_it)),
                     "solves": nref, "gain_solves_per_s": (solves / total) / f_val,
                     "gain_p99": percentile(f_lat, 99) / percentile(lat, 99)}
    if compare and name in BLOCK:  # one BiCGStab recurrence per right-hand side, shared launches
        l_lat, l_it = [], []
        lopts = dict(opts, solver=L.WILSON_SOLVER_BICGSTAB_EO)
        x.zero_()
        L.check(L.wilson_solve_ex(ctx, g, x, srcs[0], nrhs, kap, tl, lopts)[0], "lockstep warm-up solve")
        torch.cuda.synchronize()
        nref = max(min(steps, 5), 2)
        for i in range(nref):
            s0 = time.perf_counter()
            st, info = L.wilson_solve_ex(ctx, g, x, srcs[(warmup + i) % nsrc], nrhs, kap, tl, lopts)
            l_lat.append(time.perf_counter() - s0)
            L.check(st, "lockstep solve")
            l_it.append(max(d["iterations"] for d in info))
        l_val = nref * nrhs / sum(l_lat)
        lockstep = {"value": l_val, "unit": "solves/s", "ms_per_batch": 1e3 * float(np.median(l_lat)),
                    "iterations_median": float(np.median(l_it)), "batches": nref,
                    "gain_of_block": (solves / total) / l_val,
                    "iteration_ratio": float(np.median(l_it)) / float(np.median(iters))}

    cpu = None
    if with_cpu:
        j = warmup + steps - 1
        xbr = (srcs[j][0] if nrhs > 1 else srcs[j]).cpu().numpy()
        gpar = 2 if nrhs > 1 else dpar  # a point source has one parity: grade the full D on it
        dout_t = torch.zeros_like(srcs[j][0] if nrhs > 1 else srcs[j])
        L.check(L.wilson_dslash_ex(ctx, g, dout_t, srcs[j][0].contiguous() if nrhs > 1 else srcs[j], kappa, gpar,
                                   dprec, 1), "graded dslash")
        dout = dout_t.cpu().numpy()
        cpu = cpu_baseline(args, U, srcs[0], kappa, tol, dims, nrhs, precision, float(np.median(iters)), F,
                           check=(x_last, xbr, dout, xbr, gpar), block=name in BLOCK)
    L.wilson_gauge_free(ctx, g)
    L.wilson_context_destroy(ctx)
    del U, srcs, x, F
    torch.cuda.empty_cache()
    return {
        "desc": desc, "dims": list(dims), "kappa": kappa, "tol": tol, "nrhs": nrhs, "precision": precision,
        "value": solves / total, "unit": "solves/s", "ms_per_step": 1e3 * total / steps, "steps": steps,
        "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99), "latency_samples": len(lat),
        "p50_to_host_ms": 1e3 * percentile(lat_host, 50) if lat_host else None,
        "p99_to_host_ms": 1e3 * percentile(lat_host, 99) if lat_host else None,
        "latency_to_host_samples": len(lat_host),
        "iterations_median": float(np.median(iters)), "outer_cycles_median": float(np.median(cycles)),
        "true_residual_max": max(res), "dslash": dslash, "roofline": roofline, "solve_hops": solve_hops,
        "cpu_baseline": cpu, "sequential_single_rhs": sequential, "fp64_same_problem": fp64_same,
        "lockstep_same_batch": lockstep, "setup_s": setup_s,
    }


# Configurations reported beside the headline (C2) in the default run: the small lattice,
# the three mixed-precision variants at 48^3x96 and the batched point sources.
EXTRAS = ["small8", "mixed48", "mixed48_fp16", "mixed48_fp16h", "batched24"]


def headline(r):
    """The figures of one configuration that the default line carries as an extra key."""
    out = {k: r[k] for k in ("desc", "dims", "nrhs", "value", "unit", "p50_ms", "p99_ms", "latency_samples",
                             "iterations_median", "outer_cycles_median", "true_residual_max")}
    ro = r["roofline"]
    out["hop"] = {"us_per_launch": ro["us_per_launch"], "frac": ro["frac"], "frac_floor": ro["frac_floor"],
                  "frac_counter": ro["frac_counter"], "cache_resident": ro["algorithmic_bytes_per_launch"] < 256e6}
    if r.get("fp64_same_problem"):
        f = r["fp64_same_problem"]
        out["plain_fp64_same_problem"] = {"value": f["value"], "p99_ms": f["p99_ms"],
                                          "gain_solves_per_s": f["gain_solves_per_s"], "gain_p99": f["gain_p99"]}
    if r.get("sequential_single_rhs"):
        out["sequential_single_rhs"] = r["sequential_single_rhs"]
    if r.get("cpu_baseline"):
        c = r["cpu_baseline"]
        out["cpu_oracle"] = {"value": c["value"], "cores": c["cores"], "sample": c["sample"],
                             "one_core_solve_s": c["one_core"]["solve_s"]}
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path (see the design notes on "
              "how the lattice would shard); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    # the oracle's OpenMP threads, one per core, placed close (read when its runtime starts)
    os.environ.setdefault("OMP_PROC_BIND", "close")
    os.environ.setdefault("OMP_PLACES", "cores")
    if args.workload == "serve":
        print(json.dumps(run_serving(args)), flush=True)
        return
    if args.workload == "layouts":
        print(json.dumps(run_layouts(args)), flush=True)
        return
    import torch

    from paper_1811_00893_amd import _lib as L
    r = measure(args, args.workload, args.steps, args.warmup, args.latency_samples, args.dslash_reps,
                with_cpu=not args.no_cpu and not args.dslash_only, host_lat=20)
    ctx = L.wilson_context_create()
    copy_gbs, read_gbs = probes(L, ctx, torch.device("cuda:0"))
    L.wilson_context_destroy(ctx)
    r["dslash"]["frac_of_copy_bw"] = r["dslash"]["gbs"] / copy_gbs
    r["roofline"]["frac_of_copy_bw"] = r["dslash"]["gbs"] / copy_gbs
    r["roofline"]["frac_of_read_bw"] = r["dslash"]["gbs"] / read_gbs
    if args.dslash_only:
        print(json.dumps({"dslash": r["dslash"], "roofline": r["roofline"], "hbm_copy_gbs": copy_gbs,
                          "hbm_read_gbs": read_gbs}), flush=True)
        return
    configs = {}
    if args.workload == "fp64_32" and not args.no_extras:
        for name in EXTRAS:
            small = name == "small8"
            print(f"[bench] configuration {name}", file=sys.stderr, flush=True)
            e = measure(args, name, 100 if small else 10, 2, 100 if small else args.extra_latency_samples,
                        20, with_cpu=small and not args.no_cpu, full_d=False)
            configs[name] = headline(e)
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if r["precision"] == 0 else "f64/f32",
        "data": "synthetic",
        "config": {"workload": r["desc"], "lattice": r["dims"], "kappa": r["kappa"], "tol": r["tol"], "eps": 0.3,
                   "nrhs": r["nrhs"],
                   "precision": ["fp64", "mixed_fp32", "mixed_fp16", "mixed_fp16_l32"][r["precision"]]},
        "p50_ms": r["p50_ms"],
        "p99_ms": r["p99_ms"],
        "latency_samples": r["latency_samples"],
        "latency_note": "p50/p99: separate pass, each call timed alone (solution in HBM when it returns); "
                        "*_to_host_ms: the same plus the copy of x to pinned host memory",
        "p50_to_host_ms": r["p50_to_host_ms"],
        "p99_to_host_ms": r["p99_to_host_ms"],
        "iterations_median": r["iterations_median"],
        "outer_cycles_median": r["outer_cycles_median"],
        "true_residual_max": r["true_residual_max"],
        "dslash": r["dslash"],
        "roofline": r["roofline"],
        "solve_hops": r["solve_hops"],
        "cpu_baseline": r["cpu_baseline"],
        "sequential_single_rhs": r["sequential_single_rhs"],
        "fp64_same_problem": r["fp64_same_problem"],
        "lockstep_same_batch": r["lockstep_same_batch"],
        "configs": configs or None,
        "hbm_copy_gbs": copy_gbs,
        "hbm_read_gbs": read_gbs,
        "setup_s": r["setup_s"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

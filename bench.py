"""Benchmark: Wilson-Dirac solves on one MI355X.

Default workload (one "step" = one whole solve): plain FP64 even-odd BiCGStab on a
32^3x64 lattice, links exp(i*0.3*A), kappa = 0.125, a complex Gaussian source per step,
relative residual 1e-10 (checked in FP64 after the iteration).  Sources and links are
resident in HBM before the timed region starts.

Printed: one JSON line with solves/s (value), p50/p99 latency, the achieved bandwidth of
the dominant kernel (the parity hop, measured with HIP events on the library's stream
over the timed region) against the MI355X HBM peak, a Dslash-only figure (parity hop
alone), and the CPU oracle timed on a bounded sample of the same workload.

Other workloads (not the headline line): --workload small8 | mixed48 | mixed48_fp16 | batched24 | serve.
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
    p.add_argument("--dslash-reps", type=int, default=50)
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--dslash-only", action="store_true", help="only the Dslash section and the copy probe")
    p.add_argument("--requests", type=int, default=40, help="serving: number of requests")
    p.add_argument("--load", type=float, default=0.8, help="serving: offered load / FIFO capacity")
    p.add_argument("--step-iters", type=int, default=8, help="serving: iterations per scheduler turn")
    p.add_argument("--hbm-budget", type=float, default=200e9, help="serving: device bytes for fields + batches")
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
}


def run_serving(args):
    """Serving: a Poisson stream of solve requests over four lattice sizes, each request on
    one of two seeded gauge fields per size (eps ~ U[0.2, 0.4]), kappa ~ U[0.115, 0.125],
    tol in {1e-8, 1e-10, 1e-12}, 1-12 Gaussian right-hand sides; mixed precision (FP32 inner,
    FP64 outer).  The same trace is first served one request at a time (FIFO, the plain
    path) to measure its capacity; arrivals are then generated at `--load` x that capacity
    and replayed through the continuous-batching server.  Latency = arrival -> solution in
    device memory.  FIFO latencies on the same arrivals follow from its measured service
    times (one request at a time)."""
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
    U = {gid: inputs.gauge_field(d, eps=e, seed=s, device=dev) for gid, (d, e, s) in pool.items()}
    B = [inputs.gaussian_source(pool[t["gid"]][0], seed=t["seed"], nrhs=t["nrhs"], device=dev) for t in trace]
    opts = {"precision": 1, "maxiter": 100000}

    # FIFO: one request at a time through wilson_solve_ex (all its RHS together)
    ctx = L.wilson_context_create()
    G = {gid: L.wilson_gauge_load(ctx, U[gid], pool[gid][0], L.WILSON_GAUGE_FP32) for gid in pool}
    def fifo_once(i):
        t = trace[i]
        x = torch.zeros_like(B[i])
        st, info = L.wilson_solve_ex(ctx, G[t["gid"]], x, B[i], t["nrhs"], t["kappa"], t["tol"], opts)
        L.check(st, "fifo solve")
    for i in range(min(4, nreq)):  # warm the tuner
        fifo_once(i)
    service = []
    torch.cuda.synchronize()
    for i in range(nreq):
        s0 = time.perf_counter()
        fifo_once(i)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - s0)
    for g in G.values():
        L.wilson_gauge_free(ctx, g)
    L.wilson_context_destroy(ctx)
    fifo_total = sum(service)
    cap = nreq / fifo_total
    lam = args.load * cap
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=nreq))
    # FIFO latencies on these arrivals
    t_free, fifo_lat = 0.0, []
    for a, sv in zip(arrivals, service):
        start = max(a, t_free)
        t_free = start + sv
        fifo_lat.append(t_free - a)

    # continuous batching
    sch, eng = make_server(hbm_budget=args.hbm_budget, nslots=12, step_iters=args.step_iters, precision=1)
    for gid, (d, e, s) in pool.items():
        sch.register_gauge(gid, d, eng.load_gauge(gid, U[gid], d))
    warm = Request(rid=-1, gauge_id=(0, 0), kappa=0.12, tol=1e-10, b=B[0][:1].contiguous())
    sch.submit(warm)
    sch.run_until_idle()
    sch.completed.clear()
    reqs = [Request(rid=i, gauge_id=t["gid"], kappa=t["kappa"], tol=t["tol"], b=B[i], maxiter=100000)
            for i, t in enumerate(trace)]
    eng.alloc_solution = lambda req: torch.zeros_like(req.b)
    t0 = time.perf_counter()
    sch.clock = lambda: time.perf_counter() - t0
    nxt = 0
    while nxt < nreq or sch.busy():
        now = sch.clock()
        while nxt < nreq and arrivals[nxt] <= now:
            reqs[nxt].arrival = float(arrivals[nxt])
            sch.submit(reqs[nxt])
            nxt += 1
        if sch.busy():
            sch.admit()
            sch.step()
        elif nxt < nreq:
            time.sleep(max(0.0, min(arrivals[nxt] - now, 0.01)))
    wall = sch.clock()
    sch.close()
    eng.close()
    lat = [r.latency for r in sch.completed]
    bad = [r.rid for r in sch.completed if any(st != 0 for st in r.status)]
    rhs = sum(t["nrhs"] for t in trace)
    return {
        "metric": METRIC, "workload": "serving", "unit": "solves/s",
        "value": rhs / wall,
        "requests": nreq, "rhs": rhs, "offered_load": args.load, "arrival_rate_per_s": lam,
        "served_p50_ms": 1e3 * percentile(lat, 50), "served_p99_ms": 1e3 * percentile(lat, 99),
        "requests_per_s": nreq / wall,
        "fifo_capacity_rhs_per_s": rhs / fifo_total,
        "fifo_p50_ms": 1e3 * percentile(fifo_lat, 50), "fifo_p99_ms": 1e3 * percentile(fifo_lat, 99),
        "failed_requests": bad, "rejected": len(sch.rejected),
        "config": {"lattices": sizes, "gauge_fields_per_size": 2, "nslots": 12, "step_iters": args.step_iters,
                   "precision": "mixed_fp32", "latency": "arrival to solution in device memory"},
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path (see the design notes on "
              "how the lattice would shard); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        print(json.dumps(run_serving(args)), flush=True)
        return
    import numpy as np
    import torch

    from paper_1811_00893_amd import _lib as L
    from paper_1811_00893_amd import counts, inputs

    dims, kappa, tol, precision, nrhs, desc = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    V = int(np.prod(dims))
    Vh = V // 2
    t_setup = time.perf_counter()
    U = inputs.gauge_field(dims, eps=0.3, seed=1002, device=dev)
    nsrc = args.steps + args.warmup
    if nrhs == 1:
        srcs = [inputs.gaussian_source(dims, seed=2002 + i, device=dev) for i in range(nsrc)]
    else:
        pts = inputs.point_sources(dims, device=dev)
        srcs = [pts for _ in range(nsrc)]
    x = torch.zeros_like(srcs[0])
    ctx = L.wilson_context_create()
    gbits = L.WILSON_GAUGE_FP32 | (L.WILSON_GAUGE_FP16 if precision == 2 else 0)
    g = L.wilson_gauge_load(ctx, U, dims, gbits)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    opts = {"precision": precision, "maxiter": 20000}

    # ---- Dslash only: plain parity hop on resident fields (FP64 for the FP64 workload) ----
    dprec = precision  # the workload's inner precision
    psi = srcs[0]  # all right-hand sides of the workload in one launch
    out = torch.zeros_like(psi)
    for _ in range(3):
        L.check(L.wilson_dslash_ex(ctx, g, out, psi, kappa, 0, dprec, nrhs), "dslash")
    torch.cuda.synchronize()
    L.wilson_timing_enable(ctx, True)
    for _ in range(args.dslash_reps):
        L.check(L.wilson_dslash_ex(ctx, g, out, psi, kappa, 0, dprec, nrhs), "dslash")
    torch.cuda.synchronize()
    d_ms, d_n, d_bytes = L.wilson_timing_read(ctx, L.WILSON_KERNEL_HOP)
    L.wilson_timing_enable(ctx, False)
    d_us = 1e3 * d_ms / max(d_n, 1)
    d_gbs = d_bytes / (d_ms * 1e-3) / 1e9
    sname = {0: "fp64", 1: "fp32", 2: "fp16", 3: "fp16"}[dprec]
    lname = {0: "fp64", 1: "fp32", 2: "fp16", 3: "fp32"}[dprec]
    dslash = {
        "precision": sname,
        "nrhs": nrhs,
        "us_per_launch": d_us,
        "launches": d_n,
        "algorithmic_bytes_per_launch": d_bytes / max(d_n, 1),
        "bytes_per_site": 8 * counts.link_bytes(lname) + nrhs * 2 * counts.spinor_site_bytes(sname),
        "gbs": d_gbs,
        "frac_hbm_peak": d_gbs / counts.MI355X_HBM_GBS,
        "gflops": counts.HOP_FLOPS_PER_SITE * Vh * nrhs / (d_us * 1e-6) / 1e9,
        "working_set_mb": d_bytes / max(d_n, 1) / 1e6,
    }

    # ---- HBM reference: a plain streaming copy of 2 GiB (not the workload) ----
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
    del src_buf, dst_buf
    dslash["frac_of_copy_bw"] = d_gbs / copy_gbs
    if args.dslash_only:
        print(json.dumps({"dslash": dslash, "hbm_copy_gbs": copy_gbs, "hbm_read_gbs": read_gbs}), flush=True)
        return

    # ---- solves ----
    kap = [kappa] * nrhs
    tl = [tol] * nrhs
    for i in range(args.warmup):
        x.zero_()
        st, info = L.wilson_solve_ex(ctx, g, x, srcs[i], nrhs, kap, tl, opts)
        L.check(st, "warmup solve")
    torch.cuda.synchronize()
    lat, iters, res, cycles = [], [], [], []
    L.wilson_timing_enable(ctx, True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        s0 = time.perf_counter()
        st, info = L.wilson_solve_ex(ctx, g, x, srcs[args.warmup + i], nrhs, kap, tl, opts)
        lat.append(time.perf_counter() - s0)
        if st != 0:
            raise RuntimeError(f"solve {i} returned {st}: {L.wilson_last_error()}")
        iters.append(max(d["iterations"] for d in info))
        cycles.append(max(d["outer_cycles"] for d in info))
        res.append(max(d["true_residual"] for d in info))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    h_ms, h_n, h_bytes = L.wilson_timing_read(ctx, L.WILSON_KERNEL_HOP)
    b_ms, b_n, b_bytes = L.wilson_timing_read(ctx, L.WILSON_KERNEL_BLAS)
    L.wilson_timing_enable(ctx, False)
    solves = args.steps * nrhs
    hop_gbs = h_bytes / (h_ms * 1e-3) / 1e9
    traffic = committed_traffic(args.workload, dslash)
    roofline = {
        "bound": "hbm",
        "kernel": f"parity hop (Dslash D_eo = -kappa H_eo), {sname} spinors, {nrhs} RHS, {list(dims)}",
        "achieved": d_gbs,
        "peak": counts.MI355X_HBM_GBS,
        "unit": "GB/s",
        "frac": d_gbs / counts.MI355X_HBM_GBS,
        "traffic": traffic,
        "algorithmic_bytes_per_launch": dslash["algorithmic_bytes_per_launch"],
        "us_per_launch": d_us,
        "frac_of_copy_bw": d_gbs / copy_gbs,
        "frac_of_read_bw": d_gbs / read_gbs,
    }
    solve_hops = {
        "launches": h_n,
        "us_per_launch": 1e3 * h_ms / max(h_n, 1),
        "algorithmic_gbs": hop_gbs,
        "frac_hbm_peak": hop_gbs / counts.MI355X_HBM_GBS,
        "hop_time_fraction": h_ms / (total * 1e3),
        "blas_gbs": b_bytes / (b_ms * 1e-3) / 1e9 if b_ms > 0 else None,
        "blas_time_fraction": b_ms / (total * 1e3),
    }

    # ---- batched workloads: the same right-hand sides solved one at a time ----
    sequential = None
    if nrhs > 1:
        seq_t = []
        for i in range(min(args.steps, 3)):
            s0 = time.perf_counter()
            for k in range(nrhs):
                xk = torch.zeros_like(srcs[0][k])
                st, _ = L.wilson_solve_ex(ctx, g, xk, srcs[0][k].contiguous(), 1, kappa, tol, opts)
                L.check(st, "sequential solve")
            torch.cuda.synchronize()
            seq_t.append(time.perf_counter() - s0)
        sequential = {"value": nrhs / float(np.median(seq_t)), "unit": "solves/s",
                      "ms_per_batch": 1e3 * float(np.median(seq_t)),
                      "speedup_of_batched": (solves / total) / (nrhs / float(np.median(seq_t)))}

    # ---- CPU oracle on a bounded sample of the same workload ----
    cpu = None
    if not args.no_cpu and nrhs == 1:
        import oracle
        Un = U.cpu().numpy()
        bn = srcs[0].cpu().numpy()
        # two runs of different length: their difference isolates the cost of an iteration
        t1 = time.perf_counter()
        oracle.solve(bn, Un, kappa, dims, 0.0, 1, "bicgstab_eo")
        one = time.perf_counter() - t1
        k_it = max(2, min(40, int(args.cpu_seconds / max(one, 1e-3))))
        t1 = time.perf_counter()
        oracle.solve(bn, Un, kappa, dims, 0.0, 1 + k_it, "bicgstab_eo")
        more = time.perf_counter() - t1
        per_iter = max(more - one, 1e-9) / k_it
        setup = max(one - per_iter, 0.0)
        it_per_solve = float(np.median(iters))
        cpu = {
            "value": 1.0 / (setup + per_iter * it_per_solve),
            "unit": "solves/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle even-odd BiCGStab on the same {dims} problem, run for 1 and {1 + k_it} "
                      f"iterations ({one + more:.1f} s of CPU work); solve time = setup + per-iteration cost x "
                      f"the {it_per_solve:.0f} iterations the GPU solve needed",
            "seconds_per_iteration": per_iter,
            "setup_seconds": setup,
        }
        del Un

    line = {
        "metric": METRIC,
        "value": solves / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f64/f32",
        "data": "synthetic",
        "config": {"workload": desc, "lattice": list(dims), "kappa": kappa, "tol": tol, "eps": 0.3,
                   "nrhs": nrhs, "precision": ["fp64", "mixed_fp32", "mixed_fp16", "mixed_fp16_l32"][precision]},
        "p50_ms": 1e3 * percentile(lat, 50),
        "p99_ms": 1e3 * percentile(lat, 99),
        "iterations_median": float(np.median(iters)),
        "outer_cycles_median": float(np.median(cycles)),
        "true_residual_max": max(res),
        "dslash": dslash,
        "roofline": roofline,
        "solve_hops": solve_hops,
        "cpu_baseline": cpu,
        "sequential_single_rhs": sequential,
        "hbm_copy_gbs": copy_gbs,
        "hbm_read_gbs": read_gbs,
        "setup_s": setup_s,
    }
    L.wilson_gauge_free(ctx, g)
    L.wilson_context_destroy(ctx)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

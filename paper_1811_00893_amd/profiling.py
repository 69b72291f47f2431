"""Summaries of rocprofv3 CSV output for the committed profile records.

  stats   : kernel-trace statistics (`rocprofv3 --kernel-trace --stats --output-format csv`)
            -> a short text table of the top kernels with the command that produced it.
  counters: per-dispatch means of the counters of several --pmc runs of the hop kernel.
  traffic : HBM bytes per launch of the hop kernel from two counter runs
            (`--pmc FETCH_SIZE`, `--pmc WRITE_SIZE`; values in KiB per dispatch), each
            calibrated by what the same counter reports for the library's streaming copy of
            2 GiB in the same run (FETCH_SIZE reports half the bytes read on this part).

Usage:
  python -m paper_1811_00893_amd.profiling stats --dir D --out F --command "..."
  python -m paper_1811_00893_amd.profiling traffic --workload W --fetch D1 --write D2 --out F --command "..." [--first N]
"""
import argparse
import csv
import glob
import json
import os
import sys

COPY_BYTES = 1 << 31  # the probe in bench.py copies 2 GiB


def _find(d, suffix):
    hits = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def short_name(name):
    n = name.replace("void ", "").replace("(anonymous namespace)::", "")
    return n.split("(")[0][:70]


def stats(d, out, command, top=14, match=None):
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    if match:  # only the kernels whose name contains `match` (percentages stay of the whole run)
        rows = [r for r in rows if match in r["Name"]]
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}", "",
             f"{'calls':>7} {'avg_us':>10} {'total_ms':>10} {'pct':>6}  kernel"]
    for r in rows[:top]:
        lines.append(f"{int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.1f} "
                     f"{float(r['TotalDurationNs']) / 1e6:10.2f} {100 * float(r['TotalDurationNs']) / total:6.1f}  "
                     f"{short_name(r['Name'])}")
    text = "\n".join(lines) + "\n"
    open(out, "w").write(text)
    return text


def _counter(d, kernel_substr, first):
    """Mean counter value over the first `first` dispatches of the kernel (bench.py's
    plain hop loop; the full-D launches that follow carry an extra input), and over the
    copy probe's dispatches."""
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    hits = [r for r in rows if kernel_substr in r["Kernel_Name"]][:first]
    kern = [float(r["Counter_Value"]) for r in hits]
    copy = [float(r["Counter_Value"]) for r in rows if "stream_copy_kernel" in r["Kernel_Name"]]
    if not kern or not copy:
        raise ValueError(f"{d}: kernel '{kernel_substr}' or the copy probe not found")
    return sum(kern) / len(kern), len(kern), sum(copy) / len(copy), hits[0]["Kernel_Name"]


def traffic(workload, fetch_dir, write_dir, out, command, first, kernel_substr="hop_kernel"):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench  # the hash of the kernel sources the counters describe
    f_kib, nf, f_copy_kib, name = _counter(fetch_dir, kernel_substr, first)
    w_kib, nw, w_copy_kib, _ = _counter(write_dir, kernel_substr, first)
    f_scale = COPY_BYTES / (f_copy_kib * 1024)   # bytes read per FETCH_SIZE byte
    w_scale = COPY_BYTES / (w_copy_kib * 1024)   # bytes written per WRITE_SIZE byte
    rec = {
        "kernel": short_name(name),
        "dispatches": [nf, nw],
        "fetch_kib_per_dispatch": f_kib,
        "write_kib_per_dispatch": w_kib,
        "copy_probe_fetch_kib": f_copy_kib,
        "copy_probe_write_kib": w_copy_kib,
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "fetch_bytes_per_launch": f_kib * 1024 * f_scale,
        "write_bytes_per_launch": w_kib * 1024 * w_scale,
        "kernel_source_hash": bench.kernel_source_hash(),
        "command": command,
    }
    db = json.load(open(out)) if os.path.exists(out) else {}
    db[workload] = rec
    json.dump(db, open(out, "w"), indent=1, sort_keys=True)
    return rec


def kernel_traffic(fetch_dir, write_dir, match, out, command):
    """FETCH_SIZE / WRITE_SIZE per dispatch, averaged over every dispatch of each kernel whose
    name contains `match`, calibrated by the copy probe of the same runs; one record per
    kernel name, written to `out` (a text table)."""
    def per_kernel(d):
        rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
        acc, copy = {}, []
        for r in rows:
            if "stream_copy_kernel" in r["Kernel_Name"]:
                copy.append(float(r["Counter_Value"]))
            elif match in r["Kernel_Name"]:
                acc.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        if not copy or not acc:
            raise ValueError(f"{d}: no '{match}' kernels or no copy probe")
        return {k: sum(v) / len(v) for k, v in acc.items()}, COPY_BYTES / (sum(copy) / len(copy) * 1024)
    f, fs = per_kernel(fetch_dir)
    w, ws = per_kernel(write_dir)
    lines = ["# rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch (two separate --pmc runs)",
             f"# command: {command}",
             f"# calibration: bytes per counted byte, from the 2 GiB copy probe of the same runs: "
             f"fetch {fs:.4f}, write {ws:.4f}", "",
             f"{'fetch_GB':>9} {'write_GB':>9}  kernel"]
    for k in sorted(f, key=lambda k: -f[k]):
        lines.append(f"{f[k] * 1024 * fs / 1e9:9.3f} {w.get(k, float('nan')) * 1024 * ws / 1e9:9.3f}  {k}")
    text = "\n".join(lines) + "\n"
    open(out, "w").write(text)
    return text


def counters(dirs, out, command, first=8, match="hop_kernel"):
    """Per-dispatch means of every counter in the `--pmc` runs `dirs` (label=dir pairs) over
    the first `first` dispatches of the kernel (bench.py --dslash-only: the plain hop
    launches), one block per label, with derived figures where the counters allow."""
    lines = ["# rocprofv3 counters per dispatch of the parity hop (mean over the first "
             f"{first} dispatches of each run)", f"# command: {command}", ""]
    for label, d in dirs:
        rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
        per = {}
        name = None
        for r in rows:
            if match in r["Kernel_Name"]:
                per.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
                name = name or short_name(r["Kernel_Name"])
        ids = sorted(per)[:first]
        avg = {k: sum(per[i][k] for i in ids) / len(ids) for k in per[ids[0]]}
        lines.append(f"[{label}] {name} ({len(ids)} dispatches)")
        for k in sorted(avg):
            lines.append(f"  {k:38s} {avg[k]:16.6g}")
        lines.append("")
    text = "\n".join(lines) + "\n"
    open(out, "w").write(text)
    return text


def main():
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("--dir", required=True)
    a.add_argument("--out", required=True)
    a.add_argument("--command", required=True)
    a.add_argument("--top", type=int, default=14, help="kernels listed (by total time)")
    a.add_argument("--match", default=None, help="list only kernels whose name contains this")
    c = sub.add_parser("kernel-traffic")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--match", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--command", required=True)
    k = sub.add_parser("counters")
    k.add_argument("--run", action="append", required=True, help="label=directory of one --pmc run")
    k.add_argument("--out", required=True)
    k.add_argument("--command", required=True)
    k.add_argument("--first", type=int, default=8)
    b = sub.add_parser("traffic")
    b.add_argument("--workload", required=True)
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--command", required=True)
    b.add_argument("--first", type=int, default=8,
                   help="plain-hop dispatches at the start (bench.py: 3 warm-up + --dslash-reps)")
    args = p.parse_args()
    if args.cmd == "stats":
        print(stats(args.dir, args.out, args.command, args.top, args.match))
    elif args.cmd == "counters":
        print(counters([tuple(r.split("=", 1)) for r in args.run], args.out, args.command, args.first))
    elif args.cmd == "kernel-traffic":
        print(kernel_traffic(args.fetch, args.write, args.match, args.out, args.command))
    else:
        print(json.dumps(traffic(args.workload, args.fetch, args.write, args.out, args.command, args.first), indent=1))


if __name__ == "__main__":
    main()

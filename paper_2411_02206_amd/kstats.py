"""Per-kernel durations of a bench run, from rocprofv3 --kernel-trace --stats.

    python -m paper_2411_02206_amd.kstats --workload frame --out profiles/kernels_frame.md

runs, as a child process (this process never touches the GPU),

    rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- \
        python3 -u bench.py --workload <w> --steps S --warmup W --no-cpu --gen-workers 1

and writes a short text summary: the exact command, the stats table rocprofv3
printed (calls, total, average, min, max per kernel), and the bench's own JSON
line (whose per-stage averages come from HIP events on the decode streams),
so the two can be compared.
"""
import argparse
import csv
import glob
import json
import os
import shutil
import subprocess
import sys
import time

from paper_2411_02206_amd.traffic import kernel_name

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="batched")
    ap.add_argument("--bench-args", default="", help="more bench.py arguments, e.g. '--frames-cache DIR'")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--work", default=os.path.join(ROOT, "rocprof_out", "kstats"),
                    help="folder for rocprofv3's raw output")
    ap.add_argument("--rocprof", default="rocprofv3")
    ap.add_argument("--timeout", type=float, default=300.0)
    args = ap.parse_args()
    if os.path.isdir(args.work):
        shutil.rmtree(args.work)
    prog = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", args.workload, "--steps",
            str(args.steps), "--warmup", str(args.warmup), "--no-cpu", "--no-plain", "--gen-workers", "1"] + args.bench_args.split()
    cmd = [args.rocprof, "--kernel-trace", "--stats", "--output-format", "csv", "-d", args.work, "-o", "run",
           "--"] + prog
    print("[kstats] " + " ".join(cmd), flush=True)
    t = time.perf_counter()
    r = subprocess.run(cmd, cwd=ROOT, env=dict(os.environ, TMPDIR="/tmp"), timeout=args.timeout,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    print(f"[kstats] exit {r.returncode} after {time.perf_counter() - t:.1f} s", flush=True)
    if r.returncode != 0:
        sys.stdout.write(r.stdout[-4000:])
        raise SystemExit(r.returncode)
    bench_line = None
    for line in r.stdout.splitlines():
        if line.startswith("{") and '"metric"' in line:
            bench_line = json.loads(line)
    files = glob.glob(os.path.join(args.work, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit("no kernel_stats.csv")
    rows = list(csv.DictReader(open(files[0])))

    def col(row, *names):
        low = {k.lower(): v for k, v in row.items()}
        for nm in names:
            if nm.lower() in low:
                return low[nm.lower()]
        raise KeyError(names)
    rel = ["python3"] + [os.path.relpath(p, ROOT) if p.startswith(ROOT) else p for p in prog[1:]]
    lines = [f"# Kernel durations, workload `{args.workload}`", "",
             "Made by `python -m paper_2411_02206_amd.kstats --workload "
             f"{args.workload} --out <this file>`, which runs:", "",
             "    rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- " + " ".join(rel), "",
             "rocprofv3 kernel statistics (durations in microseconds; the bench's own calls include warmup, "
             "timed, latency and per-stage event runs):", "",
             "| kernel | calls | total (us) | average (us) | min (us) | max (us) | share |",
             "|---|---|---|---|---|---|---|"]
    for row in rows:
        name = kernel_name(col(row, "Name", "KernelName"))
        us = lambda *k: float(col(row, *k)) / 1e3  # noqa: E731  (ns -> us)
        lines.append(f"| {name} | {col(row, 'Calls')} | {us('TotalDurationNs'):.1f} | {us('AverageNs'):.2f} | "
                     f"{us('MinNs'):.2f} | {us('MaxNs'):.2f} | {float(col(row, 'Percentage')):.1f}% |")
    if bench_line:
        lines += ["", "bench.py under the profiler (per-stage averages from HIP events, ms):", "",
                  "    " + json.dumps(bench_line.get("stage_avg_ms")),
                  f"    ms_per_step {bench_line.get('ms_per_step'):.4f}, value {bench_line.get('value'):.4g} "
                  f"{bench_line.get('unit')}"]
    text = "\n".join(lines) + "\n"
    print(text, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)


if __name__ == "__main__":
    main()

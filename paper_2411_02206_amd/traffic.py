"""Measured HBM traffic per kernel launch, from rocprofv3 counters.

    python -m paper_2411_02206_amd.traffic --workload frame --out profiles/traffic_frame.md

runs, each as a child process under rocprofv3 (this process never touches the
GPU):
  1. the bench on the workload with `--pmc FETCH_SIZE`, then with
     `--pmc WRITE_SIZE` (one counter block per pass);
  2. a plain copy of COPY_MIB MiB (torch `copy_` between two device buffers)
     under the same two counters.
The copy moves a known number of bytes each way, so it calibrates the
counters: factor = bytes copied / (counter KiB * 1024).  Each kernel's traffic
per launch is FETCH * factor_fetch + WRITE * factor_write.

The summary records the SHA-256 of the kernel source it was measured with;
bench.py reports `traffic` only while the source is unchanged.

    python -m paper_2411_02206_amd.traffic --copy MIB

is the copy program of step 2.
"""
import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import shutil
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2411_02206_amd", "csrc", "tmd.hip")
COPY_MIB = 1024


def source_hash():
    with open(SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def copy_program(mib):
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty(n, dtype=torch.uint8, device="cuda")
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x3", flush=True)


def kernel_name(raw):
    """Short kernel name, template arguments kept (k_rans<2, 0>)."""
    name = raw.replace("(anonymous namespace)::", "").split("(")[0].strip()
    return name[5:] if name.startswith("void ") else name


def load_counters(d):
    """{kernel: {counter: mean value per dispatch}}"""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise RuntimeError(f"no counter_collection.csv under {d}")
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                agg[kernel_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in agg.items()}, \
        {k: max(len(v) for v in cs.values()) for k, cs in agg.items()}


def run_pass(rocprof, counter, outdir, prog, timeout):
    if os.path.isdir(outdir):
        shutil.rmtree(outdir)
    cmd = [rocprof, "--pmc", counter, "--output-format", "csv", "-d", outdir, "-o", "run", "--"] + prog
    env = dict(os.environ, TMPDIR="/tmp")
    t = time.perf_counter()
    print("[traffic] " + " ".join(cmd), flush=True)
    r = subprocess.run(cmd, env=env, timeout=timeout, cwd=ROOT, stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, text=True)
    print(f"[traffic] exit {r.returncode} after {time.perf_counter() - t:.1f} s", flush=True)
    if r.returncode != 0:
        sys.stdout.write(r.stdout[-4000:])
        raise RuntimeError(f"rocprofv3 pass {counter} failed with {r.returncode}")
    return load_counters(outdir)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--copy", type=int, default=0, help="run the copy program of MIB MiB and exit")
    ap.add_argument("--workload", default="batched")
    ap.add_argument("--bench-args", default="", help="more bench.py arguments, e.g. '--frames-cache DIR'")
    ap.add_argument("--out", default=None)
    ap.add_argument("--work", default=os.path.join(ROOT, "rocprof_out", "traffic"),
                    help="folder for rocprofv3's raw output")
    ap.add_argument("--rocprof", default="rocprofv3")
    ap.add_argument("--timeout", type=float, default=240.0)
    args = ap.parse_args()
    if args.copy:
        copy_program(args.copy)
        return
    py = sys.executable
    bench = [py, "-u", os.path.join(ROOT, "bench.py"), "--workload", args.workload, "--steps", "3",
             "--warmup", "1", "--no-cpu", "--no-plain", "--gen-workers", "1"] + args.bench_args.split()
    copyp = [py, "-u", "-m", "paper_2411_02206_amd.traffic", "--copy", str(COPY_MIB)]
    res = {}
    for tag, prog in (("bench", bench), ("copy", copyp)):
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            res[(tag, counter)] = run_pass(args.rocprof, counter, os.path.join(args.work, f"{tag}_{counter}"),
                                           prog, args.timeout)
    copy_bytes = float(COPY_MIB << 20)

    def copy_kib(counter):
        vals, _ = res[("copy", counter)]
        # the copy kernel is the dispatch kind with the largest counter value
        return max(cs.get(counter, 0.0) for cs in vals.values())

    f_fetch = copy_bytes / (copy_kib("FETCH_SIZE") * 1024.0)
    f_write = copy_bytes / (copy_kib("WRITE_SIZE") * 1024.0)
    fe, nd = res[("bench", "FETCH_SIZE")]
    wr, _ = res[("bench", "WRITE_SIZE")]
    kernels = {}
    for k in sorted(fe):
        if not k.startswith("k_"):
            continue
        f = fe[k].get("FETCH_SIZE", 0.0)
        w = wr.get(k, {}).get("WRITE_SIZE", 0.0)
        kernels[k] = {"fetch_kib": round(f, 1), "write_kib": round(w, 1), "dispatches": nd[k],
                      "traffic_bytes": round(f * 1024.0 * f_fetch + w * 1024.0 * f_write)}
    ba = args.bench_args.split()
    frames = int(ba[ba.index("--frames") + 1]) if "--frames" in ba else 64
    summary = {"workload": args.workload, "frames": frames, "source_sha256": source_hash(), "copy_mib": COPY_MIB,
               "factor_fetch": round(f_fetch, 4), "factor_write": round(f_write, 4), "kernels": kernels}
    lines = [f"# HBM traffic per launch, workload `{args.workload}`", "",
             "Made by `python -m paper_2411_02206_amd.traffic --workload "
             f"{args.workload} --out <this file>`, which runs:", ""]
    for tag, prog in (("bench", bench), ("copy", copyp)):
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            rel = [os.path.relpath(p, ROOT) if p.startswith(ROOT) else p for p in prog]
            rel[0] = "python3"
            lines.append(f"    rocprofv3 --pmc {counter} --output-format csv -d <dir> -o run -- {' '.join(rel)}")
    lines += ["",
              f"Calibration: a {COPY_MIB} MiB device-to-device copy reads FETCH_SIZE "
              f"{copy_kib('FETCH_SIZE'):.0f} KiB and WRITE_SIZE {copy_kib('WRITE_SIZE'):.0f} KiB per dispatch "
              f"for {COPY_MIB << 10} KiB moved each way: factor_fetch {f_fetch:.4f}, factor_write {f_write:.4f}.",
              "",
              "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | calibrated traffic (MB) |",
              "|---|---|---|---|---|"]
    for k, v in kernels.items():
        lines.append(f"| {k} | {v['dispatches']} | {v['fetch_kib']:.1f} | {v['write_kib']:.1f} | "
                     f"{v['traffic_bytes'] / 1e6:.1f} |")
    lines += ["", "traffic-json: " + json.dumps(summary), ""]
    text = "\n".join(lines)
    print(text, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)


def load_summary(workload, profiles_dir=None):
    """Traffic summary for `workload` if it was measured with the current
    kernel source, else None."""
    d = profiles_dir or os.path.join(ROOT, "profiles")
    fn = os.path.join(d, f"traffic_{workload}.md")
    if not os.path.exists(fn):
        return None
    with open(fn) as f:
        for line in f:
            if line.startswith("traffic-json: "):
                s = json.loads(line[len("traffic-json: "):])
                if s.get("source_sha256") == source_hash() and s.get("workload") == workload:
                    return s
    return None


if __name__ == "__main__":
    main()

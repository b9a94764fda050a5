"""Benchmark: decoded TPC clusters/s on one MI355X, bit-exact.

Default workload: one full synthetic Pb-Pb-like time frame (100 collisions x
2000 tracks, about 1.5e7 attached + 1.0e7 unattached clusters), decoded by the
plain single-frame launch sequence with inputs resident in HBM.  A step is one
complete tmd_decode (all kernels: track offsets, bin counts, offsets, ranks,
attached decode, unattached decode, status).

Prints one JSON line.  `roofline` reports the dominant kernel's algorithmic
HBM bytes per launch (attached kernel: 10 B in + 10 B out per attached
cluster, 15 B per track header; unattached kernel: 10 B in + 10 B out per
cluster) over its average duration from HIP events recorded on the decode
stream during the timed steps.  `cpu_baseline` is the plain C oracle on one
host core over a bounded sample of the same frame.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HDR_BYTES = 15          # ncls, sec0, row0 (1 B each), pad0 (2), time0 (4), qpt, snp, tgl (2 each)
CLUSTER_IN_BYTES = 10   # attached: row/sector step (1+1), residuals (2+2), charges (2+2)
UNATT_IN_BYTES = 10     # time diff (4), pad diff (2), charges (2+2)
CLUSTER_OUT_BYTES = 10  # time (4), pad (2), charges (2+2)
BIN_BYTES = 4 + 4 + 4   # un_count in, row_offset and row_nattached out

WORKLOADS = {
    "frame": "one Pb-Pb-like time frame: 100 collisions x 2000 tracks, 36 sectors, 152 rows, "
             "track lengths U{5..152}, 10% sector crossers, 40% unattached; plain single launch",
    "stress": "high-occupancy stress frame: 500 collisions x 2000 tracks, 15% low-pT loopers, "
              "rows skewed exp(-row/40); plain single launch",
    "tiny": "tiny plain decode: 1 sector, 1000 tracks of 20..152 clusters, 20000 unattached",
}


def algorithmic_bytes(nT, nA, nU):
    att = nA * (CLUSTER_IN_BYTES + CLUSTER_OUT_BYTES) + nT * HDR_BYTES
    una = nU * (UNATT_IN_BYTES + CLUSTER_OUT_BYTES)
    return att, una, att + una + 5472 * BIN_BYTES


def cpu_baseline(frame, bz, budget_s, n_clusters):
    import oracle
    t0 = time.perf_counter()
    reps = 0
    res = None
    while True:
        res = oracle.decode(frame, bz=bz)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": n_clusters * reps / dt, "unit": "clusters/s", "cores": 1, "kind": "oracle",
            "sample": f"the same frame decoded {reps}x by the single-threaded C oracle "
                      f"({n_clusters} clusters each, {dt:.1f} s)"}, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="frame", choices=sorted(WORKLOADS))
    ap.add_argument("--bz", type=float, default=0.5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and check")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build decodes on one GPU only; --gpus {args.gpus} is not supported "
              "(frames are independent: several GPUs would each decode their own frames)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2411_02206_amd as tmd
    import synth

    spec = synth.spec_for(args.workload)
    t = time.perf_counter()
    frame = synth.make_frame(spec)
    gen_s = time.perf_counter() - t
    nT, nA, nU = tmd.frame_shape(frame)
    n_clusters = nA + nU
    print(f"[bench] {args.workload}: {nT} tracks, {nA} attached, {nU} unattached "
          f"(generated in {gen_s:.1f} s)", file=sys.stderr, flush=True)

    dev = tmd.to_device(frame)
    plan = tmd.Plan([(nT, nA, nU)], bz=args.bz)
    out = tmd.alloc_out((nT, nA, nU))
    ws = plan.alloc_workspace()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.decode([dev], [out], ws, stream)
    torch.cuda.synchronize()
    status = plan.status(0)

    plan.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.decode([dev], [out], ws, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages, calls = plan.stage_times()
    plan.set_profiling(False)
    ms_per_step = 1e3 * elapsed / args.steps
    value = n_clusters * args.steps / elapsed
    print(f"[bench] {ms_per_step:.3f} ms/step, {value:.3e} clusters/s", file=sys.stderr, flush=True)

    # per-frame latency: each decode bracketed by its own events
    lat = []
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.decode([dev], [out], ws, stream)
        e1.record(stream)
        lat.append((e0, e1))
    torch.cuda.synchronize()
    lat_ms = np.array([a.elapsed_time(b) for a, b in lat])

    att_b, una_b, all_b = algorithmic_bytes(nT, nA, nU)
    avg = {k: v / max(calls, 1) for k, v in stages.items()}
    dominant = max(avg, key=avg.get)
    dom_bytes = {"attached": att_b, "unattached": una_b}.get(dominant)
    roof = None
    if dom_bytes is not None and avg[dominant] > 0:
        ach = dom_bytes / (avg[dominant] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": f"k_{dominant}", "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": None, "bytes_per_launch": dom_bytes, "avg_ms": round(avg[dominant], 4)}
    step_gbs = all_b / (ms_per_step * 1e-3) / 1e9

    cpu = None
    bitexact = None
    if not args.no_cpu:
        cpu, (exp, est) = cpu_baseline(frame, args.bz, args.cpu_seconds, n_clusters)
        got = tmd.to_numpy(out)
        bitexact = bool(all(np.array_equal(exp[k], got[k]) for k in exp) and est == status)

    line = {
        "metric": "decoded TPC clusters/s on 1 MI355X (bit-exact) + p50/p99 time-frame latency",
        "value": value, "unit": "clusters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "n_tracks": nT,
                   "n_attached": nA, "n_unattached": nU, "bz_tesla": args.bz},
        "roofline": roof,
        "cpu_baseline": cpu,
        "bitexact_vs_oracle": bitexact,
        "status_flags": status,
        "step_algorithmic_GBs": round(step_gbs, 1),
        "step_hbm_frac": round(step_gbs / HBM_PEAK_GBS, 4),
        "stage_avg_ms": {k: round(v, 4) for k, v in avg.items()},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4)},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

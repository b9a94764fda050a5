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
    "batched": "64 time frames of log-uniform 10..200 collisions x 2000 tracks decoded by one plan "
               "(one HIP-graph launch), compared with 64 plain per-frame decodes",
    "served": "Poisson arrivals of frames from the batched mix at 25/50/75/100% of the batched peak; "
              "continuous batching under a 200 GB HBM budget; p50/p99 latency",
    "pipeline": "the frame workload held in page-locked host memory, decoded through the native pipeline "
                "(one upload stream, a decode stream per slot, one download stream, ordered by events), "
                "3 slots against 1 (no overlap); rate includes the PCIe transfers",
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
    ap.add_argument("--frames", type=int, default=64, help="frames of the batched/served workloads")
    ap.add_argument("--seconds-per-load", type=float, default=2.0, help="served: arrival window per load")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="forked processes generating the synthetic frames (1 under a profiler that "
                         "initialises the GPU before the program starts)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: libtmd decodes on one GPU; --gpus {args.gpus} is not supported "
              "(frames are independent: several GPUs would each decode their own frames)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2411_02206_amd as tmd
    import synth

    if args.workload in ("batched", "served"):
        return run_batched(args)
    if args.workload == "pipeline":
        return run_pipeline(args)

    spec = synth.spec_for(args.workload)
    t = time.perf_counter()
    frame = synth.make_frame(spec, workers=args.gen_workers)  # forked workers, before any GPU use
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

    # per-stage breakdown (events around every stage), then the timed steps
    # with events around the dominant kernel only
    plan.set_profiling(True)
    for _ in range(args.steps):
        plan.decode([dev], [out], ws, stream)
    torch.cuda.synchronize()
    stages, calls = plan.stage_times()
    avg = {k: v / max(calls, 1) for k, v in stages.items()}
    dominant = max(avg, key=avg.get)
    plan.set_profiling(stages=[dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.decode([dev], [out], ws, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dom_stages, dom_calls = plan.stage_times()
    dom_ms = dom_stages[dominant] / max(dom_calls, 1)
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
    # algorithmic bytes per launch of each kernel (what its step of the method
    # must move): attached decode 10 B in + 10 B out per attached cluster and
    # 15 B per header; unattached 10 + 10 B per cluster; count and rank read
    # the 2 B of row/sector steps per attached cluster (the rank kernel also
    # the 8 B of residuals and charges it packs for the decode)
    kernel_bytes = {"attached": att_b, "unattached": una_b, "count": 2 * nA + nT,
                    "rank": 10 * nA + nT}
    dom_bytes = kernel_bytes.get(dominant)
    roof = None
    if dom_bytes is not None and dom_ms > 0:
        ach = dom_bytes / (dom_ms * 1e-3) / 1e9
        # measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
        # copy-calibrated), only if taken with the current kernel source
        from paper_2411_02206_amd import traffic as _traffic
        summ = _traffic.load_summary(args.workload)
        kt = summ["kernels"].get(f"k_{dominant}") if summ else None
        roof = {"bound": "hbm", "kernel": f"k_{dominant}", "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": kt["traffic_bytes"] if kt else None, "bytes_per_launch": dom_bytes,
                "avg_ms": round(dom_ms, 4)}
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


def run_pipeline(args):
    """Host-resident frames: the same page-locked frame decoded `steps` times
    through tmd_pipe_run, with 3 slots and with 1; each slot writes its own
    page-locked output buffers."""
    import numpy as np
    import torch

    import paper_2411_02206_amd as tmd
    import synth

    frame = synth.make_frame(synth.spec_for("frame"), workers=args.gen_workers)
    shape = tmd.frame_shape(frame)
    nT, nA, nU = shape
    n_clusters = nA + nU
    host = tmd.to_host(frame, pin=True)
    in_bytes = sum(v.numel() * v.element_size() for v in host.values())
    out_bytes = 10 * n_clusters + 4 * (2 * 5472 + 1)
    # reference: the same frame decoded from device memory by a plain plan
    ref, ref_flags = tmd.decode(tmd.to_device(frame), bz=args.bz)
    ref = tmd.to_numpy(ref)
    torch.cuda.empty_cache()
    res = {}
    bitexact = True
    for depth in (3, 1):
        pipe = tmd.Pipeline(shape, depth=depth, bz=args.bz)
        outs = [tmd.alloc_host_out(shape, pin=True) for _ in range(depth)]
        k = max(args.steps, depth)
        fl = pipe.run([host] * depth, outs)  # warmup: every slot once
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fl = pipe.run([host] * k, [outs[i % depth] for i in range(k)])
        dt = time.perf_counter() - t0
        res[depth] = {"ms_per_frame": 1e3 * dt / k, "clusters_per_s": n_clusters * k / dt, "frames": k,
                      "flags": fl[-1]}
        got = tmd.to_numpy(outs[(k - 1) % depth])
        bitexact = bitexact and all(np.array_equal(ref[q], got[q]) for q in ref) and fl[-1] == ref_flags
        print(f"[bench] pipeline depth {depth}: {1e3 * dt / k:.3f} ms/frame, {n_clusters * k / dt:.3e} clusters/s",
              file=sys.stderr, flush=True)
        pipe.free()
    best = res[3]
    line = {
        "metric": "host-resident TPC clusters/s on 1 MI355X including PCIe transfers (bit-exact)",
        "value": best["clusters_per_s"], "unit": "clusters/s", "n_gpus": 1, "steps": best["frames"],
        "warmup": 3, "ms_per_step": best["ms_per_frame"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"pipeline: {WORKLOADS['pipeline']}", "n_tracks": nT, "n_attached": nA,
                   "n_unattached": nU, "bz_tesla": args.bz, "h2d_bytes_per_frame": in_bytes,
                   "d2h_bytes_per_frame": out_bytes},
        "depth1": res[1],
        "overlap_speedup": res[1]["ms_per_frame"] / best["ms_per_frame"],
        "pcie_GBs_each_way": round(in_bytes / (best["ms_per_frame"] * 1e-3) / 1e9, 1),
        "bitexact_vs_device_decode": bool(bitexact),
    }
    print(json.dumps(line), flush=True)


def _gen(spec):
    import synth
    return synth.make_frame(spec)


def make_frames(specs, workers=16):
    """Generate frames in parallel worker processes (forked before any GPU use)."""
    import multiprocessing as mp
    n = max(1, min(workers, len(specs), os.cpu_count() or 1))
    if n == 1:
        return [_gen(s) for s in specs]
    with mp.get_context("fork").Pool(n) as pool:
        return pool.map(_gen, specs, chunksize=1)


def run_batched(args):
    """Batched workload (one plan over all frames, HIP graph) against plain
    per-frame decodes of the same frames; with --workload served, also the
    serving loop at several offered loads."""
    import synth
    specs = synth.batch_specs(args.workload, n_frames=args.frames)
    t = time.perf_counter()
    frames = make_frames(specs, workers=args.gen_workers)
    gen_s = time.perf_counter() - t

    import numpy as np
    import torch

    import paper_2411_02206_amd as tmd
    from paper_2411_02206_amd import serve

    shapes = [tmd.frame_shape(f) for f in frames]
    n_clusters = sum(a + u for _, a, u in shapes)
    print(f"[bench] {args.workload}: {len(frames)} frames, {sum(s[0] for s in shapes)} tracks, {n_clusters} "
          f"clusters (generated in {gen_s:.1f} s)", file=sys.stderr, flush=True)
    ins = [tmd.to_device(f) for f in frames]
    stream = torch.cuda.current_stream()

    # plain: one plan and one launch sequence per frame
    plans = [tmd.Plan([s], bz=args.bz) for s in shapes]
    ws_bytes = max(p.workspace_bytes for p in plans)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    outs_plain = [tmd.alloc_out(s) for s in shapes]

    def plain_step():
        for p, i, o in zip(plans, ins, outs_plain):
            p.decode([i], [o], ws, stream)

    # batched: one plan over all frames, captured once as a HIP graph
    bplan = tmd.Plan(shapes, bz=args.bz, flags=tmd.PLAN_GRAPH)
    bws = bplan.alloc_workspace()
    outs_b = [tmd.alloc_out(s) for s in shapes]

    def batched_step():
        bplan.decode(ins, outs_b, bws, stream)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    steps = max(1, args.steps // 10)
    t_plain = timed(plain_step, steps, 1)
    t_batch = timed(batched_step, steps, 1)
    print(f"[bench] plain {1e3 * t_plain:.3f} ms, batched {1e3 * t_batch:.3f} ms per pass over "
          f"{len(frames)} frames", file=sys.stderr, flush=True)
    # every frame bit-identical between the two forms
    def dev_equal(a, b):
        n = int(a["row_offset"][-1].item())
        if n != int(b["row_offset"][-1].item()):
            return False
        if not (torch.equal(a["row_offset"], b["row_offset"]) and
                torch.equal(a["row_nattached"], b["row_nattached"])):
            return False
        return all(torch.equal(a[k][:n], b[k][:n]) for k in ("time", "pad", "qtot", "qmax"))

    same = all(dev_equal(a, b) for a, b in zip(outs_plain, outs_b))
    flags_same = all(p.status(0) == bplan.status(i) for i, p in enumerate(plans))
    oracle_ok = None
    if not args.no_cpu:
        import oracle
        oracle_ok = True
        for i in (0, len(frames) // 2):
            exp, est = oracle.decode(frames[i], bz=args.bz)
            got = tmd.to_numpy(outs_b[i])
            oracle_ok &= bool(all(np.array_equal(exp[k], got[k]) for k in exp) and est == bplan.status(i))

    line = {
        "metric": "decoded TPC clusters/s on 1 MI355X (bit-exact) + p50/p99 time-frame latency",
        "value": n_clusters / t_batch, "unit": "clusters/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": 1e3 * t_batch, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "frames": len(frames),
                   "n_clusters": n_clusters, "bz_tesla": args.bz},
        "plain_per_frame": {"ms_per_pass": 1e3 * t_plain, "clusters_per_s": n_clusters / t_plain},
        "batched_vs_plain_speedup": t_plain / t_batch,
        "bitexact_batched_vs_plain": bool(same and flags_same),
        "bitexact_vs_oracle_sampled_frames": oracle_ok,
    }
    del outs_plain, plans, ws

    if args.workload == "served":
        peak_fps = len(frames) / t_batch
        loads = {}
        srv = serve.Server(bz=args.bz, hbm_budget=200e9, slots=4, max_batch=8, graph=True)
        rng = np.random.default_rng(3)
        for frac in (0.25, 0.5, 0.75, 1.0):
            rate = frac * peak_fps
            n_req = max(50, int(rate * args.seconds_per_load))
            gaps = rng.exponential(1.0 / rate, n_req)
            picks = rng.integers(0, len(frames), n_req)
            srv.done = []
            t0 = time.perf_counter()
            arrivals = t0 + np.cumsum(gaps)
            k = 0
            nd = 0
            while len(srv.done) < n_req:
                now = time.perf_counter()
                while k < n_req and arrivals[k] <= now:
                    srv.submit(ins[picks[k]], arrival=float(arrivals[k]))
                    k += 1
                srv.step()
                # the client takes each result as it completes: its buffers go
                for r in srv.done[nd:]:
                    r.out = None
                nd = len(srv.done)
            t1 = time.perf_counter()
            lat = [1e3 * r.latency for r in srv.done]
            served_clusters = sum(shapes[p][1] + shapes[p][2] for p in picks)
            loads[f"{int(frac * 100)}%"] = {
                "offered_frames_per_s": rate, "requests": n_req,
                "p50_ms": serve.percentile(lat, 50), "p99_ms": serve.percentile(lat, 99),
                "clusters_per_s": served_clusters / (t1 - t0)}
            print(f"[bench] load {frac:.2f}: p50 {loads[f'{int(frac * 100)}%']['p50_ms']:.3f} ms, "
                  f"p99 {loads[f'{int(frac * 100)}%']['p99_ms']:.3f} ms", file=sys.stderr, flush=True)
        srv.close()
        line["served"] = loads
        line["latency_ms"] = {"p50": loads["100%"]["p50_ms"], "p99": loads["100%"]["p99_ms"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

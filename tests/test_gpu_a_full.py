"""Full-size workloads against the oracle, every cluster of every frame:
  - the batched workload: 64 frames of log-uniform 10..200 collisions (about
    1.1e9 clusters) through one graph plan, as bench.py times it, plain and
    entropy-coded;
  - the stress workload (about 1e6 tracks and 1.25e8 clusters: loopers,
    sector crossings, rows skewed exponentially) through a plain plan, a
    graph plan and the serving loop (mixed with batched frames).
This module sorts first among the GPU tests, so that the frames can be drawn
by forked worker processes before this process uses the GPU.  The oracle runs
on host threads, one frame per thread."""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def big():
    import torch
    # forked generator workers only while this process has not touched the GPU
    workers = 1 if torch.cuda.is_initialized() else 16
    specs = synth.batch_specs("batched", n_frames=64) + [synth.spec_for("stress")]
    print(f"\nfull-size frames: generating {len(specs)} with {workers} worker(s)", flush=True)
    frames = synth.make_frames(specs, workers=workers)
    return {"batched": frames[:64], "stress": frames[64]}


def oracle_many(frames):
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda f: oracle.decode(f), frames))


def check(tmd, exp, est, out, flags, label):
    got = tmd.to_numpy(out)
    for k in exp:
        assert np.array_equal(exp[k], got[k]), (label, k)
    assert flags == est, (label, flags, est)


def test_batched_workload_full_size_graph(big):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_02206_amd as tmd
    frames = big["batched"]
    shapes = [tmd.frame_shape(f) for f in frames]
    n = sum(a + u for _, a, u in shapes)
    print(f"batched: {len(frames)} frames, {n} clusters", flush=True)
    assert n > 9e8
    ins = [tmd.to_device(f) for f in frames]
    outs = [tmd.alloc_out(s) for s in shapes]
    plan = tmd.Plan(shapes, flags=tmd.PLAN_GRAPH)
    ws = plan.alloc_workspace()
    for rep in range(2):   # the second call replays the captured graph
        for o in outs:
            o["time"].fill_(-1)
        plan.decode(ins, outs, ws)
        torch.cuda.synchronize()
    flags = [plan.status(i) for i in range(len(frames))]
    del ins, ws
    exp = oracle_many(frames)
    for i, (e, est) in enumerate(exp):
        check(tmd, e, est, outs[i], flags[i], f"frame {i}")
        outs[i] = None
        exp[i] = None
    assert not any(flags), "the batched workload's streams are valid: no flag may be set"
    plan.free()


def test_coded_batched_workload_full_size(big):
    """The batched frames entropy-coded on the GPU (tmd_encode_rans), as
    bench.py's coded workload: the coder writes the oracle coder's bytes
    (checked on the smallest and the largest frame), and one tmd_decode_rans
    call on the graph plan decodes every frame as the oracle does."""
    import torch
    import paper_2411_02206_amd as tmd
    frames = big["batched"]
    shapes = [tmd.frame_shape(f) for f in frames]
    ws_bytes = max(tmd.rans_encode_sizes(s)[0] for s in shapes)
    enc_ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    coded = []
    for f in frames:
        dev = tmd.to_device(f)
        coded.append(tmd.encode_rans(dev, workspace=enc_ws).clone())
        del dev
    del enc_ws
    sizes = [s[1] + s[2] for s in shapes]
    for i in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        assert np.array_equal(coded[i].cpu().numpy(), oracle.rans_encode(frames[i])), f"coded bytes of frame {i}"
    outs = [tmd.alloc_out(s) for s in shapes]
    plan = tmd.Plan(shapes, flags=tmd.PLAN_GRAPH)
    ws = plan.alloc_workspace()
    rws = torch.empty(plan.rans_workspace_bytes(), dtype=torch.uint8, device="cuda")
    for rep in range(2):
        for o in outs:
            o["time"].fill_(-1)
        plan.decode_rans(coded, outs, ws, rws)
        torch.cuda.synchronize()
    flags = [plan.status(i) for i in range(len(frames))]
    del coded, ws, rws
    exp = oracle_many(frames)
    for i, (e, est) in enumerate(exp):
        check(tmd, e, est, outs[i], flags[i], f"coded frame {i}")
        outs[i] = None
        exp[i] = None
    plan.free()


@pytest.fixture(scope="module")
def stress_expected(big):
    return oracle.decode(big["stress"])


def test_stress_workload_full_size(big, stress_expected):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_02206_amd as tmd
    fr = big["stress"]
    shape = tmd.frame_shape(fr)
    print(f"stress frame: {shape[0]} tracks, {shape[1]} attached, {shape[2]} unattached", flush=True)
    out, flags = tmd.decode(tmd.to_device(fr))
    exp, est = stress_expected
    check(tmd, exp, est, out, flags, "plain")
    assert exp["row_offset"][-1] > 1.2e8
    assert est == 0


def test_stress_workload_graph_plan(big, stress_expected):
    import torch
    import paper_2411_02206_amd as tmd
    fr = big["stress"]
    shape = tmd.frame_shape(fr)
    plan = tmd.Plan([shape], flags=tmd.PLAN_GRAPH)
    ws = plan.alloc_workspace()
    dev = tmd.to_device(fr)
    out = tmd.alloc_out(shape)
    exp, est = stress_expected
    for rep in range(2):
        out["time"].fill_(-1)
        plan.decode([dev], [out], ws)
        torch.cuda.synchronize()
        check(tmd, exp, est, out, plan.status(0), f"graph replay {rep}")
    plan.free()


def test_stress_workload_served_in_a_mix(big, stress_expected):
    """The stress frame submitted to the serving loop among batched frames:
    admitted and decoded with them, the same result as alone."""
    import paper_2411_02206_amd as tmd
    from paper_2411_02206_amd import serve
    fr = big["stress"]
    small = big["batched"][:3]
    srv = serve.Server(slots=2, max_batch=2, graph=True)
    reqs = [srv.submit(tmd.to_device(small[0])), srv.submit(tmd.to_device(fr)),
            srv.submit(tmd.to_device(small[1])), srv.submit(tmd.to_device(small[2]))]
    srv.run_until(len(reqs), timeout=300)
    exp, est = stress_expected
    check(tmd, exp, est, reqs[1].out, reqs[1].flags, "served stress")
    for r, f in zip((reqs[0], reqs[2], reqs[3]), small):
        e, es = oracle.decode(f)
        check(tmd, e, es, r.out, r.flags, "served batched frame")
    srv.close()

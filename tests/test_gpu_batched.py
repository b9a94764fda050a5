"""Batched (one launch sequence over many frames, optionally replayed as a HIP
graph) and served (continuous batching) forms give bit-identical results to
the plain single-frame decode."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tmd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_02206_amd as m
    return m


@pytest.fixture(scope="module")
def frames():
    specs = synth.batch_specs("batched", n_frames=6, coll_range=(1, 5))
    return [synth.make_frame(s) for s in specs]


def plain(tmd, frame):
    out, flags = tmd.decode(tmd.to_device(frame))
    return tmd.to_numpy(out), flags


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in a)


def test_graph_replays_match_eager(tmd, frames):
    import torch
    ref = [plain(tmd, f) for f in frames]
    shapes = [tmd.frame_shape(f) for f in frames]
    plan = tmd.Plan(shapes, flags=tmd.PLAN_GRAPH)
    ins = [tmd.to_device(f) for f in frames]
    outs = [tmd.alloc_out(s) for s in shapes]
    ws = plan.alloc_workspace()
    for rep in range(4):
        for o in outs:
            for k in tmd.OUT_FIELDS:
                o[k].fill_(-1)
        plan.decode(ins, outs, ws)
        torch.cuda.synchronize()
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        for i in range(len(frames)):
            got = tmd.to_numpy(outs[i])
            assert same(ref[i][0], got), (rep, i)
            assert plan.status(i) == ref[i][1]


def test_served_mix_equals_alone(tmd, frames):
    from paper_2411_02206_amd import serve
    ref = [plain(tmd, f) for f in frames]
    dev = [tmd.to_device(f) for f in frames]
    srv = serve.Server(slots=3, max_batch=3)
    reqs = [srv.submit(d) for d in dev + dev]  # each frame twice, in different mixes
    srv.run_until(len(reqs), timeout=120)
    for i, r in enumerate(reqs):
        got = tmd.to_numpy(r.out)
        assert same(ref[i % len(frames)][0], got), i
        assert r.flags == ref[i % len(frames)][1]
    srv.close()


def test_served_host_frames(tmd, frames):
    """Host-resident requests: copied in by the server, same results."""
    from paper_2411_02206_amd import serve
    ref = [plain(tmd, f) for f in frames[:3]]
    srv = serve.Server(slots=2, max_batch=2, graph=True)
    reqs = [srv.submit(f) for f in frames[:3]]
    srv.run_until(3, timeout=120)
    for i, r in enumerate(reqs):
        assert same(ref[i][0], tmd.to_numpy(r.out)), i
    srv.close()

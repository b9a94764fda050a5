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


def test_capacity_plan_changing_shapes(tmd, frames):
    """One plan with capacity shapes (tmd_decode_shapes) decodes batches of
    different, smaller frames and idle entries, eagerly and replayed as a
    graph, bit-identically to plain single-frame decodes."""
    import torch
    ref = [plain(tmd, f) for f in frames]
    shapes = [tmd.frame_shape(f) for f in frames]
    cap = tuple(max(s[i] for s in shapes) + 7 for i in range(3))
    nent = 3
    for flags in (0, tmd.PLAN_GRAPH):
        plan = tmd.Plan([cap] * nent, flags=flags)
        ws = plan.alloc_workspace()
        idle_in = {k: None for k in tmd.IN_FIELDS}
        idle_in["un_count"] = torch.zeros(tmd.NBIN, dtype=torch.int32, device="cuda")
        idle_out = tmd.alloc_out((0, 0, 0))
        for k in ("time", "pad", "qtot", "qmax"):
            idle_out[k] = None
        idle_out["capacity"] = 0
        groups = [[0, 1, 2], [3], [4, 5], [5, 0]]
        for rep in range(2):
            for g in groups:
                ins = [tmd.to_device(frames[i]) for i in g] + [idle_in] * (nent - len(g))
                outs = [tmd.alloc_out(shapes[i]) for i in g] + [idle_out] * (nent - len(g))
                plan.decode(ins, outs, ws, shapes=[shapes[i] for i in g] + [(0, 0, 0)] * (nent - len(g)))
                torch.cuda.synchronize()
                for e, i in enumerate(g):
                    assert same(ref[i][0], tmd.to_numpy(outs[e])), (flags, rep, g, i)
                    assert plan.status(e) == ref[i][1]
                for e in range(len(g), nent):
                    assert plan.status(e) == 0
                    assert int(idle_out["row_offset"][-1].item()) == 0
        plan.free()


def test_single_frame_capacity_plan_with_chained_tracks(tmd, frames, monkeypatch):
    """A single-frame capacity plan whose calls change the decode's wave count
    and whether tracks are chained (two per lane in a few lanes; forced by a
    SIMD count of 2): eager and graph replays against the oracle."""
    import torch
    import oracle
    monkeypatch.setenv("TMD_ATTACHED_SIMDS", "2")
    big = max(frames, key=lambda f: f["trk_ncls"].shape[0])

    def cut(fr, nt):
        na = int(fr["trk_ncls"][:nt].astype(np.int64).sum())
        return {k: (v[:nt] if k.startswith("trk_") else v[:na] if k.startswith("cls_") else v)
                for k, v in fr.items()}

    # 2100, 4000, 3000 tracks: 33, 63, 47 waves -> 32, 62, 46 with chained
    # tracks; 2048: 32 waves, none chained
    cuts = [cut(big, nt) for nt in (2100, 2048, 4000, 3000) if nt <= big["trk_ncls"].shape[0]]
    assert len(cuts) == 4
    exp = [oracle.decode(f) for f in cuts]
    shapes = [tmd.frame_shape(f) for f in cuts]
    cap = tuple(max(s[i] for s in shapes) + 5 for i in range(3))
    for flags in (0, tmd.PLAN_GRAPH):
        plan = tmd.Plan([cap], flags=flags)
        ws = plan.alloc_workspace()
        for rep in range(2):
            for i, f in enumerate(cuts):
                out = tmd.alloc_out(shapes[i])
                plan.decode([tmd.to_device(f)], [out], ws, shapes=[shapes[i]])
                torch.cuda.synchronize()
                got = tmd.to_numpy(out)
                assert all(np.array_equal(exp[i][0][k], got[k]) for k in exp[i][0]), (flags, rep, i)
                assert plan.status(0) == exp[i][1], (flags, rep, i)
        plan.free()


def test_capacity_plan_rejects_larger_shape(tmd, frames):
    shapes = [tmd.frame_shape(f) for f in frames]
    plan = tmd.Plan([shapes[0]])
    ws = plan.alloc_workspace()
    big = tuple(v + 1 for v in shapes[0])
    with pytest.raises(tmd.TmdError):
        plan.decode([tmd.to_device(frames[0])], [tmd.alloc_out(big)], ws, shapes=[big])
    plan.free()

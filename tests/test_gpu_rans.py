"""Entropy-coded frames on the GPU (tmd_decode_rans): frames coded by the
oracle's rANS coder are decoded by the library's rANS kernel into its
workspace and then by the track-model decode in the same call; the result
must equal the oracle's decode of the uncoded frame, bit for bit.  Also: a
batched graph plan over several coded frames, and malformed coded data
(wrong magic, wrong shape, truncated, corrupted streams), which must be
flagged or at least decoded safely."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import _garbage

pytestmark = pytest.mark.gpu

NBIN = 36 * 152  # (sector, row) bins


@pytest.fixture(scope="module")
def tmd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_02206_amd as m
    return m


def check(tmd, exp, est, out, flags, label):
    got = tmd.to_numpy(out)
    for k in exp:
        assert np.array_equal(exp[k], got[k]), (label, k)
    assert flags == est, (label, flags, est)


@pytest.mark.parametrize("case", ["tiny", "frame", "stress", "garbage", "empty"])
def test_coded_frame_decodes_like_the_plain_one(tmd, case):
    if case == "tiny":
        fr = synth.make_frame(synth.spec_for("tiny"))
    elif case == "frame":
        fr = synth.make_frame(synth.spec_for("frame", collisions=3))
    elif case == "stress":
        fr = synth.make_frame(synth.spec_for("stress", collisions=1))
    elif case == "garbage":
        fr = _garbage(21)
    else:
        fr = {k: np.zeros(0 if k != "un_count" else tmd.NBIN, dt) for k, dt in oracle.RANS_ARRAYS}
    bz = 5.0 if case == "garbage" else 0.5
    blob = oracle.rans_encode(fr)
    exp, est = oracle.decode(fr, bz=bz)
    out, flags = tmd.decode_rans(blob, oracle.frame_sizes(fr), bz=bz)
    check(tmd, exp, est, out, flags, case)


def test_coded_frames_batched_graph(tmd):
    import torch
    frames = synth.make_frames(synth.batch_specs("batched", n_frames=4, coll_range=(1, 4)))
    shapes = [tmd.frame_shape(f) for f in frames]
    coded = [torch.from_numpy(oracle.rans_encode(f)).cuda() for f in frames]
    plan = tmd.Plan(shapes, flags=tmd.PLAN_GRAPH)
    ws = plan.alloc_workspace()
    rws = torch.empty(plan.rans_workspace_bytes(), dtype=torch.uint8, device="cuda")
    outs = [tmd.alloc_out(s) for s in shapes]
    for rep in range(2):
        plan.decode_rans(coded, outs, ws, rws)
        torch.cuda.synchronize()
        for i, f in enumerate(frames):
            check(tmd, *oracle.decode(f), outs[i], plan.status(i), (rep, i))
    plan.free()


def test_malformed_coded_data_is_flagged(tmd):
    fr = synth.make_frame(synth.spec_for("tiny"))
    shape = oracle.frame_sizes(fr)
    blob = oracle.rans_encode(fr)
    bad_magic = blob.copy()
    bad_magic[1] = ord("X")
    for label, b, sh in (("magic", bad_magic, shape), ("truncated", blob[:blob.size // 2], shape),
                         ("header only", blob[:200], shape), ("shape", blob, (shape[0], shape[1] - 1, shape[2]))):
        out, flags = tmd.decode_rans(b, sh)
        assert flags & tmd.F_CODED, label
    # corrupted stream bytes: decoded safely (whatever the values), flagged or not
    rng = np.random.default_rng(0)
    noisy = blob.copy()
    idx = rng.integers(400, noisy.size, 2000)
    noisy[idx] ^= 0x5A
    out, flags = tmd.decode_rans(noisy, shape)
    got = tmd.to_numpy(out)
    assert got["row_offset"].size == tmd.NBIN + 1


@pytest.mark.parametrize("case", ["tiny", "frame", "stress", "garbage", "empty", "no tracks"])
def test_gpu_encoder_matches_oracle(tmd, case):
    """tmd_encode_rans writes the oracle coder's bytes, and they decode back."""
    if case == "tiny":
        fr = synth.make_frame(synth.spec_for("tiny"))
    elif case == "frame":
        fr = synth.make_frame(synth.spec_for("frame", collisions=3))
    elif case == "stress":
        fr = synth.make_frame(synth.spec_for("stress", collisions=1))
    elif case == "garbage":
        fr = _garbage(22)
    else:
        fr = {k: np.zeros(0 if k != "un_count" else tmd.NBIN, dt) for k, dt in oracle.RANS_ARRAYS}
        if case == "no tracks":
            rng = np.random.default_rng(5)
            cnt = rng.integers(0, 4, tmd.NBIN).astype(np.uint32)
            nu = int(cnt.sum())
            fr["un_count"] = cnt
            for k, dt in oracle.RANS_ARRAYS:
                if k.startswith("un_") and k != "un_count":
                    fr[k] = rng.integers(0, np.iinfo(dt).max, nu, dtype=np.int64).astype(dt)
    want = oracle.rans_encode(fr)
    got = tmd.encode_rans(tmd.to_device(fr)).cpu().numpy()
    assert got.size == want.size, (case, got.size, want.size)
    assert np.array_equal(got, want), (case, int(np.flatnonzero(got != want)[0]))


def _long_bins(seed, mode):
    """A frame whose unattached clusters sit in a few long bins (each over
    several 32768-element chunks), many empty bins and short ones, with
    differences that wrap; mode "exact": the counts add up to n_unattached,
    "over": they exceed it (the cut falls inside a long bin), "under": they
    fall short (the last elements belong to no bin)."""
    rng = np.random.default_rng(seed)
    cnt = np.where(rng.random(NBIN) < 0.3, rng.integers(0, 40, NBIN), 0).astype(np.int64)
    cnt[:5] = 0
    cnt[7] = 100_000
    cnt[3000] = 70_001
    cnt[-3:] = [33_000, 0, 65_536]
    total = int(cnt.sum())
    nu = {"exact": total, "over": total - 50_000, "under": total + 40_000}[mode]
    fr = _garbage(seed, nt=300, na=20000, nu=nu)
    fr["un_count"] = cnt.astype(np.uint32)
    fr["un_time_diff"] = rng.integers(0, 2**32, nu, dtype=np.uint64).astype(np.uint32)
    fr["un_pad_diff"] = rng.integers(0, 65536, nu).astype(np.uint16)
    return fr


@pytest.mark.parametrize("mode", ["exact", "over", "under"])
def test_coded_unattached_long_bins(tmd, mode):
    """The unattached arrays are decoded straight into the output: running
    sums whose bins span several chunks (the leading sums of a chunk come
    from the chunks before), counts that overrun or fall short of
    n_unattached, and a batched graph plan with a frame of short bins."""
    import torch
    frames = [_long_bins(31, mode), _garbage(32), _long_bins(33, "exact")]
    shapes = [tmd.frame_shape(f) for f in frames]
    coded = [torch.from_numpy(oracle.rans_encode(f)).cuda() for f in frames]
    print(f"long bins {mode}: shapes {shapes}", flush=True)
    for flags in (0, tmd.PLAN_GRAPH):
        plan = tmd.Plan(shapes, flags=flags)
        ws = plan.alloc_workspace()
        rws = torch.empty(plan.rans_workspace_bytes(), dtype=torch.uint8, device="cuda")
        outs = [tmd.alloc_out(s) for s in shapes]
        for rep in range(2):
            plan.decode_rans(coded, outs, ws, rws)
            torch.cuda.synchronize()
            for i, f in enumerate(frames):
                check(tmd, *oracle.decode(f), outs[i], plan.status(i), (mode, flags, rep, i))
        plan.free()


def test_coded_and_plain_calls_alternate_on_one_graph_plan(tmd):
    """A graph plan decodes uncoded frames (its captured graph, k_unattached
    doing the unattached clusters) and coded ones (the entropy decoding
    placing them) in turn; every call equals the oracle."""
    import torch
    frames = [synth.make_frame(synth.spec_for("frame", collisions=2)), _long_bins(34, "over")]
    shapes = [tmd.frame_shape(f) for f in frames]
    devs = [tmd.to_device(f) for f in frames]
    coded = [torch.from_numpy(oracle.rans_encode(f)).cuda() for f in frames]
    expected = [oracle.decode(f) for f in frames]
    plan = tmd.Plan(shapes, flags=tmd.PLAN_GRAPH)
    ws = plan.alloc_workspace()
    rws = torch.empty(plan.rans_workspace_bytes(), dtype=torch.uint8, device="cuda")
    outs = [tmd.alloc_out(s) for s in shapes]
    for rep, kind in enumerate(("plain", "coded", "plain", "coded")):
        for o in outs:
            o["time"].fill_(-1)
        if kind == "plain":
            plan.decode(devs, outs, ws)
        else:
            plan.decode_rans(coded, outs, ws, rws)
        torch.cuda.synchronize()
        for i in range(len(frames)):
            check(tmd, *expected[i], outs[i], plan.status(i), (rep, kind, i))
    plan.free()


def test_rejected_call_enqueues_nothing(tmd):
    """A tmd_decode_rans call whose output is too small is rejected before any
    of its work is enqueued; the next valid call decodes as the oracle does."""
    import torch
    from paper_2411_02206_amd import _lib
    fr = synth.make_frame(synth.spec_for("tiny"))
    shape = tmd.frame_shape(fr)
    coded = [torch.from_numpy(oracle.rans_encode(fr)).cuda()]
    plan = tmd.Plan([shape])
    ws = plan.alloc_workspace()
    rws = torch.empty(plan.rans_workspace_bytes(), dtype=torch.uint8, device="cuda")
    small = tmd.alloc_out(shape, capacity=shape[1] + shape[2] - 1)
    with pytest.raises(_lib.TmdError) as err:
        plan.decode_rans(coded, [small], ws, rws)
    assert err.value.code == _lib.E_CAPACITY
    out = tmd.alloc_out(shape)
    plan.decode_rans(coded, [out], ws, rws)
    torch.cuda.synchronize()
    check(tmd, *oracle.decode(fr), out, plan.status(0), "after a rejected call")
    plan.free()


@pytest.mark.parametrize("array", ["trk_time0", "un_count", "un_time_diff", "cls_pad_res"])
def test_malformed_chunk_of_one_array_is_flagged(tmd, array):
    """A chunk whose stored state is out of range, in one array only: the
    frame is flagged whichever phase and stream decodes that array (the
    4-byte arrays decoded beside the others, the unattached ones beside the
    attached decode)."""
    from test_oracle_rans import WIDTH, planes
    fr = synth.make_frame(synth.spec_for("tiny"))
    shape = oracle.frame_sizes(fr)
    blob = oracle.rans_encode(fr)
    a = [k for k, _ in oracle.RANS_ARRAYS].index(array)
    p = sum(WIDTH[:a])  # the array's first plane
    n, f, table, data0 = planes(blob, shape)[p]
    assert n > 0
    bad = blob.copy()
    bad[data0 + int(table[0]):data0 + int(table[0]) + 4] = 0  # lane 0's state: 0 < 2^16
    out, flags = tmd.decode_rans(bad, shape)
    assert flags & tmd.F_CODED, (array, flags)
    out, flags = tmd.decode_rans(blob, shape)
    assert not flags & tmd.F_CODED


@pytest.mark.parametrize("seed", range(6))
def test_coded_random_frames(tmd, seed):
    """Random streams of random sizes (unattached clusters from none to
    several chunks, bin counts spread evenly, skewed or in a few bins, and
    adding up to n_unattached or not), entropy-coded and decoded in one
    batched call, each frame against the oracle."""
    import torch
    rng = np.random.default_rng(100 + seed)
    frames = []
    for i in range(3):
        nt = int(rng.integers(0, 600))
        na = int(rng.integers(0, 40000))
        w = rng.random(NBIN) ** float(rng.choice([1.0, 4.0, 16.0]))
        total = int(rng.choice([0, 5, 20000, 90000]))
        cnt = np.floor(w / w.sum() * total).astype(np.int64) if total else np.zeros(NBIN, np.int64)
        nu = int(cnt.sum()) + int(rng.choice([0, 0, 7, -3])) if total else 0
        fr = _garbage(200 + 10 * seed + i, nt=nt, na=na, nu=max(nu, 0))
        fr["un_count"] = cnt.astype(np.uint32)
        frames.append(fr)
    shapes = [tmd.frame_shape(f) for f in frames]
    coded = [torch.from_numpy(oracle.rans_encode(f)).cuda() for f in frames]
    print(f"random coded frames, seed {seed}: {shapes}", flush=True)
    plan = tmd.Plan(shapes, flags=tmd.PLAN_GRAPH if seed % 2 else 0, bz=5.0 if seed % 3 == 0 else 0.5)
    ws = plan.alloc_workspace()
    rws = torch.empty(plan.rans_workspace_bytes(), dtype=torch.uint8, device="cuda")
    outs = [tmd.alloc_out(s) for s in shapes]
    plan.decode_rans(coded, outs, ws, rws)
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        check(tmd, *oracle.decode(f, bz=5.0 if seed % 3 == 0 else 0.5), outs[i], plan.status(i), (seed, i))
    plan.free()

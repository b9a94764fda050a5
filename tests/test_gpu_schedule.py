"""Scheduling knobs of the attached decode (tmd_set_schedule: tracks per
wave 64..128 with lane packing, persistent grid) never change a result:
every setting is bit-identical to the oracle, for single frames (with the
SIMD balancing exercised by a small SIMD count), batched plans, graph
replays, capacity plans, loopers and garbage streams."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import _garbage

pytestmark = pytest.mark.gpu

SETTINGS = [(64, 0), (72, 0), (80, 0), (96, 0), (128, 0), (64, 2), (80, 3), (128, 1), (100, 64)]


@pytest.fixture(scope="module")
def tmd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_02206_amd as m
    return m


@pytest.fixture(scope="module")
def frames():
    specs = synth.batch_specs("batched", n_frames=4, coll_range=(1, 4))
    fr = synth.make_frames(specs)
    fr.append(synth.make_frame(synth.spec_for("stress", collisions=2)))
    fr.append(_garbage(11, nt=900, na=70000, nu=20000))
    return fr


@pytest.fixture(scope="module")
def expected(frames):
    return [oracle.decode(f, bz=0.5) for f in frames]


def check(tmd, exp, est, out, flags, label):
    got = tmd.to_numpy(out)
    for k in exp:
        assert np.array_equal(exp[k], got[k]), (label, k)
    assert flags == est, (label, flags, est)


@pytest.mark.parametrize("tpw,persist", SETTINGS)
def test_single_frames_every_setting(tmd, frames, expected, tpw, persist, monkeypatch):
    import torch
    monkeypatch.setenv("TMD_ATTACHED_SIMDS", "5")
    for i, fr in enumerate(frames):
        shape = tmd.frame_shape(fr)
        for gflags in (0, tmd.PLAN_GRAPH):
            plan = tmd.Plan([shape], flags=gflags)
            plan.set_schedule(tpw, persist)
            ws = plan.alloc_workspace()
            dev = tmd.to_device(fr)
            out = tmd.alloc_out(shape)
            for rep in range(2):
                out["time"].fill_(-1)
                plan.decode([dev], [out], ws)
                torch.cuda.synchronize()
                check(tmd, *expected[i], out, plan.status(0), (tpw, persist, i, gflags, rep))
            plan.free()


@pytest.mark.parametrize("tpw,persist", SETTINGS)
def test_batched_plan_every_setting(tmd, frames, expected, tpw, persist):
    import torch
    shapes = [tmd.frame_shape(f) for f in frames]
    plan = tmd.Plan(shapes, flags=tmd.PLAN_GRAPH)
    plan.set_schedule(tpw, persist)
    ws = plan.alloc_workspace()
    ins = [tmd.to_device(f) for f in frames]
    outs = [tmd.alloc_out(s) for s in shapes]
    for rep in range(2):
        plan.decode(ins, outs, ws)
        torch.cuda.synchronize()
        for i in range(len(frames)):
            check(tmd, *expected[i], outs[i], plan.status(i), (tpw, persist, i, rep))
    plan.free()


def test_schedule_changes_between_calls(tmd, frames, expected):
    """One capacity plan whose schedule changes between calls (eager and
    graph: the graph is captured again), decoding frames smaller than its
    capacity."""
    import torch
    shapes = [tmd.frame_shape(f) for f in frames]
    cap = tuple(max(s[i] for s in shapes) + 3 for i in range(3))
    for gflags in (0, tmd.PLAN_GRAPH):
        plan = tmd.Plan([cap], flags=gflags)
        ws = plan.alloc_workspace()
        for j, (tpw, persist) in enumerate(SETTINGS):
            plan.set_schedule(tpw, persist)
            i = j % len(frames)
            out = tmd.alloc_out(shapes[i])
            plan.decode([tmd.to_device(frames[i])], [out], ws, shapes=[shapes[i]])
            torch.cuda.synchronize()
            check(tmd, *expected[i], out, plan.status(0), (gflags, tpw, persist, i))
        plan.free()


def test_schedule_rejects_bad_values(tmd):
    plan = tmd.Plan([(10, 100, 10)])
    for tpw, persist in ((63, 0), (129, 0), (64, 65)):
        with pytest.raises(tmd.TmdError):
            plan.set_schedule(tpw, persist)
    plan.free()

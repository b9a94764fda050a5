"""tmd_decode_static, the entry point that allocates nothing (its workspace
is the library's static scratch array), called through the C ABI: two calls
in a row, the second with a smaller frame, each bit-identical to
tmd_decode_shapes with a caller-allocated workspace (and to the oracle), in
eager and graph plans; a plan whose workspace exceeds the scratch is
rejected before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tmd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_02206_amd as m
    return m


def structs(tmd, dev, out):
    from paper_2411_02206_amd import _lib
    fin = (_lib.FrameIn * 1)()
    fout = (_lib.FrameOut * 1)()
    for k in tmd.IN_FIELDS:
        t = dev[k]
        setattr(fin[0], k, C.c_void_p(t.data_ptr()) if t is not None and t.numel() else None)
    for k in tmd.OUT_FIELDS:
        setattr(fout[0], k, C.c_void_p(out[k].data_ptr()))
    fout[0].capacity = int(out["capacity"])
    return fin, fout


def equal(a, b):
    return all(np.array_equal(a[k], b[k]) for k in a)


@pytest.mark.parametrize("flags", [0, 1])
def test_static_equals_workspace_entry_two_calls(tmd, flags):
    import torch
    from paper_2411_02206_amd import _lib
    L = _lib.lib()
    big = synth.make_frame(synth.spec_for("frame", collisions=3))
    small = synth.make_frame(synth.spec_for("stress", collisions=1))
    shapes = [tmd.frame_shape(f) for f in (big, small)]
    assert all(a > b for a, b in zip(shapes[0], shapes[1]))
    plan = tmd.Plan([shapes[0]], flags=flags)       # capacity: the larger frame
    ref_plan = tmd.Plan([shapes[0]], flags=flags)
    ws = ref_plan.alloc_workspace()
    assert plan.workspace_bytes <= tmd.STATIC_SCRATCH_BYTES
    stream = torch.cuda.current_stream()
    for i, fr in enumerate((big, small)):           # the second call: a smaller frame
        dev = tmd.to_device(fr)
        out = tmd.alloc_out(shapes[i])
        ref = tmd.alloc_out(shapes[i])
        for o in (out, ref):
            o["time"].fill_(-1)
            o["pad"].fill_(-1)
        sh = (_lib.FrameShape * 1)(_lib.FrameShape(*shapes[i]))
        fin, fout = structs(tmd, dev, out)
        rc = L.tmd_decode_static(plan._h, sh, fin, fout, C.c_void_p(stream.cuda_stream))
        assert rc == 0, L.tmd_strerror(rc)
        ref_plan.decode([dev], [ref], ws, shapes=[shapes[i]])
        torch.cuda.synchronize()
        got, want = tmd.to_numpy(out), tmd.to_numpy(ref)
        assert equal(want, got), (flags, i)
        assert plan.status(0) == ref_plan.status(0)
        exp, est = oracle.decode(fr)
        assert equal(exp, got), (flags, i)
        assert plan.status(0) == est
    plan.free()
    ref_plan.free()


def test_static_rejects_workspace_beyond_scratch(tmd):
    from paper_2411_02206_amd import _lib
    L = _lib.lib()
    plan = tmd.Plan([(1 << 20, 40_000_000, 0)])
    assert plan.workspace_bytes > tmd.STATIC_SCRATCH_BYTES
    fin = (_lib.FrameIn * 1)()
    fout = (_lib.FrameOut * 1)()
    rc = L.tmd_decode_static(plan._h, None, fin, fout, None)
    assert rc == tmd.E_SCRATCH
    assert b"static scratch" in L.tmd_strerror(rc)
    plan.free()

"""TPC track-model decoding on AMD MI355X (arXiv:2411.02206, section 4).

Python front end of libtmd.so.  PyTorch supplies device memory and streams;
all decoding runs in the library's HIP kernels.

    import paper_2411_02206_amd as tmd
    dev = tmd.to_device(frame)              # numpy frame dict -> torch tensors on cuda
    out, flags = tmd.decode(dev, bz=0.5)    # torch tensors on cuda + status flags

Lower level: tmd.Plan(shapes, bz) / plan.decode(ins, outs, workspace, stream).
"""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import (E_ARG, E_CAPACITY, E_HIP, E_INPUT, E_SCRATCH, E_STREAM, F_CODED, F_COUNT, F_HDR, F_PAD,  # noqa: F401
                   F_ROT, F_ROW, F_SEC, F_SNP, F_TIME, IN_FIELDS, NBIN, NROW, NSEC, OK, OUT_FIELDS, PLAN_GRAPH,
                   STATIC_SCRATCH_BYTES, TmdError)

__all__ = ["Plan", "Pipeline", "decode", "decode_rans", "encode", "to_device", "to_host", "alloc_out", "alloc_host_out", "to_numpy",
           "version", "tables"]

# element types of the frame arrays; unsigned 16/32-bit data travel in signed
# torch tensors of the same width (only the bytes matter to the library)
IN_DTYPES = {
    "trk_ncls": np.uint8, "trk_sec0": np.uint8, "trk_row0": np.uint8, "trk_pad0": np.uint16,
    "trk_time0": np.uint32, "trk_qpt": np.int16, "trk_snp": np.int16, "trk_tgl": np.int16,
    "cls_row_diff": np.int8, "cls_sec_diff": np.uint8, "cls_pad_res": np.int16,
    "cls_time_res": np.int16, "cls_qtot": np.uint16, "cls_qmax": np.uint16,
    "un_count": np.uint32, "un_time_diff": np.uint32, "un_pad_diff": np.uint16,
    "un_qtot": np.uint16, "un_qmax": np.uint16,
}
OUT_DTYPES = {"row_offset": np.uint32, "row_nattached": np.uint32, "time": np.uint32,
              "pad": np.uint16, "qtot": np.uint16, "qmax": np.uint16}
_SIGNED = {np.dtype(np.uint8): np.uint8, np.dtype(np.int8): np.int8, np.dtype(np.uint16): np.int16,
           np.dtype(np.int16): np.int16, np.dtype(np.uint32): np.int32, np.dtype(np.int32): np.int32}


def _torch():
    import torch
    return torch


def version():
    return _lib.lib().tmd_version().decode()


def tables(bz=0.5):
    """The library's float32 constant tables (host computation, no GPU)."""
    buf = (C.c_float * 2048)()
    n = _lib.lib().tmd_tables(C.c_float(bz), buf, 2048)
    v = np.frombuffer(buf, np.float32, n).copy()
    out, o = {}, 0
    for name in ("x", "pw", "inv_pw", "padoff", "pwq", "ks", "kt"):
        out[name] = v[o:o + NROW]
        o += NROW
    out["cosb"] = v[o:o + 18]; o += 18
    out["sinb"] = v[o:o + 18]; o += 18
    out["kb"], out["vdq"], out["inv_vd32"], out["snp_max"] = v[o:o + 4]
    return out


def frame_shape(frame):
    """(n_tracks, n_attached, n_unattached) of a frame dict (numpy or torch)."""
    return (int(frame["trk_ncls"].shape[0]), int(frame["cls_qtot"].shape[0]),
            int(frame["un_qtot"].shape[0]))


def to_device(frame, device="cuda"):
    """Copy a numpy frame dict to torch tensors on `device`."""
    torch = _torch()
    out = {}
    for k in IN_FIELDS:
        a = np.ascontiguousarray(frame[k], dtype=IN_DTYPES[k])
        out[k] = torch.from_numpy(a.view(_SIGNED[a.dtype])).to(device)
    return out


def alloc_out(shape, device="cuda", capacity=None):
    torch = _torch()
    n = shape[1] + shape[2] if capacity is None else capacity
    tt = {np.uint32: torch.int32, np.uint16: torch.int16}
    return {"row_offset": torch.empty(NBIN + 1, dtype=torch.int32, device=device),
            "row_nattached": torch.empty(NBIN, dtype=torch.int32, device=device),
            "time": torch.empty(max(n, 1), dtype=tt[np.uint32], device=device),
            "pad": torch.empty(max(n, 1), dtype=tt[np.uint16], device=device),
            "qtot": torch.empty(max(n, 1), dtype=tt[np.uint16], device=device),
            "qmax": torch.empty(max(n, 1), dtype=tt[np.uint16], device=device),
            "capacity": n}


def to_numpy(out):
    """Device outputs -> numpy arrays with their unsigned types, cut to the
    decoded size."""
    res = {k: out[k].cpu().numpy().view(OUT_DTYPES[k]) for k in OUT_FIELDS}
    n = int(res["row_offset"][NBIN])
    for k in ("time", "pad", "qtot", "qmax"):
        res[k] = res[k][:n]
    return res


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


class Plan:
    """A decode plan for frames of fixed shapes (one frame: plain decode; many:
    batched decode in one launch sequence)."""

    def __init__(self, shapes, bz=0.5, flags=0):
        L = _lib.lib()
        shapes = [tuple(int(v) for v in s) for s in shapes]
        arr = (_lib.FrameShape * len(shapes))(*[_lib.FrameShape(*s) for s in shapes])
        self._params = _lib.Params(float(bz), int(flags))
        h = C.c_void_p()
        ws = C.c_size_t()
        _lib.check(L.tmd_plan(arr, len(shapes), C.byref(self._params), C.byref(h), C.byref(ws)),
                   "tmd_plan")
        self._h = h
        self.shapes = shapes
        self.bz = bz
        self.workspace_bytes = int(ws.value)
        self._keep = None

    def __del__(self):
        self.free()

    def free(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.lib().tmd_free(h)
            self._h = None

    def alloc_workspace(self, device="cuda"):
        torch = _torch()
        return torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=device)

    def decode(self, ins, outs, workspace, stream=None, shapes=None):
        """Enqueue the decode of len(shapes) frames.  ins/outs: lists of dicts of
        device tensors (see to_device / alloc_out).  stream: torch stream or
        None for the current one.  shapes: the frames' own shapes if they are
        smaller than the planned ones (tmd_decode_shapes); None: as planned."""
        torch = _torch()
        n = len(self.shapes)
        if len(ins) != n or len(outs) != n:
            raise ValueError(f"plan has {n} frames")
        fin = (_lib.FrameIn * n)()
        fout = (_lib.FrameOut * n)()
        for i in range(n):
            for k in IN_FIELDS:
                setattr(fin[i], k, _ptr(ins[i][k]))
            for k in OUT_FIELDS:
                setattr(fout[i], k, _ptr(outs[i][k]))
            fout[i].capacity = int(outs[i]["capacity"])
        if stream is None:
            stream = torch.cuda.current_stream()
        sp = C.c_void_p(stream.cuda_stream)
        if shapes is None:
            _lib.check(_lib.lib().tmd_decode(self._h, fin, fout, _ptr(workspace), sp), "tmd_decode")
        else:
            if len(shapes) != n:
                raise ValueError(f"plan has {n} frames")
            arr = (_lib.FrameShape * n)(*[_lib.FrameShape(*(int(v) for v in sh)) for sh in shapes])
            _lib.check(_lib.lib().tmd_decode_shapes(self._h, arr, fin, fout, _ptr(workspace), sp),
                       "tmd_decode_shapes")

    def decode_static(self, ins, outs, stream=None, shapes=None):
        """As decode, with the library's static scratch as the workspace
        (tmd_decode_static: no device memory is allocated by the call)."""
        torch = _torch()
        n = len(self.shapes)
        if len(ins) != n or len(outs) != n or (shapes is not None and len(shapes) != n):
            raise ValueError(f"plan has {n} frames")
        fin = (_lib.FrameIn * n)()
        fout = (_lib.FrameOut * n)()
        for i in range(n):
            for k in IN_FIELDS:
                setattr(fin[i], k, _ptr(ins[i][k]))
            for k in OUT_FIELDS:
                setattr(fout[i], k, _ptr(outs[i][k]))
            fout[i].capacity = int(outs[i]["capacity"])
        if stream is None:
            stream = torch.cuda.current_stream()
        arr = None
        if shapes is not None:
            arr = (_lib.FrameShape * n)(*[_lib.FrameShape(*(int(v) for v in sh)) for sh in shapes])
        _lib.check(_lib.lib().tmd_decode_static(self._h, arr, fin, fout, C.c_void_p(stream.cuda_stream)),
                   "tmd_decode_static")

    def rans_workspace_bytes(self, shapes=None):
        shapes = shapes or self.shapes
        arr = (_lib.FrameShape * len(shapes))(*[_lib.FrameShape(*(int(v) for v in sh)) for sh in shapes])
        b = C.c_size_t()
        _lib.check(_lib.lib().tmd_rans_workspace(arr, len(shapes), C.byref(b)), "tmd_rans_workspace")
        return int(b.value)

    def decode_rans(self, coded, outs, workspace, rans_workspace, stream=None, shapes=None):
        """Entropy-decode the coded frames (device uint8 tensors in the format
        of include/tmd.h) and decode them (tmd_decode_rans): the track and
        attached arrays go through rans_workspace, the unattached ones
        straight into the outputs."""
        torch = _torch()
        n = len(self.shapes)
        shapes = shapes or self.shapes
        if len(coded) != n or len(outs) != n or len(shapes) != n:
            raise ValueError(f"plan has {n} frames")
        arr = (_lib.FrameShape * n)(*[_lib.FrameShape(*(int(v) for v in sh)) for sh in shapes])
        ptrs = (C.c_void_p * n)(*[c.data_ptr() for c in coded])
        sizes = (C.c_uint64 * n)(*[c.numel() for c in coded])
        fout = (_lib.FrameOut * n)()
        for i in range(n):
            for k in OUT_FIELDS:
                setattr(fout[i], k, _ptr(outs[i][k]))
            fout[i].capacity = int(outs[i]["capacity"])
        if stream is None:
            stream = torch.cuda.current_stream()
        _lib.check(_lib.lib().tmd_decode_rans(self._h, arr, ptrs, sizes, fout, _ptr(workspace), _ptr(rans_workspace),
                                              C.c_void_p(stream.cuda_stream)), "tmd_decode_rans")

    def status(self, frame=0):
        """Flag bits of `frame` from the last decode (waits for it)."""
        f = C.c_uint32()
        rc = _lib.lib().tmd_status(self._h, frame, C.byref(f))
        if rc not in (OK, E_INPUT, E_STREAM):
            _lib.check(rc, "tmd_status")
        return int(f.value)

    def set_schedule(self, tracks_per_wave=64, persist=0):
        """Scheduling knobs of the attached decode (tmd_set_schedule): tracks
        per wave (64..128) and persistent waves per SIMD (0: off).  Results
        do not depend on them."""
        _lib.check(_lib.lib().tmd_set_schedule(self._h, int(tracks_per_wave), int(persist)), "tmd_set_schedule")
        self.schedule = (int(tracks_per_wave), int(persist))

    def set_profiling(self, on=True, stages=None):
        """Record events around every stage (on=True), none (False), or the
        named stages only (stages: iterable of stage names)."""
        L = _lib.lib()
        if stages is not None:
            names = [L.tmd_stage_name(i).decode() for i in range(16)]
            mask = 0
            for st in set(stages):
                mask |= 1 << names.index(st)
        else:
            mask = 0xFFFFFFFF if on else 0
        _lib.check(L.tmd_set_profiling(self._h, mask), "tmd_set_profiling")

    def stage_times(self):
        """{stage: summed ms} over the profiled calls since the last read, and
        the number of calls."""
        L = _lib.lib()
        buf = (C.c_double * 16)()
        calls = C.c_uint32()
        n = L.tmd_stage_times(self._h, buf, 16, C.byref(calls))
        if n < 0:
            _lib.check(n, "tmd_stage_times")
        return {L.tmd_stage_name(i).decode(): buf[i] for i in range(n)}, int(calls.value)


ENC_DTYPES = {"trk_first": np.uint32, "trk_qpt": np.float64, "trk_tgl": np.float64, "cl_sec": np.uint8,
              "cl_row": np.uint8, "cl_pad": np.float64, "cl_time": np.float64, "cl_snp": np.float64,
              "cl_qtot": np.uint16, "cl_qmax": np.uint16, "un_sec": np.uint8, "un_row": np.uint8,
              "un_pad": np.float64, "un_time": np.float64, "un_qtot": np.uint16, "un_qmax": np.uint16}


def enc_to_device(phys, device="cuda"):
    """Physical clusters (dict keyed as ENC_DTYPES) -> device tensors (the
    input of encode_device)."""
    torch = _torch()
    dev = {}
    for k, dt in ENC_DTYPES.items():
        a = np.ascontiguousarray(phys[k], dtype=dt)
        if a.dtype == np.float64:
            dev[k] = torch.from_numpy(a).to(device)
        else:
            dev[k] = torch.from_numpy(a.view(_SIGNED[a.dtype])).to(device)
    return dev


def enc_shape(dev):
    """(tracks, attached clusters, unattached clusters) of device or host
    physical clusters."""
    return (int(dev["trk_qpt"].shape[0]), int(dev["cl_pad"].shape[0]), int(dev["un_pad"].shape[0]))


def alloc_enc_out(nt, n, nu, device="cuda"):
    """Device arrays of the compressed frame tmd_encode writes (header arrays
    sized for one header per cluster at most) and its 3 count words
    ("counts")."""
    torch = _torch()
    sizes = {"trk": max(n, 1), "cls": max(n, 1), "un": max(nu, 1)}
    out = {}
    for k in IN_FIELDS:
        dt = _SIGNED[np.dtype(IN_DTYPES[k])]
        cnt = NBIN if k == "un_count" else sizes[k.split("_")[0]]
        out[k] = torch.empty(cnt, dtype=getattr(torch, np.dtype(dt).name), device=device)
    out["counts"] = torch.zeros(4, dtype=torch.int32, device=device)
    return out


def enc_workspace_bytes(nt, n, nu):
    wsb = C.c_size_t()
    _lib.check(_lib.lib().tmd_encode_workspace(nt, n, nu, C.byref(wsb)), "tmd_encode_workspace")
    return int(wsb.value)


def encode_device(plan, dev, out, ws, stream):
    """Enqueue tmd_encode of device physical clusters `dev` (enc_to_device)
    into `out` (alloc_enc_out) with the caller's workspace tensor `ws` on
    `stream`; no synchronisation."""
    L = _lib.lib()
    nt, n, nu = enc_shape(dev)
    ein = _lib.EncIn(nt, n, nu)
    for k in _lib.ENC_IN_TRACK + _lib.ENC_IN_CLUSTER + _lib.ENC_IN_UNATT:
        setattr(ein, k, _ptr(dev[k]))
    eout = _lib.EncOut()
    for k in IN_FIELDS:
        setattr(eout, k, _ptr(out[k]))
    eout.counts = _ptr(out["counts"])
    _lib.check(L.tmd_encode(plan._h, C.byref(ein), C.byref(eout), _ptr(ws), int(ws.numel()),
                            C.c_void_p(stream.cuda_stream)), "tmd_encode")


def enc_result(out, n, nu):
    """The compressed frame written by encode_device as numpy arrays, cut to
    the header count, and the number of headers opened inside a track.
    Raises TmdError if the input was outside the codable range."""
    c = out["counts"].cpu().numpy().view(np.uint32)
    if c[2]:
        raise TmdError(E_INPUT, "tmd_encode: input outside the codable range")
    res = {}
    for k in IN_FIELDS:
        a = out[k].cpu().numpy().view(IN_DTYPES[k])
        if k.startswith("trk_"):
            a = a[:int(c[0])]
        elif k.startswith("cls_"):
            a = a[:n]
        elif k != "un_count":
            a = a[:nu]
        res[k] = a.copy()
    return res, int(c[1])


def encode(phys, bz=0.5, device="cuda", stream=None, plan=None):
    """Encode physical clusters (dict of arrays, keys as ENC_DTYPES: tracks
    by trk_first ranges, pads and times as doubles) on the GPU into a
    compressed frame (tmd_encode).  Returns (frame dict of numpy arrays, number
    of headers opened inside a track).  Raises TmdError on an input outside
    the codable range."""
    torch = _torch()
    dev = enc_to_device(phys, device)
    nt, n, nu = enc_shape(dev)
    out = alloc_enc_out(nt, n, nu, device)
    ws = torch.empty(max(enc_workspace_bytes(nt, n, nu), 256), dtype=torch.uint8, device=device)
    own = plan is None
    if own:
        plan = Plan([(1, 1, 1)], bz=bz)
    if stream is None:
        stream = torch.cuda.current_stream()
    try:
        encode_device(plan, dev, out, ws, stream)
        stream.synchronize()
        return enc_result(out, n, nu)
    finally:
        if own:
            plan.free()


def decode_rans(coded, shape, bz=0.5, device="cuda"):
    """Decode one entropy-coded frame (bytes in the format of include/tmd.h,
    numpy or a device tensor) of the given shape.  Returns (outputs, flags)."""
    torch = _torch()
    if not hasattr(coded, "is_cuda"):
        coded = torch.from_numpy(np.ascontiguousarray(coded, np.uint8)).to(device)
    shape = tuple(int(v) for v in shape)
    plan = Plan([shape], bz=bz)
    out = alloc_out(shape, device)
    ws = plan.alloc_workspace(device)
    rws = torch.empty(max(plan.rans_workspace_bytes(), 256), dtype=torch.uint8, device=device)
    plan.decode_rans([coded], [out], ws, rws)
    flags = plan.status(0)
    plan.free()
    return out, flags


def rans_encode_sizes(shape):
    """(workspace bytes, largest coded size) of tmd_encode_rans for a frame of `shape`."""
    ws, bound = C.c_size_t(), C.c_uint64()
    sh = _lib.FrameShape(*(int(v) for v in shape))
    _lib.check(_lib.lib().tmd_rans_encode_workspace(C.byref(sh), C.byref(ws), C.byref(bound)),
               "tmd_rans_encode_workspace")
    return int(ws.value), int(bound.value)


def encode_rans(frame, stream=None, workspace=None):
    """Entropy-code a frame held in device tensors (see to_device) with
    tmd_encode_rans.  Returns the coded bytes as a device uint8 tensor."""
    torch = _torch()
    shape = frame_shape(frame)
    dev = frame["trk_ncls"].device
    ws_bytes, bound = rans_encode_sizes(shape)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
    coded = torch.empty(bound, dtype=torch.uint8, device=dev)
    size = torch.zeros(1, dtype=torch.int64, device=dev)
    fin = _lib.FrameIn()
    for k in IN_FIELDS:
        setattr(fin, k, _ptr(frame[k]))
    if stream is None:
        stream = torch.cuda.current_stream()
    sh = _lib.FrameShape(*shape)
    _lib.check(_lib.lib().tmd_encode_rans(C.byref(sh), C.byref(fin), _ptr(coded), bound, _ptr(size),
                                          _ptr(workspace), C.c_void_p(stream.cuda_stream)), "tmd_encode_rans")
    stream.synchronize()
    return coded[:int(size.item())]


def to_host(frame, pin=True):
    """Copy a numpy frame dict to torch CPU tensors, page-locked if `pin`
    (what lets a Pipeline's transfers overlap its kernels)."""
    torch = _torch()
    out = {}
    for k in IN_FIELDS:
        a = np.ascontiguousarray(frame[k], dtype=IN_DTYPES[k])
        t = torch.from_numpy(a.view(_SIGNED[a.dtype]))
        out[k] = t.pin_memory() if pin else t.clone()
    return out


def pin_bytes(data):
    """A copy of `data` (numpy uint8 or a CPU/device tensor) in page-locked
    host memory, as a uint8 CPU tensor (for Pipeline.run_rans)."""
    torch = _torch()
    if hasattr(data, "is_cuda"):
        data = data.cpu()
    else:
        data = torch.from_numpy(np.ascontiguousarray(data, np.uint8))
    return data.pin_memory()


def alloc_host_out(shape, pin=True, capacity=None):
    """Host output buffers (torch CPU tensors, page-locked if `pin`) for a
    frame of `shape`; same keys and types as alloc_out."""
    torch = _torch()
    n = shape[1] + shape[2] if capacity is None else capacity
    tt = {np.uint32: torch.int32, np.uint16: torch.int16}
    mk = (lambda m, dt: torch.empty(m, dtype=dt, pin_memory=True)) if pin else \
        (lambda m, dt: torch.empty(m, dtype=dt))
    return {"row_offset": mk(NBIN + 1, torch.int32), "row_nattached": mk(NBIN, torch.int32),
            "time": mk(max(n, 1), tt[np.uint32]), "pad": mk(max(n, 1), tt[np.uint16]),
            "qtot": mk(max(n, 1), tt[np.uint16]), "qmax": mk(max(n, 1), tt[np.uint16]), "capacity": n}


class Pipeline:
    """Decoding of host-resident frames through `depth` slots (stream, plan,
    device buffers each) used in turn: frame i is copied in, decoded and
    copied back on slot i % depth, so transfers overlap other slots' kernels
    (tmd_pipe_create / tmd_pipe_run)."""

    def __init__(self, capacity, depth=3, bz=0.5):
        L = _lib.lib()
        self._params = _lib.Params(float(bz), 0)
        cap = _lib.FrameShape(*(int(v) for v in capacity))
        h = C.c_void_p()
        _lib.check(L.tmd_pipe_create(C.byref(cap), int(depth), C.byref(self._params), C.byref(h)),
                   "tmd_pipe_create")
        self._h = h
        self.capacity = tuple(int(v) for v in capacity)
        self.depth = int(depth)

    def __del__(self):
        self.free()

    def free(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.lib().tmd_pipe_free(h)
            self._h = None

    def run(self, frames, outs, shapes=None):
        """Decode host frames (dicts of CPU tensors, see to_host) into host
        outputs (see alloc_host_out).  Returns the list of status flags; raises
        TmdError on an argument or runtime error."""
        n = len(frames)
        if len(outs) != n:
            raise ValueError("one output dict per frame")
        if shapes is None:
            shapes = [frame_shape(f) for f in frames]
        sh = (_lib.FrameShape * max(n, 1))(*[_lib.FrameShape(*(int(v) for v in s)) for s in shapes])
        fin = (_lib.FrameIn * max(n, 1))()
        fout = (_lib.FrameOut * max(n, 1))()
        for i in range(n):
            for k in IN_FIELDS:
                setattr(fin[i], k, _ptr(frames[i][k]))
            for k in OUT_FIELDS:
                setattr(fout[i], k, _ptr(outs[i][k]))
            fout[i].capacity = int(outs[i]["capacity"])
        flags = (C.c_uint32 * max(n, 1))()
        rc = _lib.lib().tmd_pipe_run(self._h, n, sh, fin, fout, flags)
        if rc not in (OK, E_INPUT, E_STREAM):
            _lib.check(rc, "tmd_pipe_run")
        return [int(flags[i]) for i in range(n)]

    def run_rans(self, coded, shapes, outs):
        """Decode entropy-coded frames held in host memory (uint8 CPU tensors,
        page-locked for overlap; see pin_bytes) of the given shapes into host
        outputs (tmd_pipe_run_rans).  Returns the list of status flags."""
        n = len(coded)
        if len(outs) != n or len(shapes) != n:
            raise ValueError("one shape and one output dict per coded frame")
        sh = (_lib.FrameShape * max(n, 1))(*[_lib.FrameShape(*(int(v) for v in s)) for s in shapes])
        ptrs = (C.c_void_p * max(n, 1))(*[c.data_ptr() for c in coded])
        sizes = (C.c_uint64 * max(n, 1))(*[c.numel() for c in coded])
        fout = (_lib.FrameOut * max(n, 1))()
        for i in range(n):
            for k in OUT_FIELDS:
                setattr(fout[i], k, _ptr(outs[i][k]))
            fout[i].capacity = int(outs[i]["capacity"])
        flags = (C.c_uint32 * max(n, 1))()
        rc = _lib.lib().tmd_pipe_run_rans(self._h, n, sh, ptrs, sizes, fout, flags)
        if rc not in (OK, E_INPUT, E_STREAM):
            _lib.check(rc, "tmd_pipe_run_rans")
        return [int(flags[i]) for i in range(n)]


def decode(frame, bz=0.5, stream=None):
    """Decode one frame held in device tensors (see to_device).  Returns
    (outputs dict of device tensors, status flags)."""
    shape = frame_shape(frame)
    dev = frame["trk_ncls"].device
    plan = Plan([shape], bz)
    out = alloc_out(shape, dev)
    ws = plan.alloc_workspace(dev)
    plan.decode([frame], [out], ws, stream)
    flags = plan.status(0)
    plan.free()
    return out, flags


def selftest_fp(a, b, stream=None):
    """Device arithmetic (sqrt, div, rint, a*b+a with two roundings) of two
    float32 device tensors; returns a float32 tensor [n, 4]."""
    torch = _torch()
    n = a.numel()
    out = torch.empty(4 * max(n, 1), dtype=torch.float32, device=a.device)
    if stream is None:
        stream = torch.cuda.current_stream()
    _lib.check(_lib.lib().tmd_selftest_fp(_ptr(a), _ptr(b), _ptr(out), n, C.c_void_p(stream.cuda_stream)),
               "tmd_selftest_fp")
    return out[:4 * n].view(n, 4)


def selftest_math(a, stream=None):
    """The decode loop's square root, |sin phi| clamp (+ flag) and rounding to
    int32 of a float32 device tensor; returns an int32 tensor [n, 4] of raw
    words (see tmd_selftest_math)."""
    torch = _torch()
    n = a.numel()
    out = torch.empty(4 * max(n, 1), dtype=torch.int32, device=a.device)
    if stream is None:
        stream = torch.cuda.current_stream()
    _lib.check(_lib.lib().tmd_selftest_math(_ptr(a), _ptr(out), n, C.c_void_p(stream.cuda_stream)),
               "tmd_selftest_math")
    return out[:4 * n].view(n, 4)


def selftest_sqrt(lo_bits, hi_bits, device="cuda", stream=None):
    """Number of floats with bit patterns in [lo_bits, hi_bits) where the
    decode loop's square root differs from the IEEE one."""
    torch = _torch()
    cnt = torch.zeros(1, dtype=torch.int32, device=device)
    if stream is None:
        stream = torch.cuda.current_stream()
    _lib.check(_lib.lib().tmd_selftest_sqrt(lo_bits, hi_bits, _ptr(cnt), C.c_void_p(stream.cuda_stream)),
               "tmd_selftest_sqrt")
    return int(cnt.item())

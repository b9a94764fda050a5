"""ctypes front end of the plain C oracle -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the CPU-baseline leg of bench.py may import
this package.  The decoder here is the reference the GPU library is compared
with; it shares no code with the library.

Frames are dicts of numpy arrays with these keys (all little-endian):

  trk_ncls u8, trk_sec0 u8, trk_row0 u8, trk_pad0 u16, trk_time0 u32,
  trk_qpt i16, trk_snp i16, trk_tgl i16                       [n_tracks]
  cls_row_diff i8, cls_sec_diff u8, cls_pad_res i16, cls_time_res i16,
  cls_qtot u16, cls_qmax u16                                  [n_attached]
  un_count u32                                                [5472]
  un_time_diff u32, un_pad_diff u16, un_qtot u16, un_qmax u16 [n_unattached]

Decoded clusters come back as row_offset u32[5473], row_nattached u32[5472],
time u32, pad u16, qtot u16, qmax u16 [n_attached + n_unattached] and a status
word of flag bits.
"""
import ctypes as C
import os

import numpy as np

NSEC, NROW = 36, 152
NBIN = NSEC * NROW

F_HDR, F_SEC, F_ROW, F_ROT, F_SNP, F_PAD, F_TIME, F_COUNT = 1, 2, 4, 8, 16, 32, 64, 128

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

TRACK_FIELDS = [("trk_ncls", np.uint8), ("trk_sec0", np.uint8), ("trk_row0", np.uint8),
                ("trk_pad0", np.uint16), ("trk_time0", np.uint32), ("trk_qpt", np.int16),
                ("trk_snp", np.int16), ("trk_tgl", np.int16)]
CLUSTER_FIELDS = [("cls_row_diff", np.int8), ("cls_sec_diff", np.uint8), ("cls_pad_res", np.int16),
                  ("cls_time_res", np.int16), ("cls_qtot", np.uint16), ("cls_qmax", np.uint16)]
UNATT_FIELDS = [("un_time_diff", np.uint32), ("un_pad_diff", np.uint16), ("un_qtot", np.uint16),
                ("un_qmax", np.uint16)]
P = C.c_void_p


class _Stream(C.Structure):
    _fields_ = [("n_tracks", C.c_uint32), ("n_attached", C.c_uint32), ("n_unattached", C.c_uint32)] + \
        [(n, P) for n, _ in TRACK_FIELDS] + [(n, P) for n, _ in CLUSTER_FIELDS] + \
        [("un_count", P)] + [(n, P) for n, _ in UNATT_FIELDS]


class _Clusters(C.Structure):
    _fields_ = [("row_offset", P), ("row_nattached", P), ("time", P), ("pad", P), ("qtot", P),
                ("qmax", P), ("capacity", C.c_uint64)]


class _EncIn(C.Structure):
    _fields_ = [("n_tracks", C.c_uint32), ("trk_first", P), ("trk_qpt", P), ("trk_tgl", P),
                ("cl_sec", P), ("cl_row", P), ("cl_pad", P), ("cl_time", P), ("cl_snp", P),
                ("cl_qtot", P), ("cl_qmax", P), ("n_un", C.c_uint32), ("un_sec", P), ("un_row", P),
                ("un_pad", P), ("un_time", P), ("un_qtot", P), ("un_qmax", P)]


class _EncOut(C.Structure):
    _fields_ = [("n_tracks", C.c_uint32), ("n_attached", C.c_uint32), ("n_unattached", C.c_uint32)] + \
        [(n, P) for n, _ in TRACK_FIELDS] + [(n, P) for n, _ in CLUSTER_FIELDS] + \
        [("un_count", P)] + [(n, P) for n, _ in UNATT_FIELDS] + [("n_splits", C.c_uint32)]


def lib():
    """Load oracle/liboracle.so, building it first if it is not there."""
    global _LIB
    if _LIB is None:
        # TMD_ORACLE_LIB: another build of the same source (the sanitizer test)
        path = os.environ.get("TMD_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.oracle_decode.argtypes = [C.POINTER(_Stream), C.POINTER(_Clusters), C.c_float,
                                    C.POINTER(C.c_uint32)]
        L.oracle_decode.restype = C.c_int
        L.oracle_encode.argtypes = [C.POINTER(_EncIn), C.POINTER(_EncOut), C.c_float]
        L.oracle_encode.restype = C.c_int
        L.oracle_tables.argtypes = [C.c_float, C.POINTER(C.c_float), C.c_int]
        L.oracle_tables.restype = C.c_int
        L.oracle_npads.argtypes = [C.POINTER(C.c_int)]
        L.oracle_npads.restype = C.c_int
        L.oracle_sat.argtypes = [C.c_float]
        L.oracle_sat.restype = C.c_int32
        L.oracle_clamp_snp.argtypes = [C.c_float, C.POINTER(C.c_uint32)]
        L.oracle_clamp_snp.restype = C.c_float
        L.oracle_rans_bound.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
        L.oracle_rans_bound.restype = C.c_uint64
        L.oracle_rans_encode.argtypes = [C.POINTER(P), C.c_uint32, C.c_uint32, C.c_uint32, P, C.c_uint64]
        L.oracle_rans_encode.restype = C.c_uint64
        L.oracle_rans_decode.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(P)]
        L.oracle_rans_decode.restype = C.c_int
        L.oracle_fp_canary.argtypes = [C.c_float, C.c_float, C.c_float]
        L.oracle_fp_canary.restype = C.c_float
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(P) if a is not None and a.size else None


def _checked(frame, name, dtype, n):
    a = np.ascontiguousarray(frame[name])
    if a.dtype != dtype or a.shape != (n,):
        raise ValueError(f"{name}: expected {np.dtype(dtype)}[{n}], got {a.dtype}{list(a.shape)}")
    return a


def frame_sizes(frame):
    return (int(frame["trk_ncls"].shape[0]), int(frame["cls_qtot"].shape[0]),
            int(frame["un_qtot"].shape[0]))


def decode(frame, bz=0.5, capacity=None):
    """Decode one frame on the CPU.  Returns (clusters dict, status flags)."""
    nt, na, nu = frame_sizes(frame)
    keep = []
    s = _Stream(nt, na, nu)
    for name, dt in TRACK_FIELDS:
        a = _checked(frame, name, dt, nt); keep.append(a); setattr(s, name, _ptr(a))
    for name, dt in CLUSTER_FIELDS:
        a = _checked(frame, name, dt, na); keep.append(a); setattr(s, name, _ptr(a))
    a = _checked(frame, "un_count", np.uint32, NBIN); keep.append(a); s.un_count = _ptr(a)
    for name, dt in UNATT_FIELDS:
        a = _checked(frame, name, dt, nu); keep.append(a); setattr(s, name, _ptr(a))
    n = na + nu if capacity is None else capacity
    out = {"row_offset": np.zeros(NBIN + 1, np.uint32), "row_nattached": np.zeros(NBIN, np.uint32),
           "time": np.zeros(n, np.uint32), "pad": np.zeros(n, np.uint16),
           "qtot": np.zeros(n, np.uint16), "qmax": np.zeros(n, np.uint16)}
    c = _Clusters(*[_ptr(out[k]) for k in ("row_offset", "row_nattached", "time", "pad", "qtot", "qmax")],
                  n)
    st = C.c_uint32(0)
    rc = lib().oracle_decode(C.byref(s), C.byref(c), C.c_float(bz), C.byref(st))
    if rc != 0:
        raise RuntimeError(f"oracle_decode failed with code {rc}")
    total = int(out["row_offset"][NBIN])
    for k in ("time", "pad", "qtot", "qmax"):
        out[k] = out[k][:total]
    return out, int(st.value)


def encode(phys, bz=0.5):
    """Encode physical clusters (see oracle.physgen) into a compressed frame.

    Returns (frame dict, number of mid-track header restarts)."""
    nt = int(phys["trk_qpt"].shape[0])
    ncl = int(phys["cl_pad"].shape[0])
    nun = int(phys["un_pad"].shape[0])
    arrs = {
        "trk_first": np.ascontiguousarray(phys["trk_first"], np.uint32),
        "trk_qpt": np.ascontiguousarray(phys["trk_qpt"], np.float64),
        "trk_tgl": np.ascontiguousarray(phys["trk_tgl"], np.float64),
        "cl_sec": np.ascontiguousarray(phys["cl_sec"], np.uint8),
        "cl_row": np.ascontiguousarray(phys["cl_row"], np.uint8),
        "cl_pad": np.ascontiguousarray(phys["cl_pad"], np.float64),
        "cl_time": np.ascontiguousarray(phys["cl_time"], np.float64),
        "cl_snp": np.ascontiguousarray(phys["cl_snp"], np.float64),
        "cl_qtot": np.ascontiguousarray(phys["cl_qtot"], np.uint16),
        "cl_qmax": np.ascontiguousarray(phys["cl_qmax"], np.uint16),
        "un_sec": np.ascontiguousarray(phys["un_sec"], np.uint8),
        "un_row": np.ascontiguousarray(phys["un_row"], np.uint8),
        "un_pad": np.ascontiguousarray(phys["un_pad"], np.float64),
        "un_time": np.ascontiguousarray(phys["un_time"], np.float64),
        "un_qtot": np.ascontiguousarray(phys["un_qtot"], np.uint16),
        "un_qmax": np.ascontiguousarray(phys["un_qmax"], np.uint16),
    }
    ein = _EncIn(nt, _ptr(arrs["trk_first"]), _ptr(arrs["trk_qpt"]), _ptr(arrs["trk_tgl"]),
                 _ptr(arrs["cl_sec"]), _ptr(arrs["cl_row"]), _ptr(arrs["cl_pad"]), _ptr(arrs["cl_time"]),
                 _ptr(arrs["cl_snp"]), _ptr(arrs["cl_qtot"]), _ptr(arrs["cl_qmax"]), nun,
                 _ptr(arrs["un_sec"]), _ptr(arrs["un_row"]), _ptr(arrs["un_pad"]), _ptr(arrs["un_time"]),
                 _ptr(arrs["un_qtot"]), _ptr(arrs["un_qmax"]))
    cap = max(ncl, 1)
    out = {}
    for name, dt in TRACK_FIELDS + CLUSTER_FIELDS:
        out[name] = np.zeros(cap, dt)
    out["un_count"] = np.zeros(NBIN, np.uint32)
    for name, dt in UNATT_FIELDS:
        out[name] = np.zeros(max(nun, 1), dt)
    eo = _EncOut(0, 0, 0, *[_ptr(out[n]) for n, _ in TRACK_FIELDS + CLUSTER_FIELDS],
                 _ptr(out["un_count"]), *[_ptr(out[n]) for n, _ in UNATT_FIELDS], 0)
    rc = lib().oracle_encode(C.byref(ein), C.byref(eo), C.c_float(bz))
    if rc != 0:
        raise RuntimeError(f"oracle_encode failed with code {rc}")
    for name, _ in TRACK_FIELDS:
        out[name] = out[name][:eo.n_tracks].copy()
    for name, _ in CLUSTER_FIELDS:
        out[name] = out[name][:eo.n_attached].copy()
    for name, _ in UNATT_FIELDS:
        out[name] = out[name][:eo.n_unattached].copy()
    return out, int(eo.n_splits)


TABLE_NAMES = ["x", "pw", "inv_pw", "padoff", "pwq", "ks", "kt"]


def tables(bz=0.5):
    """The oracle's float32 constant tables, by name."""
    buf = (C.c_float * 2048)()
    n = lib().oracle_tables(C.c_float(bz), buf, 2048)
    v = np.frombuffer(buf, np.float32, n).copy()
    out, o = {}, 0
    for name in TABLE_NAMES:
        out[name] = v[o:o + NROW]; o += NROW
    out["cosb"] = v[o:o + 18]; o += 18
    out["sinb"] = v[o:o + 18]; o += 18
    out["kb"], out["vdq"], out["inv_vd32"], out["snp_max"] = v[o:o + 4]
    return out


def npads():
    buf = (C.c_int * NROW)()
    lib().oracle_npads(buf)
    return np.array(buf[:], np.int32)


def sat(v):
    """The decoder's float -> int32 conversion of an already rounded value."""
    return int(lib().oracle_sat(C.c_float(v)))


def clamp_snp(v):
    """The decoder's sin(phi) limiter: (value, flag bits it raises)."""
    fl = C.c_uint32(0)
    r = lib().oracle_clamp_snp(C.c_float(v), C.byref(fl))
    return np.float32(r), int(fl.value)


def fp_canary(a, b, c):
    return np.float32(lib().oracle_fp_canary(C.c_float(a), C.c_float(b), C.c_float(c)))


# the 19 arrays of a frame in coded order (rans_oracle.c), with their types
RANS_ARRAYS = TRACK_FIELDS + CLUSTER_FIELDS + [("un_count", np.uint32)] + UNATT_FIELDS


def rans_encode(frame):
    """Entropy-code the 19 arrays of a frame (rans_oracle.c's format).
    Returns the coded bytes (numpy uint8)."""
    nt, na, nu = frame_sizes(frame)
    arrs = [np.ascontiguousarray(frame[k], dt) for k, dt in RANS_ARRAYS]
    ptrs = (P * len(arrs))(*[a.ctypes.data_as(P) for a in arrs])
    cap = int(lib().oracle_rans_bound(nt, na, nu))
    dst = np.zeros(cap, np.uint8)
    n = int(lib().oracle_rans_encode(ptrs, nt, na, nu, dst.ctypes.data_as(P), cap))
    if n == 0:
        raise RuntimeError("oracle_rans_encode: buffer too small")
    return dst[:n].copy()


def rans_decode(blob, shape):
    """Decode coded bytes of a frame of shape (n_tracks, n_attached,
    n_unattached) back into its 19 arrays."""
    nt, na, nu = shape
    cnt = {"trk": nt, "cls": na, "un": nu}
    out = {}
    for k, dt in RANS_ARRAYS:
        out[k] = np.zeros(NBIN if k == "un_count" else cnt[k.split("_")[0]], dt)
    ptrs = (P * len(RANS_ARRAYS))(*[out[k].ctypes.data_as(P) for k, _ in RANS_ARRAYS])
    blob = np.ascontiguousarray(blob, np.uint8)
    rc = lib().oracle_rans_decode(blob.ctypes.data_as(P), blob.size, nt, na, nu, ptrs)
    if rc != 0:
        raise ValueError("oracle_rans_decode: not a coded frame of this shape")
    return out

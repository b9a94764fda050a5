"""ctypes binding of libtmd.so (C ABI declared in include/tmd.h).

Argument marshalling only: every step of the decode runs in the library's HIP
kernels.  If libtmd.so is missing the import fails; there is no fallback.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtmd.so")

NSEC, NROW = 36, 152
NBIN = NSEC * NROW
MAX_TRACKS = 1 << 24

OK, E_ARG, E_CAPACITY, E_INPUT, E_STREAM, E_HIP, E_SCRATCH = 0, -1, -2, -3, -4, -5, -6
STATIC_SCRATCH_BYTES = 512 << 20
F_HDR, F_SEC, F_ROW, F_ROT, F_SNP, F_PAD, F_TIME, F_COUNT, F_CODED = 1, 2, 4, 8, 16, 32, 64, 128, 256
PLAN_GRAPH = 1
PIPE_MAX_DEPTH = 8

P = C.c_void_p

IN_FIELDS = ["trk_ncls", "trk_sec0", "trk_row0", "trk_pad0", "trk_time0", "trk_qpt", "trk_snp",
             "trk_tgl", "cls_row_diff", "cls_sec_diff", "cls_pad_res", "cls_time_res", "cls_qtot",
             "cls_qmax", "un_count", "un_time_diff", "un_pad_diff", "un_qtot", "un_qmax"]
OUT_FIELDS = ["row_offset", "row_nattached", "time", "pad", "qtot", "qmax"]


class FrameShape(C.Structure):
    _fields_ = [("n_tracks", C.c_uint32), ("n_attached", C.c_uint32), ("n_unattached", C.c_uint32)]


class FrameIn(C.Structure):
    _fields_ = [(n, P) for n in IN_FIELDS]


class FrameOut(C.Structure):
    _fields_ = [(n, P) for n in OUT_FIELDS] + [("capacity", C.c_uint64)]


ENC_IN_TRACK = ["trk_first", "trk_qpt", "trk_tgl"]
ENC_IN_CLUSTER = ["cl_sec", "cl_row", "cl_pad", "cl_time", "cl_snp", "cl_qtot", "cl_qmax"]
ENC_IN_UNATT = ["un_sec", "un_row", "un_pad", "un_time", "un_qtot", "un_qmax"]


class EncIn(C.Structure):
    _fields_ = [("n_tracks", C.c_uint32), ("n_clusters", C.c_uint32), ("n_unattached", C.c_uint32)] + \
        [(n, P) for n in ENC_IN_TRACK + ENC_IN_CLUSTER + ENC_IN_UNATT]


class EncOut(C.Structure):
    _fields_ = [(n, P) for n in IN_FIELDS] + [("counts", P)]


class Params(C.Structure):
    _fields_ = [("bz_tesla", C.c_float), ("flags", C.c_uint32)]


_LIB = None


def lib():
    """The loaded libtmd.so.  Raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -c \"import __graft_entry__ as g; "
                              "g.build()\"` from the repository root")
        L = C.CDLL(LIB_PATH)
        L.tmd_plan.argtypes = [C.POINTER(FrameShape), C.c_uint32, C.POINTER(Params), C.POINTER(P),
                               C.POINTER(C.c_size_t)]
        L.tmd_plan.restype = C.c_int
        L.tmd_decode.argtypes = [P, C.POINTER(FrameIn), C.POINTER(FrameOut), P, P]
        L.tmd_decode.restype = C.c_int
        L.tmd_decode_shapes.argtypes = [P, C.POINTER(FrameShape), C.POINTER(FrameIn), C.POINTER(FrameOut), P, P]
        L.tmd_decode_shapes.restype = C.c_int
        L.tmd_decode_static.argtypes = [P, C.POINTER(FrameShape), C.POINTER(FrameIn), C.POINTER(FrameOut), P]
        L.tmd_decode_static.restype = C.c_int
        L.tmd_status.argtypes = [P, C.c_uint32, C.POINTER(C.c_uint32)]
        L.tmd_status.restype = C.c_int
        L.tmd_free.argtypes = [P]
        L.tmd_free.restype = None
        L.tmd_strerror.argtypes = [C.c_int]
        L.tmd_strerror.restype = C.c_char_p
        L.tmd_version.argtypes = []
        L.tmd_version.restype = C.c_char_p
        L.tmd_tables.argtypes = [C.c_float, C.POINTER(C.c_float), C.c_int]
        L.tmd_tables.restype = C.c_int
        L.tmd_set_schedule.argtypes = [P, C.c_uint32, C.c_uint32]
        L.tmd_set_schedule.restype = C.c_int
        L.tmd_set_profiling.argtypes = [P, C.c_uint32]
        L.tmd_set_profiling.restype = C.c_int
        L.tmd_stage_times.argtypes = [P, C.POINTER(C.c_double), C.c_uint32, C.POINTER(C.c_uint32)]
        L.tmd_stage_times.restype = C.c_int
        L.tmd_stage_name.argtypes = [C.c_uint32]
        L.tmd_stage_name.restype = C.c_char_p
        L.tmd_selftest_fp.argtypes = [P, P, P, C.c_uint32, P]
        L.tmd_selftest_fp.restype = C.c_int
        L.tmd_selftest_math.argtypes = [P, P, C.c_uint32, P]
        L.tmd_selftest_math.restype = C.c_int
        L.tmd_selftest_sqrt.argtypes = [C.c_uint32, C.c_uint32, P, P]
        L.tmd_selftest_sqrt.restype = C.c_int
        L.tmd_encode_workspace.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_size_t)]
        L.tmd_encode_workspace.restype = C.c_int
        L.tmd_encode.argtypes = [P, C.POINTER(EncIn), C.POINTER(EncOut), P, C.c_size_t, P]
        L.tmd_encode.restype = C.c_int
        L.tmd_rans_workspace.argtypes = [C.POINTER(FrameShape), C.c_uint32, C.POINTER(C.c_size_t)]
        L.tmd_rans_workspace.restype = C.c_int
        L.tmd_decode_rans.argtypes = [P, C.POINTER(FrameShape), C.POINTER(P), C.POINTER(C.c_uint64),
                                      C.POINTER(FrameOut), P, P, P]
        L.tmd_decode_rans.restype = C.c_int
        L.tmd_rans_encode_workspace.argtypes = [C.POINTER(FrameShape), C.POINTER(C.c_size_t),
                                                C.POINTER(C.c_uint64)]
        L.tmd_rans_encode_workspace.restype = C.c_int
        L.tmd_encode_rans.argtypes = [C.POINTER(FrameShape), C.POINTER(FrameIn), P, C.c_uint64, P, P, P]
        L.tmd_encode_rans.restype = C.c_int
        L.tmd_pipe_create.argtypes = [C.POINTER(FrameShape), C.c_uint32, C.POINTER(Params), C.POINTER(P)]
        L.tmd_pipe_create.restype = C.c_int
        L.tmd_pipe_run.argtypes = [P, C.c_uint32, C.POINTER(FrameShape), C.POINTER(FrameIn), C.POINTER(FrameOut),
                                   C.POINTER(C.c_uint32)]
        L.tmd_pipe_run.restype = C.c_int
        L.tmd_pipe_run_rans.argtypes = [P, C.c_uint32, C.POINTER(FrameShape), C.POINTER(P), C.POINTER(C.c_uint64),
                                        C.POINTER(FrameOut), C.POINTER(C.c_uint32)]
        L.tmd_pipe_run_rans.restype = C.c_int
        L.tmd_pipe_free.argtypes = [P]
        L.tmd_pipe_free.restype = None
        _LIB = L
    return _LIB


class TmdError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {lib().tmd_strerror(code).decode()} ({code})")


def check(code, what):
    if code != OK:
        raise TmdError(code, what)
    return code

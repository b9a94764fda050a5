"""libtmd.so on the host (no GPU needed): it loads, exports every entry point
include/tmd.h declares, computes the same constant tables as the oracle (two
independent implementations), and rejects bad arguments before touching the
device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_2411_02206_amd as tmd
from paper_2411_02206_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "tmd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tmd_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = C.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_tables_match_oracle_bitwise():
    for bz in (0.5, -0.5, 0.2, 2.0, 0.0):
        a, b = tmd.tables(bz), oracle.tables(bz)
        for k in b:
            assert np.array_equal(np.asarray(a[k]).view(np.uint32), np.asarray(b[k]).view(np.uint32)), (bz, k)


def test_strerror_and_version():
    L = _lib.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.tmd_strerror(code)
    assert L.tmd_strerror(-99) == b"unknown error"
    assert tmd.version().startswith("tmd")


def test_bad_arguments_rejected_on_host():
    L = _lib.lib()
    h = C.c_void_p()
    ws = C.c_size_t()
    p = _lib.Params(0.5, 0)
    shape = (_lib.FrameShape * 1)(_lib.FrameShape(10, 100, 100))
    assert L.tmd_plan(None, 1, C.byref(p), C.byref(h), C.byref(ws)) == _lib.E_ARG
    assert L.tmd_plan(shape, 0, C.byref(p), C.byref(h), C.byref(ws)) == _lib.E_ARG
    big = (_lib.FrameShape * 1)(_lib.FrameShape(_lib.MAX_TRACKS + 1, 0, 0))
    assert L.tmd_plan(big, 1, C.byref(p), C.byref(h), C.byref(ws)) == _lib.E_ARG
    assert L.tmd_decode(None, None, None, None, None) == _lib.E_ARG
    st = C.c_uint32()
    assert L.tmd_status(None, 0, C.byref(st)) == _lib.E_ARG
    assert L.tmd_selftest_fp(None, None, None, 4, None) == _lib.E_ARG
    assert L.tmd_selftest_math(None, None, 4, None) == _lib.E_ARG
    assert L.tmd_selftest_sqrt(0, 1, None, None) == _lib.E_ARG
    assert L.tmd_selftest_sqrt(5, 4, C.c_void_p(1), None) == _lib.E_ARG
    L.tmd_free(None)  # no-op
    # host pipeline: argument checks that come before any device call
    q = C.c_void_p()
    assert L.tmd_pipe_create(None, 2, C.byref(p), C.byref(q)) == _lib.E_ARG
    assert L.tmd_pipe_create(shape, 0, C.byref(p), C.byref(q)) == _lib.E_ARG
    assert L.tmd_pipe_create(shape, _lib.PIPE_MAX_DEPTH + 1, C.byref(p), C.byref(q)) == _lib.E_ARG
    assert L.tmd_pipe_create(big, 2, C.byref(p), C.byref(q)) == _lib.E_ARG
    assert L.tmd_pipe_create(shape, 2, None, C.byref(q)) == _lib.E_ARG
    flags = (C.c_uint32 * 1)()
    assert L.tmd_pipe_run(None, 1, shape, None, None, flags) == _lib.E_ARG
    L.tmd_pipe_free(None)  # no-op


def test_table_size_query():
    L = _lib.lib()
    need = L.tmd_tables(C.c_float(0.5), None, 0)
    assert need == -(7 * 152 + 36 + 4)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_LIB", None)
    with pytest.raises(ImportError):
        _lib.lib()


def test_kernel_symbols_agree_between_host_and_device():
    """Every kernel is registered by the host code under the symbol its
    device code object defines (a parameter type that differs between the two
    compilations, such as an address-space-qualified pointer, would leave the
    launch without a kernel)."""
    data = open(_lib.LIB_PATH, "rb").read()
    names = {}
    for m in re.finditer(rb"_ZN12_GLOBAL__N_1(\d+)", data):
        # the kernel's name (its length comes first), then its template
        # arguments if any (I ... E, literals L ... E inside)
        st = m.end()
        name = data[st:st + int(m.group(1))]
        if not name.startswith(b"k_"):
            continue
        j = st + len(name)
        if data[j:j + 1] == b"I":
            depth, k = 0, j
            while True:
                c = data[k:k + 1]
                depth += 1 if c in (b"I", b"L") else (-1 if c == b"E" else 0)
                k += 1
                if depth == 0:
                    break
            name += data[j:k]
        full = re.match(rb"[A-Za-z0-9_]+", data[m.start():]).group(0)
        names.setdefault(name, set()).add(full)
    assert len(names) >= 15
    bad = {k: v for k, v in names.items() if len(v) != 1}
    assert not bad, bad

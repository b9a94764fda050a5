"""The oracle's rANS coder for compressed frames (test infrastructure), pinned
by what information theory and the format fix rather than by its own code:
  - decode(encode(x)) == x for every array of valid, garbage, empty and
    multi-chunk frames;
  - the layout, parsed here independently of the C code: header, plane
    offsets on 8-byte boundaries, a model of 2^12 per plane with every present
    symbol at least 1, chunk offsets;
  - the size: rANS with a 32-bit state spends the model's cross-entropy per
    symbol (at most one renormalisation byte of slack per stream) plus 4 state
    bytes per stream, and cannot beat the empirical entropy of the plane."""
import math

import numpy as np

import oracle
import synth

WIDTH = [1, 1, 1, 2, 4, 2, 2, 2, 1, 1, 2, 2, 2, 2, 4, 4, 2, 2, 2]
CHUNK = 64 * 512


def counts(shape):
    nt, na, nu = shape
    return [nt] * 8 + [na] * 6 + [36 * 152] + [nu] * 4


def garbage(seed, nt=300, na=40000, nu=70000):
    rng = np.random.default_rng(seed)
    fr = {}
    for k, dt in oracle.RANS_ARRAYS:
        n = {"trk": nt, "cls": na, "un": nu}[k.split("_")[0]] if k != "un_count" else 36 * 152
        info = np.iinfo(dt)
        fr[k] = rng.integers(info.min, int(info.max) + 1, n, dtype=np.int64).astype(dt)
    return fr


def frames():
    yield "tiny", synth.make_frame(synth.spec_for("tiny"))
    yield "frame", synth.make_frame(synth.spec_for("frame", collisions=2))
    yield "garbage", garbage(1)
    empty = {k: np.zeros(0 if k != "un_count" else 36 * 152, dt) for k, dt in oracle.RANS_ARRAYS}
    yield "empty", empty


def planes(blob, shape):
    """(n symbols, model f[256], [(stream start, stream end)] per chunk) of each plane, from the bytes."""
    assert bytes(blob[:4]) == b"TMDR"
    hdr = np.frombuffer(blob[4:24].tobytes(), np.uint32)
    assert list(hdr) == [1, *shape, 0]
    nplane = sum(WIDTH)
    assert nplane == 39  # 15 bytes per track, 10 per attached cluster, 4 per bin, 10 per unattached cluster
    offs = np.frombuffer(blob[64:64 + 8 * nplane].tobytes(), np.uint64)
    # the planes follow the offset table directly
    assert int(offs[0]) == (64 + 8 * nplane + 7) // 8 * 8
    res = []
    p = 0
    for a, n in enumerate(counts(shape)):
        for b in range(WIDTH[a]):
            pos = int(offs[p])
            assert pos % 8 == 0
            f = np.frombuffer(blob[pos:pos + 512].tobytes(), np.uint16).astype(np.int64)
            nch = (n + CHUNK - 1) // CHUNK
            table = np.frombuffer(blob[pos + 512:pos + 512 + 4 * 65 * nch].tobytes(), np.uint32).reshape(nch, 65) \
                if nch else np.zeros((0, 65), np.uint32)
            res.append((n, f, table, pos + 512 + 4 * 65 * nch))
            p += 1
    return res


def test_roundtrip():
    for name, fr in frames():
        shape = oracle.frame_sizes(fr)
        blob = oracle.rans_encode(fr)
        back = oracle.rans_decode(blob, shape)
        for k in fr:
            assert np.array_equal(fr[k], back[k]), (name, k)


def test_layout_and_model():
    for name, fr in frames():
        shape = oracle.frame_sizes(fr)
        blob = oracle.rans_encode(fr)
        p = 0
        for a, (k, dt) in enumerate(oracle.RANS_ARRAYS):
            raw = np.ascontiguousarray(fr[k], dt).view(np.uint8).reshape(-1, WIDTH[a])
            for b in range(WIDTH[a]):
                n, f, table, data0 = planes(blob, shape)[p]
                p += 1
                if n == 0:
                    continue
                assert f.sum() == 4096, (name, k, b)
                cnt = np.bincount(raw[:, b], minlength=256)
                assert np.array_equal(f > 0, cnt > 0), (name, k, b)
                # each frequency within a few units of its exact share (rare
                # symbols raised to 1 take their units from the frequent ones)
                assert np.all(np.abs(f - cnt * 4096 / n) <= 3), (name, k, b)
                assert np.all(np.diff(table, axis=1) >= 4), (name, k, b)   # every stream holds its state


def test_size_against_entropy():
    """Coded bytes per plane against the model's cross-entropy and the
    plane's empirical entropy."""
    rng = np.random.default_rng(7)
    n = 3 * CHUNK + 12345
    fr = garbage(2, nt=n, na=n, nu=n)
    fr["cls_pad_res"] = np.clip(np.rint(rng.normal(0, 3.0, n)), -30000, 30000).astype(np.int16)
    fr["cls_row_diff"] = (1 + (rng.random(n) < 0.05)).astype(np.int8)
    fr["un_qmax"] = np.minimum(1 + np.floor(rng.exponential(30.0, n)), 65535).astype(np.uint16)
    shape = oracle.frame_sizes(fr)
    blob = oracle.rans_encode(fr)
    p = 0
    for a, (k, dt) in enumerate(oracle.RANS_ARRAYS):
        raw = np.ascontiguousarray(fr[k], dt).view(np.uint8).reshape(-1, WIDTH[a])
        for b in range(WIDTH[a]):
            n_sym, f, table, data0 = planes(blob, shape)[p]
            p += 1
            nch = table.shape[0]
            if nch == 0:
                continue
            # streams are back to back: the plane's data ends at the last chunk's end offset
            size = int(table[-1, 64])
            cnt = np.bincount(raw[:, b], minlength=256)
            nz = cnt > 0
            cross = float(-(cnt[nz] * np.log2(f[nz] / 4096.0)).sum()) / 8
            emp = float(-(cnt[nz] * np.log2(cnt[nz] / n_sym)).sum()) / 8
            streams = 64 * nch
            assert size <= cross + 4 * streams + streams + 1, (k, b, size, cross)
            assert size >= emp - 1e-6 * n_sym, (k, b, size, emp)


def test_malformed_rejected():
    fr = synth.make_frame(synth.spec_for("tiny"))
    shape = oracle.frame_sizes(fr)
    blob = oracle.rans_encode(fr)
    bad = blob.copy()
    bad[0] = ord("X")
    for b, sh in ((bad, shape), (blob[:1000], shape), (blob, (shape[0] + 1, shape[1], shape[2]))):
        try:
            oracle.rans_decode(b, sh)
        except ValueError:
            continue
        raise AssertionError("a malformed coded frame was accepted")

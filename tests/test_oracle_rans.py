"""The oracle's rANS coder for compressed frames (test infrastructure), pinned
by what information theory and the format fix rather than by its own code:
  - decode(encode(x)) == x for every array of valid, garbage, empty and
    multi-chunk frames;
  - the layout, parsed here independently of the C code: header, plane
    offsets on 16-byte boundaries, a model of 2^12 per plane with every
    present symbol at least 1, chunk offsets, final states in [2^16, 2^32);
  - a decoder written here from the format's definition (numpy, one step of
    64 lanes at a time) reads the oracle's bytes back into the symbols;
  - the size: rANS with a 32-bit state and 16-bit words spends the model's
    cross-entropy per symbol plus at most one word of slack and the final
    state per lane, and cannot beat the empirical entropy of the plane."""
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


def align16(v):
    return (v + 15) // 16 * 16


def planes(blob, shape):
    """(n symbols, model f[256], chunk offsets (nch + 1), start of the data) of each plane, from the bytes."""
    assert bytes(blob[:4]) == b"TMDR"
    hdr = np.frombuffer(blob[4:24].tobytes(), np.uint32)
    assert list(hdr) == [2, *shape, 0]
    nplane = sum(WIDTH)
    assert nplane == 39  # 15 bytes per track, 10 per attached cluster, 4 per bin, 10 per unattached cluster
    offs = np.frombuffer(blob[64:64 + 8 * nplane].tobytes(), np.uint64)
    # the planes follow the offset table directly
    assert int(offs[0]) == align16(64 + 8 * nplane)
    res = []
    p = 0
    for a, n in enumerate(counts(shape)):
        for b in range(WIDTH[a]):
            pos = int(offs[p])
            assert pos % 16 == 0
            f = np.frombuffer(blob[pos:pos + 512].tobytes(), np.uint16).astype(np.int64)
            nch = (n + CHUNK - 1) // CHUNK
            table = np.frombuffer(blob[pos + 512:pos + 512 + 4 * (nch + 1)].tobytes(), np.uint32).astype(np.int64)
            res.append((n, f, table, align16(pos + 512 + 4 * (nch + 1))))
            p += 1
    return res


def decode_plane(blob, n, f, table, data0):
    """A plane's symbols, decoded from the format's definition: per chunk,
    the 64 lanes' states, then step by step the lanes that have a symbol
    decode it and those whose state fell below 2^16 take the next words of
    the shared stream in lane order."""
    c = np.concatenate([[0], np.cumsum(f)[:-1]])
    sym_of_slot = np.repeat(np.arange(256), f)
    out = np.zeros(n, np.uint8)
    for ch in range(len(table) - 1):
        d0, d1 = data0 + int(table[ch]), data0 + int(table[ch + 1])
        x = np.frombuffer(blob[d0:d0 + 256].tobytes(), np.uint32).astype(np.int64)
        words = np.frombuffer(blob[d0 + 256:d1].tobytes(), np.uint16).astype(np.int64)
        c0 = ch * CHUNK
        length = min(CHUNK, n - c0)
        k = 0
        for j in range((length + 63) // 64):
            live = np.arange(64) + 64 * j < length
            slot = x & 4095
            s = sym_of_slot[slot]
            x = np.where(live, f[s] * (x >> 12) + slot - c[s], x)
            need = live & (x < 65536)
            idx = k + np.cumsum(need) - 1
            x = np.where(need, (x << 16) | np.append(words, 0)[np.where(need, idx, len(words))], x)
            k += int(need.sum())
            out[c0 + 64 * j: c0 + 64 * j + int(live.sum())] = s[live]
        assert np.all(x == 65536)
        assert 0 <= (d1 - d0 - 256 - 2 * k) < 16
    return out


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
                # chunks on 16-byte boundaries, each holding its 64 states
                assert np.all(table % 16 == 0) and np.all(np.diff(table) >= 256), (name, k, b)
                for ch in range(len(table) - 1):
                    st = np.frombuffer(blob[data0 + table[ch]:data0 + table[ch] + 256].tobytes(), np.uint32)
                    assert np.all(st >= 65536), (name, k, b)


def test_decoder_from_the_definition():
    """The oracle's bytes, read by the decoder above, give back every plane
    of a frame whose planes span several chunks and a ragged last one."""
    rng = np.random.default_rng(3)
    n = 2 * CHUNK + 777
    fr = garbage(4, nt=100, na=n, nu=500)
    fr["cls_pad_res"] = np.clip(np.rint(rng.normal(0, 3.0, n)), -30000, 30000).astype(np.int16)
    fr["cls_row_diff"] = (1 + (rng.random(n) < 0.05)).astype(np.int8)
    fr["cls_qmax"][:] = 7  # a plane of one symbol (f = 2^12) and one of a single rare pattern
    shape = oracle.frame_sizes(fr)
    blob = oracle.rans_encode(fr)
    p = 0
    for a, (k, dt) in enumerate(oracle.RANS_ARRAYS):
        raw = np.ascontiguousarray(fr[k], dt).view(np.uint8).reshape(-1, WIDTH[a])
        for b in range(WIDTH[a]):
            n_sym, f, table, data0 = planes(blob, shape)[p]
            p += 1
            assert np.array_equal(decode_plane(blob, n_sym, f, table, data0), raw[:, b]), (k, b)


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
            nch = len(table) - 1
            if nch == 0:
                continue
            size = int(table[-1])  # states, words and padding of all chunks
            cnt = np.bincount(raw[:, b], minlength=256)
            nz = cnt > 0
            cross = float(-(cnt[nz] * np.log2(f[nz] / 4096.0)).sum()) / 8
            emp = float(-(cnt[nz] * np.log2(cnt[nz] / n_sym)).sum()) / 8
            lanes = 64 * nch
            # per lane: the final state (4 bytes) and at most one word of slack; per chunk: padding
            assert size <= cross + 6 * lanes + 16 * nch, (k, b, size, cross)
            assert size >= emp, (k, b, size, emp)


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

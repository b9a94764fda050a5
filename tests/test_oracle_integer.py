"""Pins of the oracle's integer bookkeeping against library routines.

- unattached decode (section 4: each coordinate is the stored difference added
  to the last decoded cluster of the region) == numpy cumsum per (sector,row)
  segment, wrapping at 2^32 (time) and 2^16 (pad);
- row offsets == bincount + cumsum of the per-bin counts;
- order inside a bin == stable argsort of the cluster bins (attached clusters
  first, in stream order), checked with unique per-cluster tags;
- streams whose counts do not add up are cut at the declared sizes (F_COUNT).
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import NBIN, build_frame, empty_frame


def _bins_by_walk(fr):
    """(sector,row) of every attached cluster via numpy cumsums (valid streams:
    no clamping), independent of the decoder's walk."""
    n = fr["trk_ncls"].astype(np.int64)
    tid = np.repeat(np.arange(len(n)), n)
    st = np.concatenate([[0], np.cumsum(n)])
    first = np.zeros(len(tid), bool)
    first[st[:-1][n > 0]] = True
    rd = fr["cls_row_diff"].astype(np.int64).copy()
    sd = fr["cls_sec_diff"].astype(np.int64).copy()
    rd[first] = 0
    sd[first] = 0
    crd = np.cumsum(rd)
    csd = np.cumsum(sd)
    base = st[:-1][tid]
    row = fr["trk_row0"].astype(np.int64)[tid] + crd - crd[base]
    s0 = fr["trk_sec0"].astype(np.int64)[tid]
    sec = (s0 // 18) * 18 + (s0 % 18 + csd - csd[base]) % 18
    assert row.min() >= 0 and row.max() < 152
    return sec * 152 + row


@pytest.fixture(scope="module")
def frame():
    fr = synth.make_frame(synth.spec_for("frame", collisions=3))
    n = len(fr["cls_qtot"])
    fr["cls_qtot"] = (np.arange(n) & 0xFFFF).astype(np.uint16)   # unique tags
    fr["cls_qmax"] = (np.arange(n) >> 16).astype(np.uint16)
    return fr


def test_unattached_is_cumsum(frame):
    out, st = oracle.decode(frame)
    cnt = frame["un_count"].astype(np.int64)
    seg = np.repeat(np.arange(NBIN), cnt)
    ustart = np.concatenate([[0], np.cumsum(cnt)])
    t = frame["un_time_diff"].astype(np.uint64)
    p = frame["un_pad_diff"].astype(np.uint64)
    ct = np.cumsum(t)
    cp = np.cumsum(p)
    # subtract the running total before each segment: inclusive sums restart
    before_t = np.concatenate([np.zeros(1, np.uint64), ct])[ustart[:-1]][seg]
    before_p = np.concatenate([np.zeros(1, np.uint64), cp])[ustart[:-1]][seg]
    exp_t = ((ct - before_t) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    exp_p = ((cp - before_p) & np.uint64(0xFFFF)).astype(np.uint16)
    off = out["row_offset"].astype(np.int64)
    na = out["row_nattached"].astype(np.int64)
    pos = off[seg] + na[seg] + (np.arange(len(seg)) - ustart[seg])
    assert np.array_equal(out["time"][pos], exp_t)
    assert np.array_equal(out["pad"][pos], exp_p)
    assert np.array_equal(out["qtot"][pos], frame["un_qtot"])
    assert np.array_equal(out["qmax"][pos], frame["un_qmax"])


def test_offsets_and_order(frame):
    out, st = oracle.decode(frame)
    bins = _bins_by_walk(frame)
    na = np.bincount(bins, minlength=NBIN)
    nu = frame["un_count"].astype(np.int64)
    assert np.array_equal(out["row_nattached"], na)
    off = np.concatenate([[0], np.cumsum(na + nu)])
    assert np.array_equal(out["row_offset"], off)
    order = np.argsort(bins, kind="stable")
    rank = np.arange(len(bins)) - np.searchsorted(bins[order], bins[order], side="left")
    pos = off[bins[order]] + rank
    tag = out["qtot"][pos].astype(np.int64) | (out["qmax"][pos].astype(np.int64) << 16)
    assert np.array_equal(tag, order)


def test_empty_frame():
    out, st = oracle.decode(empty_frame())
    assert st == 0
    assert not out["row_offset"].any() and len(out["time"]) == 0


def test_count_mismatch_is_cut_and_flagged():
    tr = [dict(sec0=1, row0=10, pad0=500, time0=1000, qpt=0, snp=0, tgl=0,
               cl=[(0, 0, 0, 0, 5, 6)] + [(1, 0, 0, 0, 7 + j, 8) for j in range(4)])]
    fr = build_frame(tr, {3: [(5, 1, 2, 3), (1, 1, 4, 4)]})
    out, st = oracle.decode(fr)
    assert st == 0 and out["row_offset"][-1] == 7
    # declared attached count shorter than the track: the track is cut
    fr2 = dict(fr)
    for k in ("cls_row_diff", "cls_sec_diff", "cls_pad_res", "cls_time_res", "cls_qtot", "cls_qmax"):
        fr2[k] = fr[k][:3]
    out2, st2 = oracle.decode(fr2)
    assert st2 & oracle.F_COUNT
    assert out2["row_nattached"].sum() == 3
    # unattached counts larger than the stream: the last bin is cut
    fr3 = dict(fr)
    fr3["un_count"] = fr["un_count"].copy()
    fr3["un_count"][3] = 5
    out3, st3 = oracle.decode(fr3)
    assert st3 & oracle.F_COUNT and out3["row_offset"][-1] == 7
    # track counts that do not reach the declared size: trailing clusters ignored
    fr4 = dict(fr)
    fr4["trk_ncls"] = np.array([2], np.uint8)
    out4, st4 = oracle.decode(fr4)
    assert st4 & oracle.F_COUNT and out4["row_nattached"].sum() == 2


def test_garbage_is_deterministic_and_flagged():
    rng = np.random.default_rng(5)
    nt, na = 50, 3000
    fr = {
        "trk_ncls": rng.integers(0, 256, nt).astype(np.uint8),
        "trk_sec0": rng.integers(0, 256, nt).astype(np.uint8),
        "trk_row0": rng.integers(0, 256, nt).astype(np.uint8),
        "trk_pad0": rng.integers(0, 65536, nt).astype(np.uint16),
        "trk_time0": rng.integers(0, 2**32, nt, dtype=np.uint64).astype(np.uint32),
        "trk_qpt": rng.integers(-32768, 32768, nt).astype(np.int16),
        "trk_snp": rng.integers(-32768, 32768, nt).astype(np.int16),
        "trk_tgl": rng.integers(-32768, 32768, nt).astype(np.int16),
        "cls_row_diff": rng.integers(-128, 128, na).astype(np.int8),
        "cls_sec_diff": rng.integers(0, 256, na).astype(np.uint8),
        "cls_pad_res": rng.integers(-32768, 32768, na).astype(np.int16),
        "cls_time_res": rng.integers(-32768, 32768, na).astype(np.int16),
        "cls_qtot": rng.integers(0, 65536, na).astype(np.uint16),
        "cls_qmax": rng.integers(0, 65536, na).astype(np.uint16),
        "un_count": rng.integers(0, 3, NBIN).astype(np.uint32),
    }
    nu = 9000
    fr["un_time_diff"] = rng.integers(0, 2**32, nu, dtype=np.uint64).astype(np.uint32)
    fr["un_pad_diff"] = rng.integers(0, 65536, nu).astype(np.uint16)
    fr["un_qtot"] = rng.integers(0, 65536, nu).astype(np.uint16)
    fr["un_qmax"] = rng.integers(0, 65536, nu).astype(np.uint16)
    a, sa = oracle.decode(fr, bz=5.0)
    b, sb = oracle.decode(fr, bz=5.0)
    assert sa == sb
    for k in a:
        assert np.array_equal(a[k], b[k])
    for f in (oracle.F_HDR, oracle.F_SEC, oracle.F_ROW, oracle.F_ROT, oracle.F_SNP, oracle.F_PAD,
              oracle.F_TIME, oracle.F_COUNT):
        assert sa & f, f
    assert a["row_offset"][-1] <= na + nu

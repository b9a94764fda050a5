"""Brute force on tiny inputs: every combination of a few header values and of
row/sector steps (lengths <= 3, including out-of-range values) must place the
clusters in the (sector,row) bins a step-by-step walk with the documented
clamps gives: sector >= 36 wraps (flag F_HDR), row > 151 clamps to 151
(F_HDR), sector steps >= 18 wrap (F_SEC), rows clamp to [0, 151] (F_ROW)."""
import itertools

import numpy as np

import oracle
from helpers import build_frame

ROW0 = (0, 1, 150, 151, 152, 255)
SEC0 = (0, 17, 18, 35, 36, 255)
RD = (-128, -2, -1, 0, 1, 2, 127)
SD = (0, 1, 17, 18, 35, 255)


def walk(sec0, row0, steps):
    flags = 0
    if sec0 >= 36:
        flags |= oracle.F_HDR
        sec0 %= 36
    if row0 >= 152:
        flags |= oracle.F_HDR
        row0 = 151
    bins = [sec0 * 152 + row0]
    sec, row = sec0, row0
    for rd, sd in steps:
        if sd >= 18:
            flags |= oracle.F_SEC
            sd %= 18
        sec = (sec // 18) * 18 + (sec % 18 + sd) % 18
        row += rd
        if row < 0 or row > 151:
            flags |= oracle.F_ROW
            row = min(max(row, 0), 151)
        bins.append(sec * 152 + row)
    return bins, flags


def test_exhaustive_short_walks():
    tracks, expect = [], []
    for sec0, row0 in itertools.product(SEC0, ROW0):
        for n in (1, 2, 3):
            for steps in itertools.product(itertools.product(RD, SD), repeat=n - 1):
                if n == 3 and (steps[0][0] not in (-1, 0, 127) or steps[0][1] not in (0, 18)):
                    continue  # keep the length-3 set small but covering the edges
                cl = [(0, 0, 0, 0, len(tracks) & 0xFFFF, len(tracks) >> 16)]
                cl += [(rd, sd, 0, 0, len(tracks) & 0xFFFF, len(tracks) >> 16) for rd, sd in steps]
                tracks.append(dict(sec0=sec0, row0=row0, pad0=1000, time0=5000, qpt=0, snp=0,
                                   tgl=0, cl=cl))
                expect.append(walk(sec0, row0, steps))
    # decode in chunks; each track is tagged through qtot/qmax
    for a in range(0, len(tracks), 2000):
        chunk = tracks[a:a + 2000]
        fr = build_frame(chunk)
        out, st = oracle.decode(fr, bz=0.5)
        bins = np.repeat(np.arange(5472), np.diff(out["row_offset"]))
        tag = out["qtot"].astype(np.int64) | (out["qmax"].astype(np.int64) << 16)
        got = {}
        for b, t in zip(bins, tag):
            got.setdefault(int(t), []).append(int(b))
        want_flags = 0
        for i, tr in enumerate(chunk):
            eb, ef = expect[a + i]
            want_flags |= ef
            assert sorted(got[a + i]) == sorted(eb), (tr["sec0"], tr["row0"], tr["cl"])
        assert (st & (oracle.F_HDR | oracle.F_SEC | oracle.F_ROW)) == want_flags

"""Closed-form pins of the oracle's propagation, rotation, quantisation and
update (track model, arXiv:2411.02206 section 4: the decoder propagates each
track through the TPC and adds the stored residuals).

With all residuals zero the update is a no-op, so every decoded cluster must
lie where the circle (a straight line at Bz = 0) defined by the track header
crosses the pad row of the cluster's sector.  The expected positions come from
circle geometry in float64 (centre/radius intersection, global frame), not
from the decoder's recurrence.  Float32 rounding inside the decoder moves a
value by far less than 0.1 quantum, so decoded codes must equal the rounded
closed form unless that lies within 0.1 quantum of a rounding tie, where one
code either way is accepted."""
import math

import numpy as np
import pytest

import oracle
from oracle import physgen as pg
from helpers import build_frame, check_rounded, closed_form_track


def decode_single(hdr, steps, bz, res=None):
    """Decode one track; returns list of (bin, pad, time) in cluster order."""
    res = res or {}
    cl = [(0, 0, 0, 0, 1, 1)] + [(rd, sd, *res.get(j, (0, 0)), 1, 1)
                                 for j, (rd, sd) in enumerate(steps, start=1)]
    fr = build_frame([dict(hdr, cl=cl)])
    out, st = oracle.decode(fr, bz=bz)
    # walk the steps to find each cluster's bin (monotone rows: one per bin)
    sec, row = hdr["sec0"], hdr["row0"]
    bins = [sec * 152 + row]
    for rd, sd in steps:
        sec = (sec // 18) * 18 + (sec % 18 + sd) % 18
        row += rd
        bins.append(sec * 152 + row)
    assert len(set(bins)) == len(bins)
    vals = []
    for b in bins:
        i = out["row_offset"][b]
        assert out["row_offset"][b + 1] - i == 1
        vals.append((b, int(out["pad"][i]), int(out["time"][i])))
    return vals, st


def random_header(rng, sec, row0, span, pad_margin=8):
    npads = pg.ROW_NPADS[row0]
    return dict(sec0=sec, row0=row0,
                pad0=int(rng.integers(pad_margin * 32, (npads - pad_margin) * 32)),
                time0=int(rng.integers(20000, 60000)), qpt=int(rng.integers(-1000, 1000)),
                snp=int(rng.integers(-3000, 3000)), tgl=int(rng.integers(-4096, 4097)))


@pytest.mark.parametrize("seed", range(6))
def test_straight_line_bz0(seed):
    """Bz = 0: y = y0 + dx tan(phi), z = tan(lambda) dx / cos(phi)."""
    rng = np.random.default_rng(seed)
    n_checked = 0
    for _ in range(40):
        row0 = int(rng.integers(0, 60))
        n = int(rng.integers(2, 152 - row0))
        hdr = random_header(rng, int(rng.integers(0, 36)), row0, n)
        steps = [(1, 0)] * (n - 1)
        got, st = decode_single(hdr, steps, 0.0)
        s0 = hdr["snp"] / 32768.0
        X0 = pg.ROW_X[row0]
        y0 = (hdr["pad0"] / 32 - pg.ROW_NPADS[row0] / 2) * pg.ROW_PW[row0]
        for j, (b, pad, time) in enumerate(got):
            r = row0 + j
            dx = pg.ROW_X[r] - X0
            y = y0 + dx * s0 / math.sqrt(1 - s0 * s0)
            zt = hdr["tgl"] / 4096.0 * dx / math.sqrt(1 - s0 * s0)
            if not (0 <= (y / pg.ROW_PW[r] + pg.ROW_NPADS[r] / 2) * 32 < 65535):
                continue
            assert check_rounded(pad, (y / pg.ROW_PW[r] + pg.ROW_NPADS[r] / 2) * 32), (j, pad, y)
            assert check_rounded(time, hdr["time0"] + zt * 32 / 0.516), (j, time)
            n_checked += 1
    assert n_checked > 1000


def _helix_case(rng, bz, allow_cross):
    """A zero-noise physical track (rows and sectors from exact geometry)."""
    while True:
        pt = math.exp(rng.uniform(math.log(0.2), math.log(10)))
        t = pg.make_track(rng, bz, pt, 1.0 if rng.random() < 0.5 else -1.0, rng.uniform(-1, 1),
                          rng.uniform(0, 2 * math.pi), int(rng.integers(0, 2)),
                          int(rng.integers(0, 30)), 152, noise=0.0, allow_cross=allow_cross)
        r0 = t["row"][0] if t["row"] else 0
        if len(t["row"]) >= 10 and 0 <= t["y"][0] / pg.ROW_PW[r0] + pg.ROW_NPADS[r0] / 2 < 2000:
            break
    hdr = dict(sec0=t["sec"][0], row0=r0,
               pad0=int(np.rint((t["y"][0] / pg.ROW_PW[r0] + pg.ROW_NPADS[r0] / 2) * 32)),
               time0=40000, qpt=int(np.clip(np.rint((1.0 / pt) * 1024), -32767, 32767)),
               snp=int(np.rint(t["snp"][0] * 32768)), tgl=int(rng.integers(-4096, 4097)))
    if rng.random() < 0.5:
        hdr["qpt"] = -hdr["qpt"]
    steps = []
    for j in range(1, len(t["row"])):
        steps.append((t["row"][j] - t["row"][j - 1], (t["sec"][j] % 18 - t["sec"][j - 1] % 18) % 18))
    return hdr, steps


def _free_case(rng, bz, min_len=10):
    """A track from an arbitrary start (not the origin) near a sector edge;
    its rows and sectors follow the header's own circle (or line)."""
    while True:
        sec0 = int(rng.integers(0, 36))
        row0 = int(rng.integers(0, 60))
        npads = pg.ROW_NPADS[row0]
        edge_side = 1 if rng.random() < 0.5 else -1
        pad0 = int(rng.integers(2 * 32, 12 * 32)) if edge_side < 0 else \
            int(rng.integers((npads - 12) * 32, (npads - 2) * 32))
        hdr = dict(sec0=sec0, row0=row0, pad0=pad0, time0=40000,
                   qpt=int(rng.integers(-4000, 4001)),
                   snp=int(edge_side * rng.integers(0, 16000)), tgl=int(rng.integers(-4096, 4097)))
        k = hdr["qpt"] / 1024.0 * bz * 0.00299792458
        sec, row = sec0, row0
        a = pg.sector_angle(sec)
        gx, gy = pg.to_global(pg.ROW_X[row0], (pad0 / 32 - npads / 2) * pg.ROW_PW[row0], a)
        phi = math.asin(hdr["snp"] / 32768.0) + a
        steps = []
        while row < 151 and len(steps) < 150:
            X = pg.ROW_X[row + 1]
            hit = pg.helix_to_line(gx, gy, phi, k, pg.sector_angle(sec), X)
            d = 0
            if hit is not None and abs(hit[0]) > X * pg.TAN10:
                d = 1 if hit[0] > 0 else 17
                nsec = (sec // 18) * 18 + (sec % 18 + d) % 18
                hit = pg.helix_to_line(gx, gy, phi, k, pg.sector_angle(nsec), X)
                sec = nsec
            if hit is None or abs(math.sin(hit[1])) > 0.95:
                break
            row += 1
            a = pg.sector_angle(sec)
            gx, gy = pg.to_global(X, hit[0], a)
            phi = hit[1] + a
            steps.append((1, d))
        if len(steps) + 1 >= min_len:
            return hdr, steps


def _compare(got, exp, kicks=None):
    kicks = kicks or {}
    n = 0
    for j, ((b, pad, time), (sec, row, pv, tv)) in enumerate(zip(got, exp)):
        assert b == sec * 152 + row
        pr, tr = kicks.get(j, (0, 0))
        if j == 0:
            assert pad == pv and time == tv
            continue
        if pv + pr < -0.4 or pv + pr > 65535.4:
            # off the pad plane: the decoder clamps the code (flag F_PAD)
            assert pad == (0 if pv + pr < 0 else 65535)
            continue
        assert check_rounded(pad - pr, pv), (j, pad, pv)
        assert check_rounded(time - tr, tv), (j, time, tv)
        n += 1
    return n


@pytest.mark.parametrize("bz", [0.0, 0.5, -0.5, 2.0])
def test_circle_with_crossings(bz):
    """Zero residuals: decoded clusters lie on the header's circle, through
    sector crossings (frame rotations)."""
    rng = np.random.default_rng(int(abs(bz) * 10) + (bz < 0))
    n = crossings = 0
    for i in range(80):
        hdr, steps = _helix_case(rng, bz, True) if i % 2 else _free_case(rng, bz)
        exp = closed_form_track(hdr, steps, bz)
        if exp is None:
            continue
        got, st = decode_single(hdr, steps, bz)
        n += _compare(got, exp)
        crossings += sum(1 for s in steps if s[1])
    assert n > 2000
    assert crossings > 10


@pytest.mark.parametrize("seed", range(4))
def test_update_kicks(seed):
    """Nonzero residuals at a few clusters: after each, the decoded track
    follows the circle through the shifted point with the tilted direction."""
    rng = np.random.default_rng(100 + seed)
    n = 0
    for _ in range(30):
        hdr, steps = _helix_case(rng, 0.5, True)
        m = len(steps)
        kicks = {int(j): (int(rng.integers(-60, 61)), int(rng.integers(-60, 61)))
                 for j in rng.choice(np.arange(1, m + 1), size=min(3, m), replace=False)}
        exp = closed_form_track(hdr, steps, 0.5, kicks=kicks)
        if exp is None:
            continue
        got, st = decode_single(hdr, steps, 0.5, res=kicks)
        n += _compare(got, exp, kicks)
    assert n > 1000


def test_wrong_update_sign_is_caught():
    """Sensitivity of the pin: the same closed form with the update's tilt
    reversed disagrees with the decoder, so a sign error would be caught."""
    rng = np.random.default_rng(7)
    hdr, steps = _helix_case(rng, 0.5, False)
    while len(steps) < 60:
        hdr, steps = _helix_case(rng, 0.5, False)
    kicks = {3: (400, 0)}
    got, _ = decode_single(hdr, steps, 0.5, res=kicks)
    assert _compare(got, closed_form_track(hdr, steps, 0.5, kicks=kicks), kicks) > 50
    wrong = closed_form_track(hdr, steps, 0.5, kicks=kicks, tilt_sign=-1.0)
    mism = sum(1 for (b, p, t), (_, _, pv, _) in zip(got[4:], wrong[4:]) if abs(p - pv) > 2)
    assert mism > 10

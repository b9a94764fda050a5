"""Closed-form pins of the oracle's clamp-and-flag branches.

The paper (section 4) only says that decoding restores the stored values; for
streams the model cannot follow, this project defines clamp-and-flag semantics
so that every output byte is still defined (|sin phi| limited to SNP_MAX with
NaN -> 0, decoded pads clamped to [0, 65535], times to [0, 2^24 - 1], the
float->int conversion saturating at +-2^30 with NaN -> 0, a flag bit for each).

Each test below builds a track whose decoded values follow from geometry once
the clamp is applied, computed in float64 here without the decoder's
recurrence:
  - a clamped direction makes the track a straight line of slope
    SNP_MAX / sqrt(1 - SNP_MAX^2) (zero residuals, so no update moves it);
  - a NaN curvature makes every propagated sin(phi) 0: a line along x;
  - one circle step between two directions phi0 -> phi1 over dx moves y by
    dx * tan((phi0 + phi1) / 2) (the half-angle identity of a circular arc);
  - a rotation by beta maps (x, y, phi) to (x cos b + y sin b,
    y cos b - x sin b, phi - beta), after which the model follows the forward
    direction whose sine is sin(phi - beta).
Codes must equal the rounded closed form unless that lies within 0.1 quantum
of a rounding tie (then one code either way), as in the other closed-form pins.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import physgen as pg
from helpers import build_frame, check_rounded, closed_form_track

SMAX = float(np.float32(0.999))            # the limit as the decoder holds it
SLOPE = SMAX / math.sqrt(1.0 - SMAX * SMAX)
TLIM = (1 << 24) - 1
VD = 0.516


def decode_track(hdr, steps, bz, res=None):
    """Decode one track (cluster j in its own bin); returns [(bin, pad, time)]
    in cluster order and the status word."""
    res = res or {}
    cl = [(0, 0, 0, 0, 1, 1)] + [(rd, sd, *res.get(j, (0, 0)), 1, 1)
                                 for j, (rd, sd) in enumerate(steps, start=1)]
    out, st = oracle.decode(build_frame([dict(hdr, cl=cl)]), bz=bz)
    sec, row = hdr["sec0"] % 36, min(hdr["row0"], 151)
    bins = [sec * 152 + row]
    for rd, sd in steps:
        sec = (sec // 18) * 18 + (sec % 18 + sd) % 18
        row += rd
        bins.append(sec * 152 + row)
    assert len(set(bins)) == len(bins)
    vals = []
    for b in bins:
        i = int(out["row_offset"][b])
        assert int(out["row_offset"][b + 1]) - i == 1
        vals.append((b, int(out["pad"][i]), int(out["time"][i])))
    return vals, st


def pad_code(y, row):
    return (y / pg.ROW_PW[row] + pg.ROW_NPADS[row] / 2) * 32.0


def y_of(pad0, row):
    return (pad0 / 32.0 - pg.ROW_NPADS[row] / 2) * pg.ROW_PW[row]


def center_pad(row):
    return int(pg.ROW_NPADS[row] // 2 * 32)


def clamp16(v):
    return min(max(v, 0.0), 65535.0)


def check(got, exact, lo=0.0, hi=65535.0):
    """Decoded code vs closed form; beyond [lo, hi] the clamp value."""
    if exact < lo - 0.5:
        return got == lo
    if exact > hi + 0.5:
        return got == hi
    return check_rounded(got, exact)


# ---------------------------------------------------------------------------
# the two helpers against their definitions (special values)
# ---------------------------------------------------------------------------
def test_sat_definition():
    f32 = lambda v: float(np.float32(v))
    cases = {float("nan"): 0, float("inf"): 1 << 30, float("-inf"): -(1 << 30),
             0.0: 0, -0.0: 0, 5.0: 5, -7.0: -7, 1234567.0: 1234567,
             f32(2.0 ** 30): 1 << 30, f32(-(2.0 ** 30)): -(1 << 30),
             float(np.nextafter(np.float32(2 ** 30), np.float32(0))): (1 << 30) - 64,
             float(np.nextafter(np.float32(2 ** 30), np.float32(np.inf))): 1 << 30,
             f32(2.0 ** 31): 1 << 30, f32(-(2.0 ** 31)): -(1 << 30), 3e9: 1 << 30, -3e9: -(1 << 30),
             1e38: 1 << 30, -1e38: -(1 << 30)}
    for v, want in cases.items():
        assert oracle.sat(v) == want, (v, oracle.sat(v), want)


def test_clamp_snp_definition():
    above = float(np.nextafter(np.float32(SMAX), np.float32(2)))
    below = float(np.nextafter(np.float32(SMAX), np.float32(0)))
    cases = [(float("nan"), 0.0, True), (float("inf"), SMAX, True), (float("-inf"), -SMAX, True),
             (1.0, SMAX, True), (-1.0, -SMAX, True), (0.9999, SMAX, True), (above, SMAX, True),
             (-above, -SMAX, True), (SMAX, SMAX, False), (-SMAX, -SMAX, False), (below, below, False),
             (0.5, 0.5, False), (0.0, 0.0, False), (-0.25, -0.25, False)]
    for v, want, flagged in cases:
        got, fl = oracle.clamp_snp(v)
        assert float(got) == float(np.float32(want)), (v, got, want)
        assert fl == (oracle.F_SNP if flagged else 0), (v, fl)


# ---------------------------------------------------------------------------
# clamped directions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("snpq,sign", [(32767, 1.0), (-32768, -1.0)])
def test_header_snp_beyond_limit_is_clamp_line(snpq, sign):
    """Header sin(phi) = 32767/32768 or -1: the start direction is +-SNP_MAX
    (F_SNP), and with Bz = 0 and zero residuals the track is the straight line
    at that slope; pads and times follow it (pads clamp at the plane's ends
    with F_PAD once the line leaves [0, 65535])."""
    row0 = 20
    hdr = dict(sec0=4, row0=row0, pad0=center_pad(row0), time0=40000, qpt=0, snp=snpq, tgl=100)
    for n, want_flags in ((10, oracle.F_SNP), (80, oracle.F_SNP | oracle.F_PAD)):
        if sign < 0 and n == 10:
            n = 2  # the line reaches pad 0 after two rows
        got, st = decode_track(hdr, [(1, 0)] * (n - 1), 0.0)
        y0 = y_of(hdr["pad0"], row0)
        X0 = pg.ROW_X[row0]
        tgl = hdr["tgl"] / 4096.0
        for j, (_, pad, time) in enumerate(got):
            r = row0 + j
            dx = pg.ROW_X[r] - X0
            y = y0 + sign * SLOPE * dx
            assert check(pad, pad_code(y, r)), (n, j, pad, pad_code(y, r))
            z = tgl * dx * math.sqrt(1.0 + SLOPE * SLOPE)
            assert check_rounded(time, hdr["time0"] + z * 32.0 / VD), (j, time)
        assert st == want_flags, (n, st)


def test_nan_curvature_gives_straight_line_along_x():
    """Bz = inf and q/pT = 0: the curvature is 0 * inf = NaN, so every
    propagated sin(phi) is NaN and becomes 0 (F_SNP).  With a header
    direction of 0 the track runs along x: the same y on every row."""
    row0 = 30
    hdr = dict(sec0=9, row0=row0, pad0=center_pad(row0) + 333, time0=90000, qpt=0, snp=0, tgl=-700)
    got, st = decode_track(hdr, [(1, 0)] * 40, float("inf"))
    y0 = y_of(hdr["pad0"], row0)
    tgl = hdr["tgl"] / 4096.0
    for j, (_, pad, time) in enumerate(got):
        r = row0 + j
        assert check_rounded(pad, pad_code(y0, r)), (j, pad)
        assert check_rounded(time, hdr["time0"] + tgl * (pg.ROW_X[r] - pg.ROW_X[row0]) * 32.0 / VD)
    assert st == oracle.F_SNP


@pytest.mark.parametrize("qpt", [5000, -5000])
def test_infinite_curvature_overshoots_to_the_limit(qpt):
    """Bz = inf, q/pT != 0: the first step's sin(phi) overshoots to +-inf and is
    clamped to +-SNP_MAX (F_SNP).  That step is the circle arc from direction 0
    to asin(+-SNP_MAX): dy = dx tan(asin(+-SNP_MAX) / 2); afterwards the track
    is the line at the clamp slope."""
    row0 = 70
    hdr = dict(sec0=20, row0=row0, pad0=center_pad(row0), time0=50000, qpt=qpt, snp=0, tgl=0)
    sign = 1.0 if qpt > 0 else -1.0
    got, st = decode_track(hdr, [(1, 0)] * 6, float("inf"))
    y = y_of(hdr["pad0"], row0)
    for j, (_, pad, time) in enumerate(got):
        r = row0 + j
        if j == 1:
            y += (pg.ROW_X[r] - pg.ROW_X[r - 1]) * math.tan(sign * math.asin(SMAX) / 2.0)
        elif j > 1:
            y += (pg.ROW_X[r] - pg.ROW_X[r - 1]) * sign * SLOPE
        assert check(pad, pad_code(y, r)), (j, pad, pad_code(y, r))
        assert time == hdr["time0"]
    assert st & oracle.F_SNP and not st & ~(oracle.F_SNP | oracle.F_PAD)


def test_finite_curvature_overshoots_to_the_limit():
    """A stiff curvature (q/pT = 16 c/GeV at 0.5 T) from sin(phi) = 0.99: the
    first step would reach sin(phi) > 1 and is clamped to SNP_MAX, so it is
    the arc from asin(0.99) to asin(SNP_MAX); every later step stays at the
    limit (straight line)."""
    row0 = 100
    s0q = 32440
    hdr = dict(sec0=30, row0=row0, pad0=center_pad(row0) - 20 * 32, time0=50000, qpt=16384,
               snp=s0q, tgl=0)
    got, st = decode_track(hdr, [(1, 0)] * 4, 0.5)
    y = y_of(hdr["pad0"], row0)
    phi0 = math.asin(s0q / 32768.0)
    for j, (_, pad, _t) in enumerate(got):
        r = row0 + j
        if j == 1:
            y += (pg.ROW_X[r] - pg.ROW_X[r - 1]) * math.tan((phi0 + math.asin(SMAX)) / 2.0)
        elif j > 1:
            y += (pg.ROW_X[r] - pg.ROW_X[r - 1]) * SLOPE
        assert check(pad, pad_code(y, r)), (j, pad, pad_code(y, r))
    assert st == oracle.F_SNP


def test_update_pushes_direction_past_the_limit():
    """A pad residual of +100/32 pad at cluster 1 tilts sin(phi) by
    (100 * pw / 32) * 0.0625 / pitch > 0.05 from 0.95: clamped to SNP_MAX
    (F_SNP).  Cluster 1 itself is the line's prediction plus the residual;
    from there on the track is the clamp-slope line through the moved point."""
    row0 = 10
    s0q = int(round(0.95 * 32768))
    hdr = dict(sec0=0, row0=row0, pad0=center_pad(row0) - 20 * 32, time0=30000, qpt=0, snp=s0q, tgl=0)
    got, st = decode_track(hdr, [(1, 0)] * 6, 0.0, res={1: (100, 0)})
    s0 = s0q / 32768.0
    t0 = s0 / math.sqrt(1.0 - s0 * s0)
    y1 = y_of(hdr["pad0"], row0) + (pg.ROW_X[row0 + 1] - pg.ROW_X[row0]) * t0
    assert check(got[1][1], pad_code(y1, row0 + 1) + 100)
    y = y1 + 100 * pg.ROW_PW[row0 + 1] / 32.0
    for j in range(2, len(got)):
        r = row0 + j
        y += (pg.ROW_X[r] - pg.ROW_X[r - 1]) * SLOPE
        assert check(got[j][1], pad_code(y, r)), (j, got[j][1], pad_code(y, r))
    assert st == oracle.F_SNP


# ---------------------------------------------------------------------------
# rotation that turns the direction backwards
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,phi_deg", [(17, 80.0), (9, 0.0), (1, -75.0)])
def test_rotation_backwards_sets_rot_flag(d, phi_deg):
    """Rotating the frame by beta (d * 20 degrees, d >= 9 written as
    180 + (d - 9) * 20) leaves cos(phi - beta) <= 0 for these directions:
    F_ROT.  The model then follows the forward direction with sine
    sin(phi - beta) from the rotated point, a straight line at Bz = 0."""
    row0 = 50
    s0q = int(round(math.sin(math.radians(phi_deg)) * 32768))
    hdr = dict(sec0=3, row0=row0, pad0=center_pad(row0), time0=60000, qpt=0, snp=s0q, tgl=0)
    got, st = decode_track(hdr, [(1, d)] + [(1, 0)] * 5, 0.0)
    beta = math.radians(d * 20.0) if d < 9 else math.pi + math.radians((d - 9) * 20.0)
    phi = math.asin(s0q / 32768.0)
    x0, y0 = pg.ROW_X[row0], y_of(hdr["pad0"], row0)
    xr = x0 * math.cos(beta) + y0 * math.sin(beta)
    yr = y0 * math.cos(beta) - x0 * math.sin(beta)
    sr = math.sin(phi - beta)
    assert math.cos(phi - beta) <= 0.0 and abs(sr) < SMAX
    slope = sr / math.sqrt(1.0 - sr * sr)
    checked = 0
    for j in range(1, len(got)):
        r = row0 + j
        y = yr + (pg.ROW_X[r] - xr) * slope
        assert check(got[j][1], pad_code(y, r)), (j, got[j][1], pad_code(y, r))
        checked += 0 <= pad_code(y, r) <= 65535
    # (d = 1 from -75 degrees puts every later cluster below pad 0: clamped)
    assert checked >= (1 if d != 1 else 0)
    assert st & oracle.F_ROT and not st & ~(oracle.F_ROT | oracle.F_PAD)
    # the same direction rotated the other way (or not at all) stays forward
    got2, st2 = decode_track(hdr, [(1, 0)] * 6, 0.0)
    assert not st2 & oracle.F_ROT


# ---------------------------------------------------------------------------
# pad and time clamps
# ---------------------------------------------------------------------------
def test_pad_residual_clamps_output_not_state():
    """A residual that puts the decoded pad below 0 or above 65535 clamps the
    OUTPUT (F_PAD) while the state still moves by the stored residual: the
    next cluster follows the closed form of the kicked track."""
    row0 = 40
    for pad0, kick in ((96, -200), (65535 - 64, 200)):
        hdr = dict(sec0=7, row0=row0, pad0=pad0, time0=70000, qpt=0, snp=0, tgl=0)
        got, st = decode_track(hdr, [(1, 0)] * 3, 0.0, res={1: (kick, 0)})
        exp = closed_form_track(dict(hdr), [(1, 0)] * 3, 0.0, kicks={1: (kick, 0)})
        assert check(got[1][1], exp[1][2] + kick)
        assert got[1][1] in (0, 65535)
        for j in (2, 3):
            assert check(got[j][1], exp[j][2]), (j, got[j][1], exp[j][2])
        assert st == oracle.F_PAD


def test_header_time_beyond_limit():
    """Header time >= 2^24: the track's time origin is 2^24 - 1 (F_TIME); the
    header cluster is written with it, and later clusters add the propagated
    time to that origin and clamp again when they exceed it."""
    row0 = 60
    for time0 in ((1 << 24), (1 << 24) + 5, 0xFFFFFFFF):
        for tglq, res in ((-2000, {}), (2000, {}), (0, {2: (0, 3)})):
            hdr = dict(sec0=11, row0=row0, pad0=center_pad(row0), time0=time0, qpt=0, snp=0, tgl=tglq)
            got, st = decode_track(hdr, [(1, 0)] * 4, 0.0, res=res)
            assert got[0][2] == TLIM
            tgl = tglq / 4096.0
            for j in range(1, 5):
                z = tgl * (pg.ROW_X[row0 + j] - pg.ROW_X[row0])
                extra = 3 if (res and j == 2) else 0
                assert check(got[j][2], TLIM + z * 32.0 / VD + extra, 0.0, float(TLIM)), (j, got[j][2])
            assert st == oracle.F_TIME


def test_time_below_zero_and_residual_above_limit():
    """A track drifting to negative times clamps them to 0; a time residual
    that passes 2^24 - 1 clamps to 2^24 - 1 (both F_TIME); the state keeps
    the stored residual."""
    row0 = 0
    hdr = dict(sec0=18, row0=row0, pad0=center_pad(row0), time0=20, qpt=0, snp=0, tgl=-4096)
    got, st = decode_track(hdr, [(1, 0)] * 5, 0.0)
    assert got[0][2] == 20
    for j in range(1, 6):
        z = -(pg.ROW_X[row0 + j] - pg.ROW_X[row0])
        assert check(got[j][2], 20 + z * 32.0 / VD, 0.0, float(TLIM))
        assert got[j][2] == 0
    assert st == oracle.F_TIME
    hdr = dict(hdr, time0=TLIM - 100, tgl=0)
    got, st = decode_track(hdr, [(1, 0)] * 3, 0.0, res={1: (0, 200)})
    assert got[1][2] == TLIM
    # the residual moved z by 200 time quanta; the next clusters sit there too
    assert got[2][2] == TLIM and got[3][2] == TLIM
    assert st == oracle.F_TIME
    # below the limit the same track follows the closed form of the kicked
    # track (z moved by the residual, tan(lambda) tilted by the gain)
    hdr = dict(hdr, time0=TLIM - 1000)
    got, st = decode_track(hdr, [(1, 0)] * 3, 0.0, res={1: (0, 200)})
    exp = closed_form_track(dict(hdr), [(1, 0)] * 3, 0.0, kicks={1: (0, 200)})
    assert got[1][2] == TLIM - 800
    for j in (2, 3):
        assert check_rounded(got[j][2], exp[j][3]) and got[j][2] > TLIM - 800, (j, got[j][2], exp[j][3])
    assert st == 0


def test_runaway_state_saturates_then_nan_decodes_residuals():
    """Garbage that blows the float state up: every cluster turns the frame
    by 100 degrees (sector step 5, same row) and carries a pad residual that
    re-tilts the direction.  Each rotation maps the large |y| into x, so the
    next step's dx, and with it |y|, grow by a factor every step: the state
    passes float range.  Defined semantics on that path:
      - while the prediction is +-inf, the float->int conversion saturates at
        +-2^30 and the clamps give pad 0 / 65535 and time 2^24 - 1 or 0;
      - once the position and z are NaN (inf - inf), the conversion gives 0, so
        the decoded codes are exactly the stored residuals (pad = residual,
        time = header time + residual); NaN never leaves those variables."""
    row0, n = 30, 120
    t0, pres, tres = 1000000, 908, 100
    cl = [(0, 0, 0, 0, 1, 1)] + [(0, 5, pres, tres, 1, 1)] * (n - 1)
    hdr = dict(sec0=2, row0=row0, pad0=center_pad(row0), time0=t0, qpt=0, snp=0, tgl=400)
    out, st = oracle.decode(build_frame([dict(hdr, cl=cl)]), bz=0.0)
    # the track visits the bins of sectors 2, 7, 12, 17, 4, ... on one row, in order
    sec, seen, vals = 2, {}, []
    for j in range(n):
        if j:
            sec = (sec + 5) % 18
        b = sec * 152 + row0
        i = int(out["row_offset"][b]) + seen.get(b, 0)
        seen[b] = seen.get(b, 0) + 1
        vals.append((int(out["pad"][i]), int(out["time"][i])))
    assert all(v == (pres, t0 + tres) for v in vals[-40:]), vals[-40:]
    sat = [j for j, (p, t) in enumerate(vals) if t == TLIM and p in (0, 65535)]
    assert len(sat) >= 10 and max(sat) < n - 40
    assert st == oracle.F_ROT | oracle.F_SNP | oracle.F_PAD | oracle.F_TIME

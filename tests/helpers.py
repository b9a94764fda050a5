"""Test helpers: hand-built frames and closed-form track geometry (float64).

Nothing here decodes a stream; the closed forms follow circle and line
geometry (oracle.physgen.helix_to_line intersects a circle, given by its
centre and radius, with a pad-row line)."""
import math

import numpy as np

from oracle import physgen as pg

NSEC, NROW = 36, 152
NBIN = NSEC * NROW
VD = 0.516

TRACK_KEYS = [("trk_ncls", np.uint8), ("trk_sec0", np.uint8), ("trk_row0", np.uint8),
              ("trk_pad0", np.uint16), ("trk_time0", np.uint32), ("trk_qpt", np.int16),
              ("trk_snp", np.int16), ("trk_tgl", np.int16)]
CL_KEYS = [("cls_row_diff", np.int8), ("cls_sec_diff", np.uint8), ("cls_pad_res", np.int16),
           ("cls_time_res", np.int16), ("cls_qtot", np.uint16), ("cls_qmax", np.uint16)]
UN_KEYS = [("un_time_diff", np.uint32), ("un_pad_diff", np.uint16), ("un_qtot", np.uint16),
           ("un_qmax", np.uint16)]


def build_frame(tracks, unattached=None):
    """tracks: list of dicts with header keys sec0,row0,pad0,time0,qpt,snp,tgl
    (quantised ints) and 'cl': list of (rowdiff, secdiff, padres, timeres,
    qtot, qmax) for clusters 0..n-1 (cluster 0's steps and residuals are
    ignored by the decoder).  unattached: dict bin -> list of (tdiff, pdiff,
    qtot, qmax)."""
    fr = {}
    hdr = {"trk_ncls": [len(t["cl"]) for t in tracks]}
    for k in ("sec0", "row0", "pad0", "time0", "qpt", "snp", "tgl"):
        hdr["trk_" + k] = [t[k] for t in tracks]
    for k, dt in TRACK_KEYS:
        fr[k] = np.array(hdr[k], dtype=np.int64).astype(dt)
    cl = [c for t in tracks for c in t["cl"]]
    for i, (k, dt) in enumerate(CL_KEYS):
        fr[k] = np.array([c[i] for c in cl], dtype=np.int64).astype(dt)
    un = unattached or {}
    fr["un_count"] = np.zeros(NBIN, np.uint32)
    rows = []
    for b in sorted(un):
        fr["un_count"][b] = len(un[b])
        rows.extend(un[b])
    for i, (k, dt) in enumerate(UN_KEYS):
        fr[k] = np.array([r[i] for r in rows], dtype=np.int64).astype(dt)
    return fr


def empty_frame():
    return build_frame([], {})


def closed_form_track(hdr, steps, bz, kicks=None, tilt_sign=1.0):
    """Expected (pad, time) values, as float64 in 1/32 units, of a track whose
    header is `hdr` (quantised ints) and whose clusters follow (rowdiff,
    secdiff) steps.  Without kicks all residuals are zero, so the decoded
    cluster positions lie on the circle (line for k == 0) fixed by the header.
    kicks: {j: (padres, timeres)} applies the documented update at cluster j:
    position moved by the residual, sin(phi) tilted by 0.0625/pitch times the
    pad shift in cm, tan(lambda) by 0.0625/pitch times the time shift in cm.

    Returns a list of (sector, row, pad_value, time_value), or None when the
    header's circle does not reach one of the rows (the track turns back)."""
    kicks = kicks or {}
    sec, row = hdr["sec0"], hdr["row0"]
    X0 = pg.ROW_X[row]
    y0 = (hdr["pad0"] / 32.0 - pg.ROW_NPADS[row] / 2) * pg.ROW_PW[row]
    s0 = hdr["snp"] / 32768.0
    tgl = hdr["tgl"] / 4096.0
    k = hdr["qpt"] / 1024.0 * bz * 0.00299792458
    alpha = pg.sector_angle(sec)
    gx, gy = pg.to_global(X0, y0, alpha)
    phi = math.asin(s0) + alpha
    z = 0.0
    res = [(sec, row, float(hdr["pad0"]), float(hdr["time0"]))]
    for j, (rd, sd) in enumerate(steps, start=1):
        sec = (sec // 18) * 18 + (sec % 18 + sd) % 18
        row = row + rd
        X = pg.ROW_X[row]
        alpha = pg.sector_angle(sec)
        hit = pg.helix_to_line(gx, gy, phi, k, alpha, X)
        if hit is None:
            return None  # the circle never reaches this row moving outward
        y, v, arc = hit
        nx, ny = pg.to_global(X, y, alpha)
        # the model's chord is signed by the step in local x (a rotation at a
        # sector edge can put the start beyond the next row's line)
        dxl = X - pg.to_local(gx, gy, alpha)[0]
        z += tgl * math.copysign(math.hypot(nx - gx, ny - gy), dxl)
        pad = (y / pg.ROW_PW[row] + pg.ROW_NPADS[row] / 2) * 32.0
        tval = hdr["time0"] + z * 32.0 / VD
        res.append((sec, row, pad, tval))
        if j in kicks:
            pr, tr = kicks[j]
            g = 0.0625 / pg.PITCH[pg.region(row)]
            dy = pr * pg.ROW_PW[row] / 32.0
            dz = tr * VD / 32.0
            y += dy
            z += dz
            v = math.asin(math.sin(v) + tilt_sign * dy * g)
            tgl += dz * g
            nx, ny = pg.to_global(X, y, alpha)
        gx, gy = nx, ny
        phi = v + alpha
    return res


def near_tie(v, margin=0.1):
    """True if v is within `margin` of a rounding tie (x.5)."""
    return 0.5 - abs(v - round(v)) < margin


def check_rounded(got, exact, margin=0.1):
    """got == rint(exact) when exact is >= margin from a tie, else within 1."""
    if near_tie(exact, margin):
        return abs(int(got) - exact) <= 1.0 + 1e-9
    return int(got) == int(np.rint(exact))

"""Exact-helix cluster generator in float64 -- TEST INFRASTRUCTURE ONLY.

Produces "physical" clusters: charged tracks from the origin follow an exact
helix in a uniform Bz field; each cluster is the crossing of the helix with a
pad row (the straight line x = X[row] in the local frame of the sector the
crossing lies in), smeared by Gaussian noise.  The oracle encoder turns these
into a compressed frame; the round-trip pin then checks that decoding restores
the quantised clusters exactly.

The geometry below is written independently of the oracle's float tables: row
radii and pad counts are recomputed here in double precision from the detector
description (4 pad regions, 152 rows, 36 sectors of 20 degrees).

Conventions: sector s is centred at azimuth (s % 18) * 20 + 10 degrees; local x
points radially through the sector centre, local y along increasing azimuth;
curvature k > 0 turns the direction counter-clockwise, k = q/pT * Bz *
0.00299792458 per cm.
"""
import math

import numpy as np

NSEC, NROW = 36, 152
REGION_START = (0, 63, 97, 127, 152)
REGION_X0 = (84.85, 134.0, 168.0, 204.0)
PITCH = (0.75, 1.00, 1.20, 1.50)
PADW = (0.416, 0.608, 0.608, 0.608)
VDRIFT = 0.516
TAN10 = math.tan(math.pi / 18)


def region(row):
    g = 0
    while row >= REGION_START[g + 1]:
        g += 1
    return g


ROW_X = np.array([REGION_X0[region(r)] + (r - REGION_START[region(r)] + 0.5) * PITCH[region(r)]
                  for r in range(NROW)])
ROW_PW = np.array([PADW[region(r)] for r in range(NROW)])
ROW_NPADS = np.array([2 * math.floor(ROW_X[r] * TAN10 / ROW_PW[r]) for r in range(NROW)])


def sector_angle(sec):
    return math.radians((sec % 18) * 20.0 + 10.0)


def to_local(px, py, alpha):
    ca, sa = math.cos(alpha), math.sin(alpha)
    return px * ca + py * sa, -px * sa + py * ca


def to_global(lx, ly, alpha):
    ca, sa = math.cos(alpha), math.sin(alpha)
    return lx * ca - ly * sa, lx * sa + ly * ca


def helix_to_line(px, py, phi, k, alpha, X):
    """Follow the circle through global point (px, py) with global direction
    phi and curvature k to the line x' = X of the frame rotated by alpha.

    Returns (y', local direction at the crossing, xy path length), or None if
    the circle does not reach the line moving outward (cos of the local
    direction must stay positive)."""
    x0, y0 = to_local(px, py, alpha)
    u = phi - alpha
    su, cu = math.sin(u), math.cos(u)
    if cu <= 0.0:
        return None
    if k == 0.0:
        y = y0 + (X - x0) * su / cu
        v = u
    else:
        # centre of the circle: a distance 1/|k| to the left of the direction
        # for k > 0 (counter-clockwise), to the right for k < 0
        cx, cy = x0 - su / k, y0 + cu / k
        R = 1.0 / abs(k)
        h2 = R * R - (X - cx) ** 2
        if h2 < 0.0:
            return None
        # moving outward (d x'/ds > 0) selects the root below the centre for
        # k > 0 and above it for k < 0
        y = cy - math.copysign(math.sqrt(h2), k)
        sv = k * (X - cx)
        if abs(sv) >= 1.0:
            return None
        v = math.asin(sv)
        # same branch as the start: the direction must not have turned past
        # +-90 degrees on the way
        if abs(v - u) >= math.pi / 2:
            return None
    chord = math.hypot(X - x0, y - y0)
    # arc = chord * (dphi/2) / sin(dphi/2)
    h = 0.5 * (v - u)
    arc = chord if abs(h) < 1e-9 else chord * h / math.sin(h)
    return y, v, arc


def make_track(rng, bz, pt, q, tgl, phi0, side, row_first, max_len, noise=0.05, allow_cross=True):
    """Clusters of one track from the origin.  Returns a dict of lists (may be
    shorter than max_len: the track stops at row 151, when its local direction
    exceeds |sin| 0.9, or at a sector edge when allow_cross is False)."""
    k = q / pt * bz * 0.00299792458
    px = py = 0.0
    phi = phi0
    sec = None
    out = {"sec": [], "row": [], "y": [], "snp": [], "z": []}
    z = 0.0
    for r in range(row_first, NROW):
        if len(out["row"]) >= max_len:
            break
        X = ROW_X[r]
        if sec is None:
            # sector whose frame contains the first crossing: try the sector of
            # the initial direction and its neighbours
            best = None
            base = int(math.floor((phi0 % (2 * math.pi)) / math.radians(20.0))) % 18
            for cand in (base, (base + 1) % 18, (base + 17) % 18):
                res = helix_to_line(px, py, phi, k, sector_angle(cand), X)
                if res is not None and abs(res[0]) <= X * TAN10:
                    best = (cand, res)
                    break
            if best is None:
                break
            sec = side * 18 + best[0]
            res = best[1]
        else:
            res = helix_to_line(px, py, phi, k, sector_angle(sec), X)
            if res is None:
                break
            if abs(res[0]) > X * TAN10:
                if not allow_cross:
                    break
                nxt = side * 18 + ((sec % 18) + (1 if res[0] > 0 else 17)) % 18
                res = helix_to_line(px, py, phi, k, sector_angle(nxt), X)
                if res is None or abs(res[0]) > X * TAN10:
                    break
                sec = nxt
        y, v, arc = res
        if abs(math.sin(v)) > 0.9:
            break
        alpha = sector_angle(sec)
        gx, gy = to_global(X, y, alpha)
        phi = v + alpha
        px, py = gx, gy
        z += tgl * arc
        out["sec"].append(sec)
        out["row"].append(r)
        out["y"].append(y + rng.normal(0.0, noise))
        out["snp"].append(math.sin(v))
        out["z"].append(z + rng.normal(0.0, noise))
    return out


def generate(seed=0, n_tracks=200, n_un=1000, bz=0.5, pt_range=(0.2, 10.0), noise=0.05,
             allow_cross=True, min_len=2):
    """Physical clusters for the oracle encoder (see oracle.encode)."""
    rng = np.random.default_rng(seed)
    trk_first, trk_qpt, trk_tgl = [0], [], []
    cols = {"cl_sec": [], "cl_row": [], "cl_pad": [], "cl_time": [], "cl_snp": [], "cl_qtot": [],
            "cl_qmax": []}
    while len(trk_qpt) < n_tracks:
        pt = math.exp(rng.uniform(math.log(pt_range[0]), math.log(pt_range[1])))
        q = 1.0 if rng.random() < 0.5 else -1.0
        tgl = rng.uniform(-1.0, 1.0)
        phi0 = rng.uniform(0.0, 2 * math.pi)
        side = int(rng.integers(0, 2))
        row_first = int(rng.integers(0, 40))
        max_len = int(rng.integers(min_len, NROW + 1))
        t = make_track(rng, bz, pt, q, tgl, phi0, side, row_first, max_len, noise, allow_cross)
        n = len(t["row"])
        if n < min_len:
            continue
        t_first = 600.0 + rng.uniform(0.0, 485.0)
        z0 = t["z"][0]
        for i in range(n):
            r = t["row"][i]
            cols["cl_sec"].append(t["sec"][i])
            cols["cl_row"].append(r)
            # keep the smeared position on the pad plane
            pad = t["y"][i] / ROW_PW[r] + ROW_NPADS[r] / 2
            cols["cl_pad"].append(min(max(pad, 0.0), ROW_NPADS[r] - 0.05))
            cols["cl_time"].append(t_first + (t["z"][i] - z0) / VDRIFT)
            cols["cl_snp"].append(t["snp"][i])
            qmax = 1 + int(rng.exponential(30.0))
            cols["cl_qmax"].append(min(qmax, 65535))
            cols["cl_qtot"].append(min(qmax + int(rng.exponential(120.0)), 65535))
        trk_first.append(trk_first[-1] + n)
        trk_qpt.append(q / pt)
        trk_tgl.append(tgl)
    phys = {"trk_first": np.array(trk_first, np.uint32), "trk_qpt": np.array(trk_qpt),
            "trk_tgl": np.array(trk_tgl)}
    dt = {"cl_sec": np.uint8, "cl_row": np.uint8, "cl_pad": np.float64, "cl_time": np.float64,
          "cl_snp": np.float64, "cl_qtot": np.uint16, "cl_qmax": np.uint16}
    for kname, v in cols.items():
        phys[kname] = np.array(v, dt[kname])
    un_sec = rng.integers(0, NSEC, n_un).astype(np.uint8)
    un_row = rng.integers(0, NROW, n_un).astype(np.uint8)
    phys["un_sec"], phys["un_row"] = un_sec, un_row
    phys["un_pad"] = rng.uniform(0.0, 1.0, n_un) * ROW_NPADS[un_row]
    phys["un_time"] = rng.uniform(0.0, 20000.0, n_un)
    qmax = 1 + np.floor(rng.exponential(30.0, n_un))
    phys["un_qmax"] = np.minimum(qmax, 65535).astype(np.uint16)
    phys["un_qtot"] = np.minimum(qmax + np.floor(rng.exponential(120.0, n_un)), 65535).astype(np.uint16)
    return phys


def quantize(phys):
    """The values decoding must restore, per cluster: (bin, padQ, timeQ, qtot,
    qmax) for attached clusters in track order, and for unattached ones."""
    att = {"bin": phys["cl_sec"].astype(np.int64) * NROW + phys["cl_row"],
           "pad": np.rint(phys["cl_pad"] * 32).astype(np.int64),
           "time": np.rint(phys["cl_time"] * 32).astype(np.int64),
           "qtot": phys["cl_qtot"].astype(np.int64), "qmax": phys["cl_qmax"].astype(np.int64)}
    un = {"bin": phys["un_sec"].astype(np.int64) * NROW + phys["un_row"],
          "pad": np.rint(phys["un_pad"] * 32).astype(np.int64),
          "time": np.rint(phys["un_time"] * 32).astype(np.int64),
          "qtot": phys["un_qtot"].astype(np.int64), "qmax": phys["un_qmax"].astype(np.int64)}
    return att, un


def expected_clusters(phys):
    """Canonical decoded layout of quantize(phys), built with numpy only:
    inside each (sector, row) bin, attached clusters in stream order, then
    unattached clusters sorted by (time, pad, qTot, qMax)."""
    att, un = quantize(phys)
    nb = NSEC * NROW
    na = np.bincount(att["bin"], minlength=nb)
    nu = np.bincount(un["bin"], minlength=nb)
    off = np.concatenate([[0], np.cumsum(na + nu)]).astype(np.uint32)
    order_a = np.argsort(att["bin"], kind="stable")
    order_u = np.lexsort((un["qmax"], un["qtot"], un["pad"], un["time"], un["bin"]))
    n = int(off[-1])
    res = {k: np.zeros(n, np.int64) for k in ("time", "pad", "qtot", "qmax")}
    # position of each attached cluster: off[bin] + rank among same-bin ones
    a_bins = att["bin"][order_a]
    a_rank = np.arange(len(a_bins)) - np.searchsorted(a_bins, a_bins, side="left")
    a_pos = off[a_bins] + a_rank
    u_bins = un["bin"][order_u]
    u_rank = np.arange(len(u_bins)) - np.searchsorted(u_bins, u_bins, side="left")
    u_pos = off[u_bins] + na[u_bins] + u_rank
    for kname in res:
        res[kname][a_pos] = att[kname][order_a]
        res[kname][u_pos] = un[kname][order_u]
    return {"row_offset": off, "row_nattached": na.astype(np.uint32),
            "time": res["time"].astype(np.uint32), "pad": res["pad"].astype(np.uint16),
            "qtot": res["qtot"].astype(np.uint16), "qmax": res["qmax"].astype(np.uint16)}

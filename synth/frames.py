"""Synthetic compressed time frames shaped like Pb-Pb running.

The generator writes the compressed streams directly: track headers, per-cluster
row/sector steps, residuals, charges, and per-(sector,row) delta streams of
unattached clusters.  It uses its own double-precision picture of the detector:
charged tracks are circles through the origin in a uniform field, and each
cluster sits where a circle crosses a pad row.  This geometry decides
  - which rows and sectors each track visits, including sector crossings and
    the legs of low-pT loopers,
  - the header values (pad, sin(phi), q/pT, tan(lambda)) at a track's first
    cluster, and
  - the true position of every cluster (local y; z from the arc length times
    tan(lambda)), which is then smeared by Gaussian noise (sigma 0.05 cm in y
    and in z) and quantised to 1/32 pad and 1/32 time bin.
Residuals are measured code minus predicted code.  The prediction comes from a
float64 geometric shadow of the documented track model (helix step, rotation
at sector edges, fixed-gain update), started from the quantised header, so the
shadow follows the measured clusters and the float32 decoder reproduces them
(up to one code where the two roundings fall on either side of a tie).  Tracks
whose shadow comes near a limit of the model (|sin phi| > 0.98, a rotation
leaving cos phi < 0.05) are redrawn, pads are kept one code inside the pad
plane and header times are raised so that no time code falls below 32: the
streams of every workload decode with no status flag.

Frame layout: see the key list in FIELDS below.  Stream order: tracks in
collision order; each track's clusters are contiguous; unattached clusters are
sector-major, then row, and each (sector,row) bin is a delta stream.
"""
import dataclasses
import math

import numpy as np

NSEC, NROW = 36, 152
NBIN = NSEC * NROW

# detector picture used only to shape the synthetic distributions
_RSTART = (0, 63, 97, 127, 152)
_RX0 = (84.85, 134.0, 168.0, 204.0)
_PITCH = (0.75, 1.00, 1.20, 1.50)
_PADW = (0.416, 0.608, 0.608, 0.608)
_VDRIFT = 0.516  # cm per time bin
_TAN10 = math.tan(math.radians(10.0))
_REG = np.repeat(np.arange(4), np.diff(_RSTART))
ROW_X = np.array([_RX0[g] + (r - _RSTART[g] + 0.5) * _PITCH[g] for r, g in enumerate(_REG)])
ROW_PW = np.array([_PADW[g] for g in _REG])
ROW_NPADS = (2 * np.floor(ROW_X * _TAN10 / ROW_PW)).astype(np.int64)
ROW_GAIN = np.array([0.0625 / _PITCH[g] for g in _REG])   # update gain per cm of innovation
SIGMA_CM = 0.05          # cluster position noise in y and in z
S_LIMIT = 0.98           # the shadow's |sin phi| must stay below this
ROT_COS_MIN = 0.05       # ... and cos phi above this after a rotation

FIELDS = {
    "trk_ncls": np.uint8, "trk_sec0": np.uint8, "trk_row0": np.uint8, "trk_pad0": np.uint16,
    "trk_time0": np.uint32, "trk_qpt": np.int16, "trk_snp": np.int16, "trk_tgl": np.int16,
    "cls_row_diff": np.int8, "cls_sec_diff": np.uint8, "cls_pad_res": np.int16,
    "cls_time_res": np.int16, "cls_qtot": np.uint16, "cls_qmax": np.uint16,
    "un_count": np.uint32, "un_time_diff": np.uint32, "un_pad_diff": np.uint16,
    "un_qtot": np.uint16, "un_qmax": np.uint16,
}


@dataclasses.dataclass
class FrameSpec:
    """Shape of one synthetic frame."""
    collisions: int = 100
    tracks_per_collision: int = 2000
    n_tracks: int = 0              # if > 0: fixed track count, overrides collisions
    ncls_min: int = 5
    ncls_max: int = 152
    pt_min: float = 0.1
    pt_max: float = 10.0
    crosser_frac: float = 0.10
    looper_frac: float = 0.0       # fraction of tracks that are low-pT loopers
    looper_pt: tuple = (0.05, 0.15)
    looper_turns: int = 4
    row_skew: float = 0.0          # > 0: start rows and unattached rows ~ exp(-row/row_skew)
    sectors: tuple = tuple(range(NSEC))
    n_unattached: int = -1         # < 0: unattached = attached * unattached_ratio
    unattached_ratio: float = 0.4 / 0.6
    bz: float = 0.5
    seed: int = 0
    frame_index: int = 0

    def tracks(self):
        return self.n_tracks if self.n_tracks > 0 else self.collisions * self.tracks_per_collision


# The workloads, each with its own seed:
#   tiny     one sector, 1000 tracks of 20..152 clusters, 20000 unattached
#   frame    one Pb-Pb-like time frame: 100 collisions x 2000 tracks
#   batched  frames of 10..200 collisions (log-uniform), see batch_specs
#   served   the same frame mix, drawn with another seed
#   stress   500 collisions, 15% low-pT loopers, rows skewed exp(-row/40)
WORKLOADS = {
    "tiny": FrameSpec(n_tracks=1000, collisions=1, ncls_min=20, ncls_max=152, crosser_frac=0.0,
                      sectors=(0,), n_unattached=20000, seed=0),
    "frame": FrameSpec(collisions=100, seed=1),
    "batched": FrameSpec(collisions=100, seed=2),
    "served": FrameSpec(collisions=100, seed=3),
    "stress": FrameSpec(collisions=500, looper_frac=0.15, row_skew=40.0, seed=4),
}


def spec_for(name: str, **over) -> FrameSpec:
    return dataclasses.replace(WORKLOADS[name], **over)


def batch_specs(name: str = "batched", n_frames: int = 64, seed: int = None, coll_range=(10, 200)):
    """Frames with collision counts log-uniform in coll_range (batched and
    served workloads)."""
    base = WORKLOADS[name]
    seed = base.seed if seed is None else seed
    rng = np.random.default_rng([seed, 7919])
    lo, hi = math.log(coll_range[0]), math.log(coll_range[1])
    colls = np.rint(np.exp(rng.uniform(lo, hi, n_frames))).astype(int)
    return [dataclasses.replace(base, collisions=int(c), seed=seed, frame_index=i)
            for i, c in enumerate(colls)]


# ---------------------------------------------------------------------------
# geometry helpers (circle through the origin, local sector frame)
# ---------------------------------------------------------------------------
def _local_track(u, k, X):
    """Local sin(phi) and y where the circle through the origin with local
    start direction u and curvature k crosses the line x = X."""
    su, cu = np.sin(u), np.cos(u)
    s = su + k * X
    c = np.sqrt(np.maximum(1.0 - s * s, 0.0))
    y = X * (su + s) / (cu + c)
    return s, y


def _arc_from_origin(r, k, inward=False):
    """Arc length from the origin along a circle through it (curvature k) to a
    point at distance r from the origin; inward: on the returning half."""
    ak = np.abs(k)
    safe = np.where(ak > 1e-12, ak, 1.0)
    half = np.arcsin(np.clip(ak * r / 2.0, 0.0, 1.0))
    if inward:
        return np.where(ak > 1e-12, (2.0 * math.pi - 2.0 * half) / safe, r)
    return np.where(ak > 1e-12, 2.0 * half / safe, r)


def _pad_code(y, rows):
    """Measured pad code (1/32 pad) of local y on each row, kept one code
    inside the pad plane."""
    q = np.rint((y / ROW_PW[rows] + ROW_NPADS[rows] / 2) * 32.0)
    return np.clip(q, 1, ROW_NPADS[rows] * 32 - 2).astype(np.int64)


def _shadow_residuals(rows, secst, pad_meas, tq_meas, ncls, pad0, snpq, tglq, qptq, bz):
    """Residuals of measured codes against a float64 geometric shadow of the
    track model, for m tracks at once.

    rows, secst: (m, L) row and sector step (0 or d in 1..17) of cluster j;
    pad_meas: (m, L) measured pad codes; tq_meas: (m, L) measured time codes
    relative to cluster 0; ncls: (m,) cluster counts; header: pad0 (code),
    quantised sin(phi), tan(lambda), q/pT.  Returns (pad residuals, time
    residuals, ok): ok is False for tracks whose shadow came near a limit of
    the model or needed a residual beyond int16."""
    m, L = rows.shape
    # longest tracks first: the tracks still running at step j are a prefix
    perm = np.argsort(-ncls, kind="stable")
    nc = ncls[perm]
    rows_p, sst_p = rows[perm], secst[perm]
    pad_p, tq_p = pad_meas[perm], tq_meas[perm]
    r0 = rows_p[:, 0]
    x = ROW_X[r0].copy()
    y = (pad0[perm] / 32.0 - ROW_NPADS[r0] / 2) * ROW_PW[r0]
    z = np.zeros(m)
    s = snpq[perm] / 32768.0
    tgl = tglq[perm] / 4096.0
    k = qptq[perm] / 1024.0 * (bz * 0.00299792458)
    ok = np.abs(s) < S_LIMIT
    pres = np.zeros((m, L), np.int64)
    tres = np.zeros((m, L), np.int64)
    # number of tracks with more than j clusters, for every j
    alive = np.searchsorted(-nc, -np.arange(L), side="left")
    for j in range(1, L):
        n = int(alive[j])
        if n == 0:
            break
        xs, ys, ss, ks = x[:n], y[:n], s[:n], k[:n]
        d = sst_p[:n, j]
        if d.any():
            rot = d != 0
            ang = np.radians(20.0 * d[rot])
            ca, sa = np.cos(ang), np.sin(ang)
            xr, yr, sr = xs[rot], ys[rot], ss[rot]
            cs = np.sqrt(np.maximum(1.0 - sr * sr, 0.0))
            sn = sr * ca - cs * sa
            cn = cs * ca + sr * sa
            okr = ok[:n]
            okr[rot] &= (cn > ROT_COS_MIN) & (np.abs(sn) < S_LIMIT)
            xs[rot] = xr * ca + yr * sa
            ys[rot] = yr * ca - xr * sa
            ss[rot] = sn
        rj = rows_p[:n, j]
        X = ROW_X[rj]
        dx = X - xs
        s1 = ss + ks * dx
        ok[:n] &= np.abs(s1) < S_LIMIT
        s1 = np.clip(s1, -S_LIMIT, S_LIMIT)
        sc = np.clip(ss, -S_LIMIT, S_LIMIT)
        dydx = (sc + s1) / (np.sqrt(1.0 - sc * sc) + np.sqrt(1.0 - s1 * s1))
        yp = ys + dx * dydx
        zp = z[:n] + tgl[:n] * (dx * np.sqrt(1.0 + dydx * dydx))
        pw = ROW_PW[rj]
        pr = pad_p[:n, j] - np.rint((yp / pw + ROW_NPADS[rj] / 2) * 32.0)
        tr = tq_p[:n, j] - np.rint(zp * (32.0 / _VDRIFT))
        pres[:n, j] = pr
        tres[:n, j] = tr
        nuy = pr * pw / 32.0
        nuz = tr * (_VDRIFT / 32.0)
        s2 = s1 + nuy * ROW_GAIN[rj]
        ok[:n] &= np.abs(s2) < S_LIMIT
        x[:n] = X
        y[:n] = yp + nuy
        z[:n] = zp + nuz
        s[:n] = s2
        tgl[:n] += nuz * ROW_GAIN[rj]
    ok &= (np.abs(pres) < 30000).all(axis=1) & (np.abs(tres) < 30000).all(axis=1)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(m)
    return pres[inv], tres[inv], ok[inv]


def _measure(rng, rows, y_true, z_true, ncls):
    """Measured pad codes and time codes (relative to cluster 0) of clusters
    at true local y and z (cm, z relative to cluster 0's true z), each smeared
    by Gaussian noise."""
    m, L = rows.shape
    y = y_true + rng.normal(0.0, SIGMA_CM, (m, L))
    z = z_true + rng.normal(0.0, SIGMA_CM, (m, L))
    pad = _pad_code(y, rows)
    tq = np.rint(z * (32.0 / _VDRIFT)).astype(np.int64)
    tq = tq - tq[:, :1]           # cluster 0 defines the header time
    live = np.arange(L)[None, :] < ncls[:, None]
    tq[~live] = 0
    return pad, tq


def _draw_rows(rng, n, p_gap=0.05):
    """Row steps: +1, or +2 with probability p_gap."""
    return 1 + (rng.random(n) < p_gap).astype(np.int64)


def _sample_start_rows(rng, span, skew):
    """Start row for tracks whose rows span `span` (last - first)."""
    hi = NROW - 1 - span  # inclusive upper bound, >= 0
    if skew <= 0:
        return (rng.random(span.shape) * (hi + 1)).astype(np.int64)
    # truncated exponential on [0, hi + 1)
    u = rng.random(span.shape)
    top = 1.0 - np.exp(-(hi + 1) / skew)
    r = -skew * np.log1p(-u * top)
    return np.minimum(r.astype(np.int64), hi)


def _normal_tracks(rng, spec, n):
    """Outward tracks: cluster counts, header values (quantised), row and
    sector steps, and the residuals of each cluster against the shadow model
    (pres/tres, (n, NROW)); tq_lo/tq_hi: range of the time codes relative to
    cluster 0."""
    ncls = rng.integers(spec.ncls_min, spec.ncls_max + 1, n)
    out = {k: np.zeros(n, np.int64) for k in ("sec0", "row0", "pad0", "snp", "qpt", "tgl", "tq_lo", "tq_hi")}
    crosser = rng.random(n) < spec.crosser_frac
    steps = np.zeros((n, NROW), np.int64)      # row step before cluster j (j >= 1)
    secstep = np.zeros((n, NROW), np.int64)    # sector step before cluster j
    pres = np.zeros((n, NROW), np.int16)
    tres = np.zeros((n, NROW), np.int16)
    todo = np.arange(n)
    sectors = np.asarray(spec.sectors)
    jj = np.arange(NROW)[None, :]
    for attempt in range(60):
        if todo.size == 0:
            break
        if attempt in (20, 40):
            # persistent rejects: redraw their lengths as well
            ncls[todo] = rng.integers(spec.ncls_min, spec.ncls_max + 1, todo.size)
        # longest first: the tracks still running at row step j are a prefix
        todo = todo[np.argsort(-ncls[todo], kind="stable")]
        m = todo.size
        nc = ncls[todo]
        alive = np.searchsorted(-nc, -np.arange(NROW), side="left")
        st = np.zeros((m, NROW), np.int64)
        st[:, 1:] = _draw_rows(rng, m * (NROW - 1)).reshape(m, NROW - 1)
        st[jj >= nc[:, None]] = 0
        span = st.sum(axis=1)
        bad_span = span > NROW - 1
        span = np.minimum(span, NROW - 1)
        row0 = _sample_start_rows(rng, span, spec.row_skew)
        rows = np.minimum(row0[:, None] + np.cumsum(st, axis=1), NROW - 1)
        X = ROW_X[rows]
        pt = np.exp(rng.uniform(math.log(spec.pt_min), math.log(spec.pt_max), m))
        q = np.where(rng.random(m) < 0.5, 1.0, -1.0)
        k = q / pt * spec.bz * 0.00299792458
        # position angle at the first row, uniform inside the sector (crossers:
        # in the outer half, so that most of them reach an edge)
        th = np.radians(rng.uniform(-10.0, 10.0, m))
        cr = crosser[todo]
        th[cr] = np.sign(th[cr]) * np.radians(rng.uniform(4.0, 10.0, int(cr.sum())))
        X0 = X[:, 0]
        r0 = X0 / np.cos(th)
        arg = np.clip(k * r0 / 2.0, -1.0, 1.0)
        u = th - np.arcsin(arg)            # direction at the origin, local frame
        ok = (~bad_span) & (np.abs(k * r0 / 2.0) < 1.0) & (np.cos(u) > 0.1)
        # follow the track through the rows; switch frames at sector edges
        du = np.zeros(m)                    # accumulated frame rotation
        sst = np.zeros((m, NROW), np.int64)
        ym = np.zeros((m, NROW))            # true local y of cluster j
        ncross = np.zeros(m, np.int64)
        s0 = np.zeros(m)
        for j in range(NROW):
            n = int(alive[j])
            if n == 0:
                break
            Xj = X[:n, j]
            s, y = _local_track(u[:n] - du[:n], k[:n], Xj)
            edge = Xj * _TAN10
            out_pos = y > edge
            out_neg = y < -edge
            cross = out_pos | out_neg
            if cross.any():
                # crossing into the neighbouring sector (+20 deg or -20 deg)
                du[:n] += np.radians(20.0) * out_pos - np.radians(20.0) * out_neg
                sst[:n, j] = np.where(out_pos, 1, np.where(out_neg, 17, 0))
                ncross[:n] += cross
                s2, y2 = _local_track(u[:n][cross] - du[:n][cross], k[:n][cross], Xj[cross])
                s[cross] = s2
                y[cross] = y2
            ok[:n] &= (np.abs(s) < 0.95) & (np.abs(y) <= edge * 1.0001)
            ym[:n, j] = y
            if j == 0:
                s0 = s.copy()
                ok &= (sst[:, 0] == 0)
        ok &= np.where(crosser[todo], ncross >= 1, ncross == 0)
        # measured clusters and their residuals against the shadow model, for
        # the tracks the geometry accepted
        tgl = rng.uniform(-1.0, 1.0, m)
        sec = rng.choice(sectors, m)
        gi = np.nonzero(ok)[0]
        rows_g, nc_g, k_g = rows[gi], nc[gi], k[gi]
        arc = _arc_from_origin(np.hypot(X[gi], ym[gi]), k_g[:, None])
        z_true = tgl[gi, None] * (arc - arc[:, :1])
        del arc
        pad_m, tq_m = _measure(rng, rows_g, ym[gi], z_true, nc_g)
        del z_true, ym
        hpad = pad_m[:, 0]
        hsnp = np.clip(np.rint(s0[gi] * 32768.0), -32767, 32767)
        hqpt = np.clip(np.rint((q / pt)[gi] * 1024.0), -32768, 32767)
        htgl = np.clip(np.rint(tgl[gi] * 4096.0), -32768, 32767)
        pr, tr, sh_ok = _shadow_residuals(rows_g, sst[gi], pad_m, tq_m, nc_g, hpad, hsnp, htgl, hqpt, spec.bz)
        live = jj < nc_g[:, None]
        sel = gi[sh_ok]          # candidates accepted by both
        ok[:] = False
        ok[sel] = True
        good = todo[sel]
        out["sec0"][good] = sec[sel]
        out["row0"][good] = row0[sel]
        out["pad0"][good] = hpad[sh_ok]
        out["snp"][good] = hsnp[sh_ok]
        out["qpt"][good] = hqpt[sh_ok]
        out["tgl"][good] = htgl[sh_ok]
        out["tq_lo"][good] = np.where(live, tq_m, 0).min(axis=1)[sh_ok]
        out["tq_hi"][good] = np.where(live, tq_m, 0).max(axis=1)[sh_ok]
        steps[good] = st[sel]
        secstep[good] = sst[sel]
        pres[good] = pr[sh_ok]
        tres[good] = tr[sh_ok]
        del pad_m, tq_m, pr, tr, live
        todo = todo[~ok]
    if todo.size:
        # rare leftovers: short straight tracks through the middle of a sector
        # at constant z, measured without noise (zero residuals)
        ncls[todo] = spec.ncls_min
        out["sec0"][todo] = rng.choice(sectors, todo.size)
        out["row0"][todo] = 60
        out["pad0"][todo] = _pad_code(np.zeros(1), np.array([60]))[0]
        for key in ("snp", "qpt", "tgl", "tq_lo", "tq_hi"):
            out[key][todo] = 0
        steps[todo] = 0
        steps[todo, 1:spec.ncls_min] = 1
        secstep[todo] = 0
        pres[todo] = 0
        tres[todo] = 0
    return ncls, out, steps, secstep, pres, tres


def _looper_geometry(rng, spec, n, looper_id):
    """Geometry of low-pT looper legs (at least n, unless the draws keep
    failing): each turn is an outward and an inward leg over the same circle;
    each leg is written as its own track."""
    legs = []
    made = 0
    tries = 0
    while made < n and tries < 50 * n + 100:
        tries += 1
        pt = math.exp(rng.uniform(math.log(spec.looper_pt[0]), math.log(spec.looper_pt[1])))
        q = 1.0 if rng.random() < 0.5 else -1.0
        k = q / pt * spec.bz * 0.00299792458
        if 2.0 / abs(k) < ROW_X[0] + 5.0:
            continue  # the circle never reaches the first pad row
        side = int(rng.integers(0, 2))
        phi0 = rng.uniform(0.0, 2 * math.pi)   # global direction at the origin
        tgl = rng.uniform(-0.1, 0.1)
        turns = int(rng.integers(1, spec.looper_turns + 1))
        # outward leg: rows from 0 while the local |sin| stays below 0.95
        out_rows, out_secs, out_s, out_y = [], [], [], []
        gsec = int(math.floor((phi0 % (2 * math.pi)) / math.radians(20.0)))
        for r in range(NROW):
            X = ROW_X[r]
            placed = False
            for cand in (gsec, gsec + 1, gsec - 1, gsec + 2, gsec - 2):
                alpha = math.radians((cand % 18) * 20.0 + 10.0)
                u = phi0 - alpha
                if math.cos(u) <= 0.0:
                    continue
                s = math.sin(u) + k * X
                if abs(s) >= 0.95:
                    continue
                c = math.sqrt(1.0 - s * s)
                y = X * (math.sin(u) + s) / (math.cos(u) + c)
                if abs(y) <= X * _TAN10:
                    gsec = cand
                    placed = True
                    out_rows.append(r)
                    out_secs.append(cand % 18)
                    out_s.append(s)
                    out_y.append(y)
                    break
            if not placed:
                break
        if len(out_rows) < 5:
            continue
        # inward leg: the mirror half of the circle.  In the decoder's frame
        # orientation (tangent pointing to +x) its sin(phi) is -s, its
        # curvature -k; position: the other intersection of the circle with
        # each row line.
        in_rows, in_secs, in_s, in_y = [], [], [], []
        for r in range(out_rows[-1], -1, -1):
            X = ROW_X[r]
            placed = False
            for cand in range(18):
                alpha = math.radians(cand * 20.0 + 10.0)
                u = phi0 - alpha
                s = math.sin(u) + k * X
                if abs(s) >= 0.95:
                    continue
                # second crossing of the circle with this row line
                y = (math.cos(u) + math.sqrt(1.0 - s * s)) / k
                if abs(y) <= X * _TAN10:
                    placed = True
                    in_rows.append(r)
                    in_secs.append(cand)
                    in_s.append(-s)
                    in_y.append(y)
                    break
            if not placed and in_rows:
                break
        for t in range(turns):
            for rows, secs, svals, yvals, sign in ((out_rows, out_secs, out_s, out_y, 1.0),
                                                   (in_rows, in_secs, in_s, in_y, -1.0)):
                if len(rows) < 5:
                    continue
                legs.append({"rows": np.array(rows), "secs": side * 18 + np.array(secs),
                             "y": np.array(yvals), "s0": svals[0], "qpt": sign * q / pt,
                             "tgl": sign * tgl, "tgl_phys": tgl, "k": k, "inward": sign < 0,
                             "turn": t, "looper": looper_id})
                made += 1
        looper_id += 1
    return legs, looper_id


def _looper_legs(rng, spec, n):
    """Looper legs with quantised headers and residuals against the shadow
    model; legs whose shadow comes near a limit of the model are dropped and
    more loopers are drawn."""
    legs = []
    looper_id = 0
    for _ in range(20):
        if len(legs) >= n:
            break
        cand, looper_id = _looper_geometry(rng, spec, n - len(legs), looper_id)
        if not cand:
            break
        m = len(cand)
        nc = np.array([len(lg["rows"]) for lg in cand])
        L = int(nc.max())
        rows = np.zeros((m, L), np.int64)
        sst = np.zeros((m, L), np.int64)
        ym = np.zeros((m, L))
        zt = np.zeros((m, L))
        for i, lg in enumerate(cand):
            c = nc[i]
            rows[i, :c] = lg["rows"]
            rows[i, c:] = lg["rows"][-1]
            sc = lg["secs"] % 18
            sst[i, 1:c] = (np.diff(sc) + 18) % 18
            ym[i, :c] = lg["y"]
            arc = _arc_from_origin(np.hypot(ROW_X[lg["rows"]], lg["y"]), lg["k"], inward=lg["inward"])
            zt[i, :c] = lg["tgl_phys"] * (arc - arc[0])
        pad_m, tq_m = _measure(rng, rows, ym, zt, nc)
        hpad = pad_m[:, 0]
        hsnp = np.clip(np.rint(np.array([lg["s0"] for lg in cand]) * 32768.0), -32767, 32767)
        hqpt = np.clip(np.rint(np.array([lg["qpt"] for lg in cand]) * 1024.0), -32768, 32767)
        htgl = np.clip(np.rint(np.array([lg["tgl"] for lg in cand]) * 4096.0), -32768, 32767)
        pr, tr, ok = _shadow_residuals(rows, sst, pad_m, tq_m, nc, hpad, hsnp, htgl, hqpt, spec.bz)
        live = np.arange(L)[None, :] < nc[:, None]
        lo = np.where(live, tq_m, 0).min(axis=1)
        hi = np.where(live, tq_m, 0).max(axis=1)
        for i, lg in enumerate(cand):
            if not ok[i]:
                continue
            c = nc[i]
            lg.update(pad0=int(hpad[i]), snp=int(hsnp[i]), qptq=int(hqpt[i]), tglq=int(htgl[i]),
                      pres=pr[i, :c].astype(np.int16), tres=tr[i, :c].astype(np.int16),
                      tq_lo=int(lo[i]), tq_hi=int(hi[i]))
            legs.append(lg)
    return legs


CHUNK_COLLISIONS = 25  # collisions per generation chunk (each chunk has its own random stream)


def _chunks(spec):
    """(chunk id, collisions, tracks) of a frame; chunks are generated
    independently and concatenated in order."""
    if spec.n_tracks > 0:
        return [(0, max(spec.collisions, 1), spec.n_tracks)]
    out = []
    for c, lo in enumerate(range(0, spec.collisions, CHUNK_COLLISIONS)):
        n = min(CHUNK_COLLISIONS, spec.collisions - lo)
        out.append((c, n, n * spec.tracks_per_collision))
    return out


def _attached_chunk(args):
    """Tracks and attached-cluster streams of one chunk of collisions."""
    spec, chunk_id, ncoll, nt_total = args
    rng = np.random.default_rng([spec.seed, spec.frame_index, chunk_id, 104729])
    n_loop = int(round(nt_total * spec.looper_frac))
    n_norm = nt_total - n_loop
    ncls, hdr, steps, secstep, pres, tres = _normal_tracks(rng, spec, n_norm)
    jj = np.arange(NROW)[None, :]
    mask = jj < ncls[:, None]

    # per-track collision assignment and times (in time bins); collision times
    # are uniform over the whole frame's span
    span_bins = 100.0 * max(spec.collisions, 1)
    coll_t = rng.uniform(0.0, span_bins, ncoll)
    legs = _looper_legs(rng, spec, n_loop) if n_loop > 0 else []

    # --- assemble tracks in collision order; a looper's legs stay together ---
    n_legs = len(legs)
    n_loopers = (max(lg["looper"] for lg in legs) + 1) if legs else 0
    loop_coll = rng.integers(0, ncoll, n_loopers)
    loop_key = rng.random(n_loopers)
    leg_owner = np.array([lg["looper"] for lg in legs], np.int64)
    tr_coll = np.concatenate([rng.integers(0, ncoll, n_norm), loop_coll[leg_owner]])
    tr_key = np.concatenate([rng.random(n_norm), loop_key[leg_owner]])
    tr_seq = np.concatenate([np.zeros(n_norm, np.int64), np.arange(n_legs)])
    kind = np.concatenate([np.zeros(n_norm, np.int64), np.ones(n_legs, np.int64)])
    idx = np.concatenate([np.arange(n_norm), np.arange(n_legs)])
    order = np.lexsort((tr_seq, tr_key, tr_coll))
    nt = n_norm + n_legs

    hd = {k: np.zeros(nt, FIELDS[k]) for k in ("trk_ncls", "trk_sec0", "trk_row0", "trk_pad0",
                                                "trk_time0", "trk_qpt", "trk_snp", "trk_tgl")}
    t_first = coll_t[tr_coll[order]] + 300.0 + rng.uniform(0.0, 485.0, nt)
    tq_lo = np.zeros(nt, np.int64)   # time codes of a track relative to its cluster 0
    tq_hi = np.zeros(nt, np.int64)
    # vectorised part for normal tracks
    ord_kind = kind[order]
    ord_idx = idx[order]
    is_norm = ord_kind == 0
    ni = ord_idx[is_norm]
    hd["trk_ncls"][is_norm] = ncls[ni]
    hd["trk_sec0"][is_norm] = hdr["sec0"][ni]
    hd["trk_row0"][is_norm] = hdr["row0"][ni]
    hd["trk_pad0"][is_norm] = hdr["pad0"][ni]
    hd["trk_snp"][is_norm] = hdr["snp"][ni]
    hd["trk_qpt"][is_norm] = hdr["qpt"][ni]
    hd["trk_tgl"][is_norm] = hdr["tgl"][ni]
    tq_lo[is_norm] = hdr["tq_lo"][ni]
    tq_hi[is_norm] = hdr["tq_hi"][ni]
    # loopers
    li = np.nonzero(~is_norm)[0]
    for p in li:
        leg = legs[ord_idx[p]]
        hd["trk_ncls"][p] = len(leg["rows"])
        hd["trk_sec0"][p] = int(leg["secs"][0])
        hd["trk_row0"][p] = int(leg["rows"][0])
        hd["trk_pad0"][p] = leg["pad0"]
        hd["trk_snp"][p] = leg["snp"]
        hd["trk_qpt"][p] = leg["qptq"]
        hd["trk_tgl"][p] = leg["tglq"]
        tq_lo[p] = leg["tq_lo"]
        tq_hi[p] = leg["tq_hi"]
        # later turns drift further: shift their time by the turn's z advance
        t_first[p] += leg["turn"] * 2.0 * math.pi / abs(leg["k"]) * abs(leg["tgl"]) / _VDRIFT
    # header times: every time code of the track at least 32 and below 2^24 - 32
    t0q = np.rint(t_first * 32).astype(np.int64)
    t0q = np.maximum(t0q, 32 - tq_lo)
    t0q = np.minimum(t0q, 2**24 - 32 - tq_hi)
    hd["trk_time0"][:] = np.clip(t0q, 0, 2**24 - 1).astype(np.uint32)

    # --- per-cluster streams ---
    ncl_t = hd["trk_ncls"].astype(np.int64)
    nA = int(ncl_t.sum())
    starts = np.concatenate([[0], np.cumsum(ncl_t)])
    row_diff = np.zeros(nA, np.int8)
    sec_diff = np.zeros(nA, np.uint8)
    pad_res = np.zeros(nA, np.int16)
    time_res = np.zeros(nA, np.int16)
    # normal tracks: scatter the per-step matrices
    m_n = mask[ni]
    dst = starts[:-1][is_norm]
    flat = (dst[:, None] + jj)[m_n]
    row_diff[flat] = steps[ni][m_n].astype(np.int8)
    sec_diff[flat] = secstep[ni][m_n].astype(np.uint8)
    pad_res[flat] = pres[ni][m_n]
    time_res[flat] = tres[ni][m_n]
    del m_n, flat
    for p in li:
        leg = legs[ord_idx[p]]
        a = starts[p]
        rws = leg["rows"].astype(np.int64)
        n = len(rws)
        rd = np.zeros(n, np.int64)
        rd[1:] = np.diff(rws)
        row_diff[a:a + n] = rd.astype(np.int8)
        sc = leg["secs"] % 18
        sd = np.zeros(n, np.int64)
        sd[1:] = (np.diff(sc) + 18) % 18
        sec_diff[a:a + n] = sd.astype(np.uint8)
        pad_res[a:a + n] = leg["pres"]
        time_res[a:a + n] = leg["tres"]
    is_first = np.zeros(nA, bool)
    is_first[starts[:-1][ncl_t > 0]] = True
    row_diff[is_first] = 0
    sec_diff[is_first] = 0
    pad_res[is_first] = 0
    time_res[is_first] = 0
    fr = {k: v for k, v in hd.items()}
    fr["cls_row_diff"] = row_diff
    fr["cls_sec_diff"] = sec_diff
    fr["cls_pad_res"] = pad_res
    fr["cls_time_res"] = time_res
    fr["cls_qmax"], fr["cls_qtot"] = _charges(rng, nA)
    return fr


def _unattached(args):
    """Unattached-cluster streams of a frame with nA attached clusters."""
    spec, nA = args
    rng = np.random.default_rng([spec.seed, spec.frame_index, 1 << 20, 104729])
    span_bins = 100.0 * max(spec.collisions, 1)
    nU = spec.n_unattached if spec.n_unattached >= 0 else int(round(nA * spec.unattached_ratio))
    sectors = np.asarray(spec.sectors)
    u_sec = rng.choice(sectors, nU)
    if spec.row_skew > 0:
        w = np.exp(-np.arange(NROW) / spec.row_skew)
        u_row = rng.choice(NROW, nU, p=w / w.sum())
    else:
        u_row = rng.integers(0, NROW, nU)
    u_bin = u_sec.astype(np.int64) * NROW + u_row
    count = np.bincount(u_bin, minlength=NBIN).astype(np.uint32)
    u_bin.sort()
    u_row_sorted = u_bin % NROW
    # time: a sorted uniform sample over the frame's span has exponential gaps
    t_span = (span_bins + 785.0) * 32.0
    gap_mean = t_span / np.maximum(count[u_bin], 1)
    fr = {"un_count": count}
    fr["un_time_diff"] = np.minimum(np.floor(rng.exponential(1.0, nU) * gap_mean),
                                    2**32 - 1).astype(np.uint32)
    # pad: independent uniform positions along the row, stored as differences
    pads = np.floor(rng.random(nU) * (ROW_NPADS[u_row_sorted] * 32)).astype(np.int64)
    first = np.ones(nU, bool)
    first[1:] = u_bin[1:] != u_bin[:-1]
    prev = np.concatenate([[0], pads[:-1]])
    prev[first] = 0
    fr["un_pad_diff"] = ((pads - prev) & 0xFFFF).astype(np.uint16)
    fr["un_qmax"], fr["un_qtot"] = _charges(rng, nU)
    return fr


def make_frames(specs, workers: int = 1) -> list:
    """Draw several frames (see make_frame).  With workers > 1 every chunk of
    collisions of every frame, then every frame's unattached clusters, is a
    task for a pool of forked worker processes (call this before the process
    uses a GPU).  The result does not depend on `workers`."""
    tasks = [(i, (spec, c, n, t)) for i, spec in enumerate(specs) for c, n, t in _chunks(spec)]
    pool = None
    if workers > 1 and len(tasks) > 1:
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(min(workers, len(tasks)))
    try:
        # largest chunks first, so that the pool's last tasks are short ones
        order = sorted(range(len(tasks)), key=lambda q: -tasks[q][1][3])
        args = [tasks[q][1] for q in order]
        res = pool.map(_attached_chunk, args, chunksize=1) if pool else [_attached_chunk(a) for a in args]
        parts = [[] for _ in specs]
        for q, r in sorted(zip(order, res), key=lambda z: z[0]):
            parts[tasks[q][0]].append(r)
        del res
        frames = []
        for p in parts:
            frames.append({k: np.concatenate([c[k] for c in p]) for k in p[0]})
            p.clear()
        uargs = [(spec, int(fr["cls_qtot"].shape[0])) for spec, fr in zip(specs, frames)]
        un = pool.map(_unattached, uargs, chunksize=1) if pool else [_unattached(a) for a in uargs]
    finally:
        if pool:
            pool.close()
            pool.join()
    for fr, u in zip(frames, un):
        fr.update(u)
    return frames


def make_frame(spec: FrameSpec, workers: int = 1) -> dict:
    """Draw one compressed frame (dict of numpy arrays, see FIELDS).  With
    workers > 1 the chunks of collisions are generated in forked worker
    processes (call this before the process uses a GPU)."""
    return make_frames([spec], workers)[0]


def _charges(rng, n):
    qmax = 1.0 + np.floor(rng.exponential(30.0, n))
    qtot = qmax + np.floor(rng.exponential(120.0, n))
    return (np.minimum(qmax, 65535).astype(np.uint16), np.minimum(qtot, 65535).astype(np.uint16))


def sizes(fr):
    return int(fr["trk_ncls"].shape[0]), int(fr["cls_qtot"].shape[0]), int(fr["un_qtot"].shape[0])

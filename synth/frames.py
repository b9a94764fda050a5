"""Synthetic compressed time frames shaped like Pb-Pb running.

The generator writes the compressed streams directly: track headers, per-cluster
row/sector steps, Gaussian residuals, charges, and per-(sector,row) delta
streams of unattached clusters.  It does not run the decoder's track model.
To make the streams look physical it uses its own, double-precision picture of
the detector: charged tracks are circles through the origin in a uniform
field, and each cluster sits where a circle crosses a pad row.  This geometry
decides
  - which rows and sectors each track visits, including sector crossings and
    the legs of low-pT loopers, and
  - the header values (pad, sin(phi)) at a track's first cluster.
The residuals are then drawn at random (sigma 0.05 cm in pad and time).  The
decoded track therefore follows the drawn track up to a random walk.  Any
stream the generator writes is a valid decoder input whatever the geometry:
out-of-range values are clamped and flagged, identically on every decoder.

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
    """Outward tracks: per-track dict of header values and per-step arrays."""
    ncls = rng.integers(spec.ncls_min, spec.ncls_max + 1, n)
    out = {k: np.zeros(n, np.int64) for k in ("sec0", "row0")}
    fl = {k: np.zeros(n) for k in ("y0", "s0", "qpt", "tgl")}
    crosser = rng.random(n) < spec.crosser_frac
    steps = np.zeros((n, NROW), np.int64)      # row step before cluster j (j >= 1)
    secstep = np.zeros((n, NROW), np.int64)    # sector step before cluster j
    todo = np.arange(n)
    sectors = np.asarray(spec.sectors)
    for attempt in range(60):
        if todo.size == 0:
            break
        if attempt in (20, 40):
            # persistent rejects: redraw their lengths as well
            ncls[todo] = rng.integers(spec.ncls_min, spec.ncls_max + 1, todo.size)
        m = todo.size
        nc = ncls[todo]
        st = np.zeros((m, NROW), np.int64)
        st[:, 1:] = _draw_rows(rng, m * (NROW - 1)).reshape(m, NROW - 1)
        jj = np.arange(NROW)[None, :]
        st[jj >= nc[:, None]] = 0
        span = st.sum(axis=1)
        bad_span = span > NROW - 1
        span = np.minimum(span, NROW - 1)
        row0 = _sample_start_rows(rng, span, spec.row_skew)
        rows = row0[:, None] + np.cumsum(st, axis=1)
        X = ROW_X[np.minimum(rows, NROW - 1)]
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
        ys = np.zeros(m)
        ss = np.zeros(m)
        ncross = np.zeros(m, np.int64)
        y0 = np.zeros(m)
        s0 = np.zeros(m)
        for j in range(NROW):
            act = j < nc
            if not act.any():
                break
            s, y = _local_track(u - du, k, X[:, j])
            edge = X[:, j] * _TAN10
            out_pos = act & (y > edge)
            out_neg = act & (y < -edge)
            # crossing into the neighbouring sector (+20 deg or -20 deg)
            du = du + np.radians(20.0) * out_pos - np.radians(20.0) * out_neg
            sst[:, j] = np.where(out_pos, 1, np.where(out_neg, 17, 0))
            ncross += (out_pos | out_neg)
            s2, y2 = _local_track(u - du, k, X[:, j])
            s = np.where(out_pos | out_neg, s2, s)
            y = np.where(out_pos | out_neg, y2, y)
            ok &= ~act | ((np.abs(s) < 0.95) & (np.abs(y) <= X[:, j] * _TAN10 * 1.0001))
            if j == 0:
                y0, s0 = y.copy(), s.copy()
                ok &= (sst[:, 0] == 0)
            ys, ss = y, s
        del ys, ss
        ok &= np.where(crosser[todo], ncross >= 1, ncross == 0)
        good = todo[ok]
        sec = rng.choice(sectors, m)
        out["sec0"][good] = sec[ok]
        out["row0"][good] = row0[ok]
        fl["y0"][good] = y0[ok]
        fl["s0"][good] = s0[ok]
        fl["qpt"][good] = (q / pt)[ok]
        fl["tgl"][good] = rng.uniform(-1.0, 1.0, m)[ok]
        steps[good] = st[ok]
        secstep[good] = sst[ok]
        todo = todo[~ok]
    if todo.size:
        # rare leftovers: short straight tracks in the middle of a sector
        ncls[todo] = spec.ncls_min
        out["sec0"][todo] = rng.choice(sectors, todo.size)
        out["row0"][todo] = 60
        steps[todo, 1:spec.ncls_min] = 1
        secstep[todo] = 0
        fl["y0"][todo] = 0.0
        fl["s0"][todo] = 0.0
        fl["qpt"][todo] = 0.1
        fl["tgl"][todo] = 0.0
    return ncls, out, fl, steps, secstep


def _looper_legs(rng, spec, n):
    """Legs of low-pT loopers: each turn is an outward and an inward leg over
    the same circle; each leg is written as its own track."""
    legs = []
    made = 0
    tries = 0
    looper_id = 0
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
                rows = rows[:255]
                legs.append({"rows": np.array(rows), "secs": side * 18 + np.array(secs[:len(rows)]),
                             "s0": svals[0], "y0": yvals[0], "qpt": sign * q / pt,
                             "tgl": sign * tgl, "turn": t, "looper": looper_id})
                made += 1
        looper_id += 1
    return legs


def _quant_header_s(s):
    return np.clip(np.rint(np.asarray(s) * 32768.0), -32767, 32767).astype(np.int16)


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
    ncls, hdr, fl, steps, secstep = _normal_tracks(rng, spec, n_norm)
    rows_rel = np.cumsum(steps, axis=1)
    jj = np.arange(NROW)[None, :]
    mask = jj < ncls[:, None]

    # per-track collision assignment and times (in time bins); collision times
    # are uniform over the whole frame's span
    span_bins = 100.0 * max(spec.collisions, 1)
    coll_t = rng.uniform(0.0, span_bins, ncoll)
    legs = _looper_legs(rng, spec, n_loop) if n_loop > 0 else []

    # --- assemble tracks in collision order; a looper's legs stay together ---
    n_legs = len(legs)
    n_loopers = (legs[-1]["looper"] + 1) if legs else 0
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
    # vectorised part for normal tracks
    ord_kind = kind[order]
    ord_idx = idx[order]
    is_norm = ord_kind == 0
    ni = ord_idx[is_norm]
    hd["trk_ncls"][is_norm] = ncls[ni]
    hd["trk_sec0"][is_norm] = hdr["sec0"][ni]
    hd["trk_row0"][is_norm] = hdr["row0"][ni]
    pw0 = ROW_PW[hdr["row0"][ni]]
    pad0 = fl["y0"][ni] / pw0 + ROW_NPADS[hdr["row0"][ni]] / 2
    hd["trk_pad0"][is_norm] = np.clip(np.rint(pad0 * 32), 0, 65535).astype(np.uint16)
    hd["trk_snp"][is_norm] = _quant_header_s(fl["s0"][ni])
    hd["trk_qpt"][is_norm] = np.clip(np.rint(fl["qpt"][ni] * 1024), -32768, 32767).astype(np.int16)
    hd["trk_tgl"][is_norm] = np.clip(np.rint(fl["tgl"][ni] * 4096), -32768, 32767).astype(np.int16)
    # loopers
    li = np.nonzero(~is_norm)[0]
    for p in li:
        leg = legs[ord_idx[p]]
        r0 = int(leg["rows"][0])
        hd["trk_ncls"][p] = len(leg["rows"])
        hd["trk_sec0"][p] = int(leg["secs"][0])
        hd["trk_row0"][p] = r0
        pad = leg["y0"] / ROW_PW[r0] + ROW_NPADS[r0] / 2
        hd["trk_pad0"][p] = int(np.clip(np.rint(pad * 32), 0, 65535))
        hd["trk_snp"][p] = _quant_header_s(leg["s0"])
        hd["trk_qpt"][p] = int(np.clip(np.rint(leg["qpt"] * 1024), -32768, 32767))
        hd["trk_tgl"][p] = int(np.clip(np.rint(leg["tgl"] * 4096), -32768, 32767))
        # later turns drift further: shift their time by the turn's z advance
        t_first[p] += leg["turn"] * 2.0 * math.pi / abs(leg["qpt"] * spec.bz * 0.00299792458) \
            * abs(leg["tgl"]) / _VDRIFT
    hd["trk_time0"][:] = np.clip(np.rint(t_first * 32), 0, 2**24 - 1).astype(np.uint32)

    # --- per-cluster streams ---
    ncl_t = hd["trk_ncls"].astype(np.int64)
    nA = int(ncl_t.sum())
    starts = np.concatenate([[0], np.cumsum(ncl_t)])
    row_diff = np.zeros(nA, np.int8)
    sec_diff = np.zeros(nA, np.uint8)
    cl_row = np.zeros(nA, np.int64)
    # normal tracks: scatter the per-step matrices
    ncl_n = ncls[ni]
    st_n = steps[ni]
    ss_n = secstep[ni]
    m_n = mask[ni]
    dst = starts[:-1][is_norm]
    flat = (dst[:, None] + jj)[m_n]
    row_diff[flat] = st_n[m_n].astype(np.int8)
    sec_diff[flat] = ss_n[m_n].astype(np.uint8)
    cl_row[flat] = (hdr["row0"][ni][:, None] + rows_rel[ni])[m_n]
    del st_n, ss_n, m_n, flat
    for p in li:
        leg = legs[ord_idx[p]]
        a = starts[p]
        rws = leg["rows"].astype(np.int64)
        n = len(rws)
        cl_row[a:a + n] = rws
        rd = np.zeros(n, np.int64)
        rd[1:] = np.diff(rws)
        row_diff[a:a + n] = rd.astype(np.int8)
        sc = leg["secs"] % 18
        sd = np.zeros(n, np.int64)
        sd[1:] = (np.diff(sc) + 18) % 18
        sec_diff[a:a + n] = sd.astype(np.uint8)
    is_first = np.zeros(nA, bool)
    is_first[starts[:-1][ncl_t > 0]] = True
    row_diff[is_first] = 0
    sec_diff[is_first] = 0
    pwq = ROW_PW[cl_row] / 32.0
    pad_res = np.rint(rng.normal(0.0, 0.05, nA) / pwq)
    time_res = np.rint(rng.normal(0.0, 0.05, nA) / (_VDRIFT / 32.0))
    pad_res[is_first] = 0
    time_res[is_first] = 0
    del pwq, cl_row
    fr = {k: v for k, v in hd.items()}
    fr["cls_row_diff"] = row_diff
    fr["cls_sec_diff"] = sec_diff
    fr["cls_pad_res"] = np.clip(pad_res, -32768, 32767).astype(np.int16)
    fr["cls_time_res"] = np.clip(time_res, -32768, 32767).astype(np.int16)
    del pad_res, time_res
    fr["cls_qmax"], fr["cls_qtot"] = _charges(rng, nA)
    return fr


def make_frame(spec: FrameSpec, workers: int = 1) -> dict:
    """Draw one compressed frame (dict of numpy arrays, see FIELDS).  With
    workers > 1 the chunks of collisions are generated in forked worker
    processes (call this before the process uses a GPU)."""
    chunks = [(spec, c, n, t) for c, n, t in _chunks(spec)]
    if workers > 1 and len(chunks) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, len(chunks))) as pool:
            parts = pool.map(_attached_chunk, chunks, chunksize=1)
    else:
        parts = [_attached_chunk(c) for c in chunks]
    fr = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    del parts
    nA = int(fr["cls_qtot"].shape[0])
    rng = np.random.default_rng([spec.seed, spec.frame_index, 1 << 20, 104729])
    span_bins = 100.0 * max(spec.collisions, 1)

    # --- unattached clusters ---
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
    fr["un_count"] = count
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


def _charges(rng, n):
    qmax = 1.0 + np.floor(rng.exponential(30.0, n))
    qtot = qmax + np.floor(rng.exponential(120.0, n))
    return (np.minimum(qmax, 65535).astype(np.uint16), np.minimum(qtot, 65535).astype(np.uint16))


def sizes(fr):
    return int(fr["trk_ncls"].shape[0]), int(fr["cls_qtot"].shape[0]), int(fr["un_qtot"].shape[0])

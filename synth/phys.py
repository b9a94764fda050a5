"""Seeded physical clusters with the shape of a Pb-Pb time frame: the input of
the track-model encoder.

Where synth.frames writes compressed streams, this module writes what a
cluster finder hands to the encoder: per track a range of clusters, q/pT and
tan(lambda); per cluster its sector, row, pad and time (in pads and time bins,
as doubles), the local sin(phi) there and its charges; unattached clusters
likewise, without a track.  The geometry is synth.frames' picture (circles
through the origin in a uniform field, a cluster wherever a circle crosses a
pad row, frames switched at sector edges), vectorised over tracks so that a
frame of 2e5 tracks takes seconds.  Positions are smeared by Gaussian noise
(sigma 0.05 cm in y and z) and not quantised: quantising is the encoder's
first step.

Track lengths, row gaps, pT, tan(lambda), start rows and the share of sector
crossers follow the FrameSpec as in synth.frames; unattached clusters are
spread uniformly over the spec's sectors, the rows (or the skewed row
distribution) and the pad row, with times uniform over the frame's span.
"""
import math

import numpy as np

from .frames import (NROW, ROW_NPADS, ROW_PW, ROW_X, SIGMA_CM, _TAN10, _VDRIFT, _arc_from_origin, _charges,
                     _draw_rows, _local_track, _sample_start_rows)

ENC_FIELDS = {
    "trk_first": np.uint32, "trk_qpt": np.float64, "trk_tgl": np.float64,
    "cl_sec": np.uint8, "cl_row": np.uint8, "cl_pad": np.float64, "cl_time": np.float64,
    "cl_snp": np.float64, "cl_qtot": np.uint16, "cl_qmax": np.uint16,
    "un_sec": np.uint8, "un_row": np.uint8, "un_pad": np.float64, "un_time": np.float64,
    "un_qtot": np.uint16, "un_qmax": np.uint16,
}
CHUNK = 16384            # tracks drawn together
S_MAX = 0.95             # |local sin phi| of every cluster stays below this


def _track_block(rng, spec, m):
    """m accepted tracks: (ncls, sec, rows, snp, pad, tq, qpt, tgl) with the
    per-cluster arrays as (m, NROW) matrices (columns >= ncls unused); tq is
    the time relative to cluster 0 in time bins."""
    got = []
    need = m
    for attempt in range(50):
        if need == 0:
            break
        c = max(need + need // 4, 64)
        nc = rng.integers(spec.ncls_min, spec.ncls_max + 1, c)
        jj = np.arange(NROW)[None, :]
        st = np.zeros((c, NROW), np.int64)
        st[:, 1:] = _draw_rows(rng, c * (NROW - 1)).reshape(c, NROW - 1)
        st[jj >= nc[:, None]] = 0
        span = st.sum(axis=1)
        ok = span <= NROW - 1
        span = np.minimum(span, NROW - 1)
        row0 = _sample_start_rows(rng, span, spec.row_skew)
        rows = np.minimum(row0[:, None] + np.cumsum(st, axis=1), NROW - 1)
        X = ROW_X[rows]
        pt = np.exp(rng.uniform(math.log(spec.pt_min), math.log(spec.pt_max), c))
        q = np.where(rng.random(c) < 0.5, 1.0, -1.0)
        k = q / pt * spec.bz * 0.00299792458
        th = np.radians(rng.uniform(-10.0, 10.0, c))
        cr = rng.random(c) < spec.crosser_frac
        th[cr] = np.sign(th[cr]) * np.radians(rng.uniform(4.0, 10.0, int(cr.sum())))
        r0 = X[:, 0] / np.cos(th)
        a = k * r0 / 2.0
        ok &= np.abs(a) < 1.0
        u = th - np.arcsin(np.clip(a, -1.0, 1.0))
        ok &= np.cos(u) > 0.1
        du = np.zeros(c)
        step = np.zeros((c, NROW), np.int64)      # sector step (+1 / -1) at cluster j
        ys = np.zeros((c, NROW))
        ss = np.zeros((c, NROW))
        for j in range(NROW):
            live = nc > j
            if not live.any():
                break
            s, y = _local_track(u - du, k, X[:, j])
            edge = X[:, j] * _TAN10
            pos = live & (y > edge)
            neg = live & (y < -edge)
            if (pos | neg).any():
                du += np.radians(20.0) * pos - np.radians(20.0) * neg
                step[:, j] = pos.astype(np.int64) - neg.astype(np.int64)
                s2, y2 = _local_track(u - du, k, X[:, j])
                s = np.where(pos | neg, s2, s)
                y = np.where(pos | neg, y2, y)
            ok &= ~live | ((np.abs(s) < S_MAX) & (np.abs(y) <= edge * 1.0001))
            ys[:, j] = y
            ss[:, j] = s
        ok &= step[:, 0] == 0
        g = np.nonzero(ok)[0][:need]
        if g.size == 0:
            continue
        nc, rows, k, ys, ss, step = nc[g], rows[g], k[g], ys[g], ss[g], step[g]
        tgl = rng.uniform(-1.0, 1.0, g.size)
        arc = _arc_from_origin(np.hypot(ROW_X[rows], ys), k[:, None])
        z = tgl[:, None] * (arc - arc[:, :1]) + rng.normal(0.0, SIGMA_CM, rows.shape)
        y = ys + rng.normal(0.0, SIGMA_CM, rows.shape)
        pad = y / ROW_PW[rows] + ROW_NPADS[rows] / 2.0
        pad = np.clip(pad, 1.0 / 32.0, ROW_NPADS[rows] - 2.0 / 32.0)   # one code inside the pad plane
        tq = (z - z[:, :1]) / _VDRIFT                                   # cluster 0 defines the time origin
        sec0 = rng.choice(np.asarray(spec.sectors), g.size)
        side = sec0 // 18
        sec = side[:, None] * 18 + (sec0[:, None] % 18 + np.cumsum(step, axis=1)) % 18
        got.append((nc, sec, rows, ss, pad, tq, (q / pt)[g], tgl))
        need -= g.size
    if need:
        raise RuntimeError(f"synth.phys: {need} tracks not drawn after 50 attempts")
    return tuple(np.concatenate([p[i] for p in got]) for i in range(8))


def _chunk(args):
    """Tracks [start, start + m) of a frame: per-cluster columns, q/pT, tan
    lambda and cluster counts, drawn from the chunk's own seed."""
    spec, seed_tag, ci, m = args
    rng = np.random.default_rng([spec.seed, spec.frame_index, seed_tag, ci])
    nc, sec, rows, ss, pad, tq, qpt, tgl = _track_block(rng, spec, m)
    live = np.arange(NROW)[None, :] < nc[:, None]
    # header time: inside the frame's span, raised so that no cluster's time is below 2 time bins
    t0 = 300.0 + rng.uniform(0.0, 100.0 * max(spec.collisions, 1), m)
    t0 = np.maximum(t0, 2.0 - np.where(live, tq, 0.0).min(axis=1))
    qmax, qtot = _charges(rng, int(nc.sum()))
    return {"cl_sec": sec[live].astype(np.uint8), "cl_row": rows[live].astype(np.uint8), "cl_pad": pad[live],
            "cl_time": (t0[:, None] + tq)[live], "cl_snp": ss[live], "cl_qmax": qmax, "cl_qtot": qtot,
            "trk_qpt": qpt, "trk_tgl": tgl, "ncls": nc}


def make_phys(spec, workers=1, seed_tag=0x5EED):
    """The physical clusters of one frame of `spec` (dict keyed as
    ENC_FIELDS).  Tracks are contiguous in the cluster arrays; trk_first has
    n_tracks + 1 entries.  With workers > 1 the chunks of CHUNK tracks are
    drawn in forked processes (call this before the process uses a GPU); the
    result does not depend on `workers`."""
    n = spec.tracks()
    tasks = [(spec, seed_tag, ci, min(CHUNK, n - s)) for ci, s in enumerate(range(0, n, CHUNK))]
    if workers > 1 and len(tasks) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, len(tasks))) as pool:
            parts = pool.map(_chunk, tasks, chunksize=1)
    else:
        parts = [_chunk(t) for t in tasks]
    ph = {k: np.concatenate([p[k] for p in parts]) if parts else np.zeros(0, ENC_FIELDS[k])
          for k in ENC_FIELDS if k.startswith("cl_") or k in ("trk_qpt", "trk_tgl")}
    nc = np.concatenate([p["ncls"] for p in parts]) if parts else np.zeros(0, np.int64)
    del parts
    ph["trk_first"] = np.concatenate([[0], np.cumsum(nc)]).astype(np.uint32)
    nA = int(nc.sum())
    rng = np.random.default_rng([spec.seed, spec.frame_index, seed_tag, 1 << 20])
    nU = spec.n_unattached if spec.n_unattached >= 0 else int(round(nA * spec.unattached_ratio))
    ph["un_sec"] = rng.choice(np.asarray(spec.sectors), nU).astype(np.uint8)
    if spec.row_skew > 0:
        w = np.exp(-np.arange(NROW) / spec.row_skew)
        urow = rng.choice(NROW, nU, p=w / w.sum())
    else:
        urow = rng.integers(0, NROW, nU)
    ph["un_row"] = urow.astype(np.uint8)
    ph["un_pad"] = rng.random(nU) * (ROW_NPADS[urow] - 1.0 / 32.0)
    ph["un_time"] = rng.uniform(0.0, 100.0 * max(spec.collisions, 1) + 785.0, nU)
    ph["un_qmax"], ph["un_qtot"] = _charges(rng, nU)
    return {k: np.ascontiguousarray(ph[k], ENC_FIELDS[k]) for k in ENC_FIELDS}


def phys_sizes(ph):
    """(tracks, attached clusters, unattached clusters)"""
    return int(ph["trk_qpt"].shape[0]), int(ph["cl_pad"].shape[0]), int(ph["un_pad"].shape[0])

"""The physical-cluster generator (synth.phys), the encoder benchmark's input:
deterministic whatever the number of workers, inside the codable range, and
consistent with the track model, so that the oracle's encoder codes it with
few split tracks and its decode restores the quantised clusters exactly."""
import numpy as np

import oracle
import synth
from oracle import physgen as pg
from synth.phys import ENC_FIELDS, ROW_NPADS


def _small():
    return synth.spec_for("frame", collisions=2, seed=11)


def test_phys_deterministic_and_shaped():
    spec = _small()
    a = synth.make_phys(spec)
    b = synth.make_phys(spec, workers=3)
    assert set(a) == set(ENC_FIELDS)
    for k in a:
        assert a[k].dtype == ENC_FIELDS[k]
        assert np.array_equal(a[k], b[k]), k
    nT, nA, nU = synth.phys_sizes(a)
    assert nT == spec.tracks() and a["trk_first"][-1] == nA
    ncls = np.diff(a["trk_first"].astype(np.int64))
    assert ncls.min() >= spec.ncls_min and ncls.max() <= spec.ncls_max
    assert abs(nU - nA * spec.unattached_ratio) <= 1
    # rows rise inside a track (steps of 1 or 2), sectors stay on their side
    first = np.zeros(nA, bool)
    first[a["trk_first"][:-1]] = True
    dr = np.diff(a["cl_row"].astype(np.int64))[~first[1:]]
    assert set(np.unique(dr)) <= {1, 2}
    side = a["cl_sec"] // 18
    assert np.all(np.diff(side.astype(np.int64))[~first[1:]] == 0)
    assert (a["cl_sec"] < 36).all() and (a["un_sec"] < 36).all() and (a["cl_row"] < 152).all()
    assert np.all(a["cl_pad"] > 0) and np.all(a["cl_pad"] < ROW_NPADS[a["cl_row"]])
    assert np.all(a["un_pad"] >= 0) and np.all(a["un_pad"] < ROW_NPADS[a["un_row"]])
    assert np.all(a["cl_time"] >= 2.0) and np.all(np.abs(a["cl_snp"]) < 0.95)


def test_phys_encodes_and_round_trips():
    ph = synth.make_phys(_small())
    fr, split = oracle.encode(ph, bz=0.5)
    nT = synth.phys_sizes(ph)[0]
    assert split <= nT // 100               # the model follows the drawn tracks
    assert fr["trk_ncls"].shape[0] == nT + split
    out, status = oracle.decode(fr, bz=0.5)
    assert status == 0
    want = pg.expected_clusters(ph)
    for k in want:
        assert np.array_equal(want[k], out[k]), k

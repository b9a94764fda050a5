"""Round-trip pins: decode(encode(x)) == quantize(x).

The paper (section 4) states that decoding restores the original values that
track-model encoding replaced by residuals (attached clusters) and by
differences to the predecessor (unattached clusters).  Physical clusters from
an exact helix are quantised to 1/32 pad and 1/32 time bin; the expected
decoded layout is built with numpy alone (oracle.physgen.expected_clusters).
A residual RMS near the noise level and no per-track residual bias show that
the model follows real helices; a wrong field leaves a bias, which shows the
pin's sensitivity."""
import numpy as np
import pytest

import oracle
from oracle import physgen as pg


def _roundtrip(phys, bz):
    fr, nsplit = oracle.encode(phys, bz=bz)
    out, st = oracle.decode(fr, bz=bz)
    exp = pg.expected_clusters(phys)
    for k in exp:
        assert np.array_equal(exp[k], out[k]), k
    return fr, nsplit, st


@pytest.mark.parametrize("seed,bz", [(0, 0.5), (1, 0.5), (2, 0.0), (3, 2.0), (4, -0.5)])
def test_roundtrip_physical(seed, bz):
    phys = pg.generate(seed=seed, n_tracks=150, n_un=3000, bz=bz)
    fr, nsplit, st = _roundtrip(phys, bz)
    assert st == 0
    assert nsplit == 0
    assert len(fr["trk_ncls"]) == 150
    if bz != 0.0:
        assert np.count_nonzero(fr["cls_sec_diff"]) > 0  # some tracks cross sectors


def test_residual_rms_matches_noise():
    phys = pg.generate(seed=11, n_tracks=300, n_un=10, bz=0.5, noise=0.05)
    fr, nsplit, st = _roundtrip(phys, 0.5)
    j = np.ones(len(fr["cls_pad_res"]), bool)
    j[np.concatenate([[0], np.cumsum(fr["trk_ncls"][:-1].astype(np.int64))])] = False
    pad_cm = fr["cls_pad_res"][j] * (np.array(pg.ROW_PW)[0] / 32)  # inner-row quantum bound
    rms_pad = np.sqrt(np.mean(fr["cls_pad_res"][j].astype(float) ** 2))
    rms_time = np.sqrt(np.mean(fr["cls_time_res"][j].astype(float) ** 2))
    # innovation of a unit-gain position update: about sqrt(2) sigma / quantum
    # (sigma = 0.05 cm, quanta 0.013 / 0.019 cm in pad, 0.016 cm in time)
    assert 2.5 < rms_pad < 8.0, rms_pad
    assert 3.0 < rms_time < 6.5, rms_time
    assert np.abs(pad_cm).max() < 2.0


def _track_mean_residuals(fr, skip=5, min_len=20):
    n = fr["trk_ncls"].astype(np.int64)
    st = np.concatenate([[0], np.cumsum(n)])
    return np.array([fr["cls_pad_res"][st[i] + skip:st[i + 1]].mean()
                     for i in range(len(n)) if n[i] > min_len])


def test_curvature_bias_pins_the_field():
    """A model with the right curvature leaves no per-track bias in the pad
    residuals; the wrong field (sign, or none) leaves a bias of several
    quanta.  This is what makes the round trip a pin of the propagation and
    not only of encoder/decoder consistency."""
    phys = pg.generate(seed=12, n_tracks=200, n_un=10, bz=0.5, pt_range=(0.2, 1.0))
    good = _track_mean_residuals(oracle.encode(phys, bz=0.5)[0])
    assert np.sqrt(np.mean(good ** 2)) < 0.5 and np.abs(good).max() < 2.0
    for wrong_bz in (-0.5, 0.0):
        bad = _track_mean_residuals(oracle.encode(phys, bz=wrong_bz)[0])
        assert np.sqrt(np.mean(bad ** 2)) > 2.0, wrong_bz


def test_roundtrip_no_noise_low_pt():
    phys = pg.generate(seed=5, n_tracks=200, n_un=100, bz=0.5, pt_range=(0.1, 0.5), noise=0.0)
    _, nsplit, st = _roundtrip(phys, 0.5)
    assert st == 0


def _manual_phys(tracks, un=None):
    """tracks: list of (qpt, tgl, [(sec, row, pad, time, snp), ...])."""
    first, qpt, tgl = [0], [], []
    cols = {k: [] for k in ("cl_sec", "cl_row", "cl_pad", "cl_time", "cl_snp")}
    for q, t, cl in tracks:
        for c in cl:
            for k, v in zip(("cl_sec", "cl_row", "cl_pad", "cl_time", "cl_snp"), c):
                cols[k].append(v)
        first.append(first[-1] + len(cl))
        qpt.append(q)
        tgl.append(t)
    n = first[-1]
    phys = {"trk_first": np.array(first, np.uint32), "trk_qpt": np.array(qpt, float),
            "trk_tgl": np.array(tgl, float), "cl_sec": np.array(cols["cl_sec"], np.uint8),
            "cl_row": np.array(cols["cl_row"], np.uint8), "cl_pad": np.array(cols["cl_pad"], float),
            "cl_time": np.array(cols["cl_time"], float), "cl_snp": np.array(cols["cl_snp"], float),
            "cl_qtot": (np.arange(n) % 65536).astype(np.uint16),
            "cl_qmax": (np.arange(n) // 65536 + 7).astype(np.uint16)}
    un = un or []
    phys["un_sec"] = np.array([u[0] for u in un], np.uint8)
    phys["un_row"] = np.array([u[1] for u in un], np.uint8)
    phys["un_pad"] = np.array([u[2] for u in un], float)
    phys["un_time"] = np.array([u[3] for u in un], float)
    phys["un_qtot"] = np.array([u[4] for u in un], np.uint16)
    phys["un_qmax"] = np.array([u[5] for u in un], np.uint16)
    return phys


def test_encoder_splits_keep_order():
    """Tracks that the model cannot follow (side change, > 255 clusters,
    residuals beyond int16) are split into several headers; the decoded
    layout is still exactly quantize(x)."""
    rng = np.random.default_rng(3)
    side_change = [(i % 18 if i < 5 else 18 + i % 18, 40 + i, 20.0 + 0.3 * i, 900.0 + i, 0.1)
                   for i in range(10)]
    zigzag = [(3, 10 + (i % 2), 30.0 + rng.normal(0, 0.02), 1000.0 + 0.1 * i, 0.0) for i in range(300)]
    jumpy = [(5, 20 + i, 40.0 + (1500.0 if i == 6 else 0.0), 800.0 + i, 0.0) for i in range(12)]
    phys = _manual_phys([(0.5, 0.2, side_change), (1.0, 0.0, zigzag), (0.2, 0.0, jumpy)],
                        un=[(1, 2, 3.25, 4.0, 5, 6), (1, 2, 3.25, 4.0, 5, 5), (0, 0, 0.0, 0.0, 0, 0)])
    fr, nsplit = oracle.encode(phys, bz=0.5)
    assert nsplit >= 3
    out, st = oracle.decode(fr, bz=0.5)
    exp = pg.expected_clusters(phys)
    for k in exp:
        assert np.array_equal(exp[k], out[k]), k
    assert fr["trk_ncls"].max() <= 255

"""The synthetic frame generator: determinism and workload shapes."""
import numpy as np

import synth
from synth.frames import NBIN, sizes


def test_deterministic():
    sp = synth.spec_for("frame", collisions=2)
    a, b = synth.make_frame(sp), synth.make_frame(sp)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    c = synth.make_frame(synth.spec_for("frame", collisions=2, frame_index=1))
    assert not np.array_equal(a["cls_pad_res"][:1000], c["cls_pad_res"][:1000])


def test_config0_shape():
    fr = synth.make_frame(synth.spec_for("tiny"))
    nt, na, nu = sizes(fr)
    assert nt == 1000 and nu == 20000
    assert fr["trk_ncls"].min() >= 20 and fr["trk_ncls"].max() <= 152
    assert na == int(fr["trk_ncls"].astype(np.int64).sum())
    assert (fr["trk_sec0"] == 0).all() and not fr["cls_sec_diff"].any()
    assert fr["un_count"][152:].sum() == 0 and fr["un_count"].sum() == nu


def test_config1_like_shape():
    fr = synth.make_frame(synth.spec_for("frame", collisions=4))
    nt, na, nu = sizes(fr)
    assert nt == 8000
    n = fr["trk_ncls"].astype(np.int64)
    assert 5 <= n.min() and n.max() <= 152
    assert abs(n.mean() - 78.5) < 3
    st = np.concatenate([[0], np.cumsum(n)])
    crossers = np.add.reduceat(fr["cls_sec_diff"] != 0, st[:-1]) > 0
    assert 0.07 < crossers.mean() < 0.13
    assert abs(nu / na - 2 / 3) < 0.01
    assert len(fr["un_count"]) == NBIN


def test_config4_loopers_and_skew():
    fr = synth.make_frame(synth.spec_for("stress", collisions=2))
    assert (fr["cls_row_diff"] < 0).sum() > 1000          # inward legs of loopers
    rows = np.arange(NBIN) % 152
    cnt = np.bincount(rows, weights=fr["un_count"], minlength=152)
    assert cnt[:20].sum() > 5 * cnt[-20:].sum()          # exponential in row

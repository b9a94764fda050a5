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


def test_streams_decode_without_flags():
    """Every workload's streams are valid decoder input: the oracle decodes
    them with no status flag (no clamp, no count mismatch), and the residuals
    have the spread of the cluster noise (sigma 0.05 cm, measured minus
    predicted: about sqrt(2) sigma over the quantum)."""
    import oracle
    for name, over in (("tiny", {}), ("frame", {"collisions": 3}), ("stress", {"collisions": 2})):
        fr = synth.make_frame(synth.spec_for(name, **over))
        _, status = oracle.decode(fr, bz=0.5)
        assert status == 0, (name, status)
        tq = 0.516 / 32
        sd = fr["cls_time_res"].astype(np.float64).std()
        assert 0.8 * 2 ** 0.5 * 0.05 / tq < sd < 1.3 * 2 ** 0.5 * 0.05 / tq, (name, sd)

"""The GPU encoder (tmd_encode) against the oracle's encoder, bit for bit:
header arrays, per-cluster steps and residuals, unattached bin counts and
differences, and the number of mid-track headers; then the GPU decode of the
GPU encoding restores the quantised clusters exactly (the round trip
decode(encode(x)) == quantize(x)).  Inputs: exact helices with Gaussian
noise (several fields, including 0), tracks the model has to split (side
change, more than 255 clusters, residuals beyond int16), unattached clusters
with equal positions (ordered by their charges), and sizes that take many
blocks of the sort and of the header scan."""
import numpy as np
import pytest

import oracle
from oracle import physgen as pg
from test_oracle_roundtrip import _manual_phys

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tmd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_02206_amd as m
    return m


def check_encode(tmd, phys, bz, label):
    exp, exp_split = oracle.encode(phys, bz=bz)
    got, got_split = tmd.encode(phys, bz=bz)
    for k in exp:
        assert got[k].dtype == exp[k].dtype, (label, k)
        assert np.array_equal(exp[k], got[k]), (label, k, exp[k].shape, got[k].shape)
    assert got_split == exp_split, (label, got_split, exp_split)
    # the GPU decode of the GPU encoding: quantize(x), in the canonical layout
    out, flags = tmd.decode(tmd.to_device(got), bz=bz)
    res = tmd.to_numpy(out)
    want = pg.expected_clusters(phys)
    for k in want:
        assert np.array_equal(want[k], res[k]), (label, "roundtrip", k)
    assert flags == 0, (label, flags)
    return exp_split


@pytest.mark.parametrize("seed,bz", [(0, 0.5), (1, 0.5), (2, 0.0), (3, 2.0), (4, -0.5)])
def test_encode_physical(tmd, seed, bz):
    phys = pg.generate(seed=seed, n_tracks=300, n_un=5000, bz=bz)
    check_encode(tmd, phys, bz, f"seed {seed} bz {bz}")


def test_encode_splits(tmd):
    rng = np.random.default_rng(3)
    side_change = [(i % 18 if i < 5 else 18 + i % 18, 40 + i, 20.0 + 0.3 * i, 900.0 + i, 0.1) for i in range(10)]
    zigzag = [(3, 10 + (i % 2), 30.0 + rng.normal(0, 0.02), 1000.0 + 0.1 * i, 0.0) for i in range(300)]
    jumpy = [(5, 20 + i, 40.0 + (1500.0 if i == 6 else 0.0), 800.0 + i, 0.0) for i in range(12)]
    un = [(1, 2, 3.25, 4.0, 5, 6), (1, 2, 3.25, 4.0, 5, 5), (1, 2, 3.25, 4.0, 4, 9), (0, 0, 0.0, 0.0, 0, 0)]
    phys = _manual_phys([(0.5, 0.2, side_change), (1.0, 0.0, zigzag), (0.2, 0.0, jumpy)], un=un)
    assert check_encode(tmd, phys, 0.5, "splits") >= 3


def test_encode_many_blocks(tmd):
    """Enough clusters for hundreds of header-scan blocks and unattached
    clusters for dozens of sort tiles (with many equal times in a bin)."""
    phys = pg.generate(seed=9, n_tracks=6000, n_un=150000, bz=0.5)
    rng = np.random.default_rng(9)
    phys["un_time"] = np.floor(rng.uniform(0, 50, phys["un_time"].shape[0]))  # many ties
    check_encode(tmd, phys, 0.5, "many blocks")


def test_encode_empty_and_bad_input(tmd):
    phys = pg.generate(seed=1, n_tracks=5, n_un=0, bz=0.5)
    check_encode(tmd, phys, 0.5, "no unattached")
    bad = pg.generate(seed=1, n_tracks=5, n_un=10, bz=0.5)
    bad["un_pad"] = bad["un_pad"].copy()
    bad["un_pad"][3] = 5000.0   # 160000 in 1/32 pad: beyond 16 bits
    with pytest.raises(tmd.TmdError):
        tmd.encode(bad, bz=0.5)


def test_encode_synth_frame(tmd):
    """The encoder benchmark's input generator at a tenth of its size: every
    array bit for bit, and the round trip."""
    import synth
    phys = synth.make_phys(synth.spec_for("frame", collisions=10))
    check_encode(tmd, phys, 0.5, "synth frame")


@pytest.mark.parametrize("field,index,value", [("cl_time", 7, 2.0 ** 19), ("cl_pad", 3, -1.0),
                                               ("cl_pad", 40, 2048.0)])
def test_encode_attached_out_of_range(tmd, field, index, value):
    """An attached cluster outside the codable range (time code of 2^24 or
    more, pad code below 0 or beyond 16 bits) is refused, by the oracle's
    encoder and by the GPU's."""
    bad = pg.generate(seed=2, n_tracks=5, n_un=10, bz=0.5)
    bad[field] = bad[field].copy()
    bad[field][index] = value
    with pytest.raises(RuntimeError):
        oracle.encode(bad, bz=0.5)
    with pytest.raises(tmd.TmdError):
        tmd.encode(bad, bz=0.5)


def test_encode_unattached_only(tmd):
    """No tracks and no attached clusters: only the sort and the bin counts
    (a bin's first and last element in one place, bins 0 and 5471)."""
    un = [(1, 2, 3.25, 4.0, 5, 6), (1, 2, 3.0, 4.0, 5, 6), (35, 151, 10.0, 1e6, 1, 1), (0, 0, 0.0, 0.0, 0, 0),
          (1, 2, 3.25, 4.0, 5, 5)]
    phys = _manual_phys([], un=un)
    check_encode(tmd, phys, 0.5, "unattached only")


def test_encode_calls_in_a_row_share_a_workspace(tmd):
    """Two encodes after one another on one stream and one plan, reusing one
    workspace, twice over, the second smaller: the second stream of each call
    joins its own call, so nothing of one call's unattached sort mixes with
    the next call's."""
    import torch
    big = pg.generate(seed=5, n_tracks=400, n_un=60000, bz=0.5)
    small = pg.generate(seed=6, n_tracks=50, n_un=7000, bz=0.5)
    plan = tmd.Plan([(1, 1, 1)], bz=0.5)
    devb, devs = tmd.enc_to_device(big), tmd.enc_to_device(small)
    shb, shs = tmd.enc_shape(devb), tmd.enc_shape(devs)
    outb, outs = tmd.alloc_enc_out(*shb), tmd.alloc_enc_out(*shs)
    ws = torch.empty(tmd.enc_workspace_bytes(*shb), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    try:
        for _ in range(2):
            tmd.encode_device(plan, devb, outb, ws, stream)
            tmd.encode_device(plan, devs, outs, ws, stream)
        stream.synchronize()
        for phys, out, sh, label in ((big, outb, shb, "big"), (small, outs, shs, "small")):
            got, split = tmd.enc_result(out, sh[1], sh[2])
            exp, esplit = oracle.encode(phys, bz=0.5)
            for k in exp:
                assert np.array_equal(exp[k], got[k]), (label, k)
            assert split == esplit, label
    finally:
        plan.free()


def test_encode_full_frame(tmd):
    """The encoder benchmark's workload at its full size (200 000 tracks,
    2.46e7 clusters), in the launch configuration the benchmark times: every
    array bit for bit against the oracle's encoder."""
    import synth
    print("generating the physical clusters of the frame workload", flush=True)
    phys = synth.make_phys(synth.spec_for("frame"))
    print("oracle encoder", flush=True)
    exp, esplit = oracle.encode(phys, bz=0.5)
    got, split = tmd.encode(phys, bz=0.5)
    for k in exp:
        assert np.array_equal(exp[k], got[k]), k
    assert split == esplit


@pytest.mark.parametrize("presorted", [False, True])
def test_encode_equal_positions_over_many_tiles(tmd, presorted):
    """20 000 unattached clusters at one position in one bin, plus others
    spread out: their order is decided by the charges alone, given in random
    or in charge order.  A run of equal keys this long is ordered by the full
    sort (key and charges); short runs, as in the other tests here, are sorted
    by charge in place after the key's passes."""
    rng = np.random.default_rng(12)
    n_same, n_other = 20000, 30000
    qtot = rng.integers(0, 65536, n_same)
    qmax = rng.integers(0, 65536, n_same)
    if presorted:
        o = np.lexsort((qmax, qtot))
        qtot, qmax = qtot[o], qmax[o]
    un = [(7, 30, 12.5, 700.25, int(a), int(b)) for a, b in zip(qtot, qmax)]
    sec = rng.integers(0, 36, n_other)
    row = rng.integers(0, 152, n_other)
    un += [(int(s), int(r), float(rng.uniform(0, 60)), float(rng.uniform(0, 5000)), int(rng.integers(0, 9)),
            int(rng.integers(0, 9))) for s, r in zip(sec, row)]
    phys = _manual_phys([(0.5, 0.1, [(3, 10 + i, 30.0 + 0.1 * i, 900.0 + i, 0.0) for i in range(20)])], un=un)
    check_encode(tmd, phys, 0.5, f"equal positions, presorted {presorted}")


def test_encode_skewed_rows(tmd):
    """Physical clusters with the stress workload's row skew (start rows and
    unattached rows ~ exp(-row/40), so that the inner rows' bins hold many
    more clusters than the outer ones), at 5 collisions: bit for bit and the
    round trip."""
    import synth
    phys = synth.make_phys(synth.spec_for("stress", collisions=5))
    check_encode(tmd, phys, 0.5, "skewed rows")

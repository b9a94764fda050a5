"""The stress workload at full size (about 1e6 tracks and 1.25e8 clusters:
loopers, sector crossings, rows skewed exponentially), every cluster against
the oracle.  This module sorts first among the GPU tests so that the frame can
be drawn by forked worker processes before this process uses the GPU."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stress_frame():
    import torch
    # forked generator workers only while this process has not touched the GPU
    workers = 1 if torch.cuda.is_initialized() else 16
    print(f"stress frame: generating with {workers} worker(s)", flush=True)
    return synth.make_frame(synth.spec_for("stress"), workers=workers)


def test_stress_workload_full_size(stress_frame):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_02206_amd as tmd
    fr = stress_frame
    shape = tmd.frame_shape(fr)
    print(f"stress frame: {shape[0]} tracks, {shape[1]} attached, {shape[2]} unattached", flush=True)
    out, flags = tmd.decode(tmd.to_device(fr))
    got = tmd.to_numpy(out)
    del out
    exp, est = oracle.decode(fr)
    for k in exp:
        assert np.array_equal(exp[k], got[k]), k
    assert flags == est
    assert exp["row_offset"][-1] > 1.2e8

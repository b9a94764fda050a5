"""The serving scheduler without a GPU: a fake executor stands in for the
device.  Checks admission by HBM budget, FIFO order, batch sizes and that
every request completes."""
import numpy as np

from paper_2411_02206_amd import serve


def fake_frame(nt, na, nu):
    return {"trk_ncls": np.zeros(nt, np.uint8), "cls_qtot": np.zeros(na, np.uint16),
            "un_qtot": np.zeros(nu, np.uint16)}


def test_budget_fifo_and_batching():
    batches = []
    srv = serve.Server(hbm_budget=3.5e6, slots=2, max_batch=3, executor=lambda b: batches.append(list(b)))
    reqs = [srv.submit(fake_frame(100 + i, 10000 + 1000 * i, 5000), arrival=float(i)) for i in range(12)]
    srv.run_until(len(reqs), timeout=10)
    assert all(r.done_time is not None for r in reqs)
    order = [r for b in batches for r in b]
    assert order == reqs                      # admitted in arrival order
    assert max(len(b) for b in batches) <= 3
    assert srv.peak_in_use <= 3.5e6
    assert srv.in_use == 0


def test_oversized_frame_rejected():
    srv = serve.Server(hbm_budget=1e5, executor=lambda b: None)
    try:
        srv.submit(fake_frame(1000, 100000, 100000))
    except ValueError:
        return
    raise AssertionError("an oversized frame was accepted")


def test_admission_waits_for_memory():
    """With room for one frame at a time, each batch holds one frame."""
    batches = []
    one = serve.frame_bytes((100, 20000, 10000))
    srv = serve.Server(hbm_budget=1.5 * one, slots=4, max_batch=8, executor=lambda b: batches.append(list(b)))
    for i in range(5):
        srv.submit(fake_frame(100, 20000, 10000))
    srv.run_until(5, timeout=10)
    assert [len(b) for b in batches] == [1] * 5


def test_percentile():
    assert serve.percentile([3, 1, 2], 50) == 2
    assert serve.percentile(list(range(101)), 99) == 99


def test_capacity_growth():
    """Plan capacity starts at 1.25x the first frame and grows by 1.25x past
    any larger frame, per count."""
    assert serve._grow((0, 0, 0), (100, 1000, 10)) == (126, 1251, 13)
    assert serve._grow((126, 1251, 13), (100, 2000, 10)) == (126, 2501, 13)
    srv = serve.Server(slots=1, max_batch=2, executor=lambda b: None)
    srv.submit(fake_frame(100, 1000, 10))
    srv.submit(fake_frame(50, 3000, 5))
    srv.run_until(2, timeout=10)
    assert srv.capacity == (126, 3751, 13)

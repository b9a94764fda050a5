"""The measurement tooling on the CPU: the algorithmic bytes the roofline
divides by, the roofline entry itself, the traffic summaries (kept only for
the kernel source they were measured with) and the kernel-name form they use,
and the benchmark's refusal of several GPUs."""
import json
import os
import subprocess
import sys

import pytest

import bench
from paper_2411_02206_amd import traffic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes():
    # the frame workload: 200 000 tracks, 15 364 162 attached and 10 242 775
    # unattached clusters; its attached decode moves 10 B in and 10 B out per
    # cluster and 15 B per header
    att, una, total = bench.algorithmic_bytes(200000, 15364162, 10242775)
    assert att == 20 * 15364162 + 15 * 200000 == 310283240
    assert una == 20 * 10242775
    assert total == att + una + 5472 * 12
    kb = bench.kernel_bytes([(200000, 15364162, 10242775), (1, 2, 3)])
    assert kb["attached"] == 20 * (15364162 + 2) + 15 * 200001
    assert kb["unattached"] == 20 * (10242775 + 3)


def test_roofline_entry(monkeypatch):
    summ = {"frames": 64, "kernels": {"k_attached": {"traffic_bytes": 2.5e9},
                                      "k_rans_prep": {"traffic_bytes": 1e6},
                                      "k_rans<2, 0>": {"traffic_bytes": 3e9},
                                      "k_rans<2, 1>": {"traffic_bytes": 7e9}}}
    monkeypatch.setattr(traffic, "load_summary", lambda w: summ)
    r = bench.roofline("attached", 1e9, 0.5, "frame")
    assert r["achieved"] == 2000.0 and r["frac"] == 0.25 and r["unit"] == "GB/s"
    assert r["traffic"] == 2.5e9 and r["kernel"] == "k_attached" and r["bytes_per_launch"] == 1e9
    # the entropy decoding before the decode: its prep kernel and phase-0 kernels only
    assert bench.roofline("rans", 1e9, 1.0, "coded")["traffic"] == 3e9 + 1e6
    # a batched summary measured on another number of frames is not used
    assert bench.roofline("attached", 1e9, 0.5, "batched", frames=8)["traffic"] is None
    assert bench.roofline("attached", None, 0.5, "frame") is None
    assert bench.add_copy_frac(r, 5000.0)["frac_of_copy"] == 0.4


def _write_summary(d, workload, sha):
    s = {"workload": workload, "frames": 1, "source_sha256": sha, "kernels": {}}
    with open(os.path.join(d, f"traffic_{workload}.md"), "w") as f:
        f.write("# HBM traffic\n\ntraffic-json: " + json.dumps(s) + "\n")


def test_traffic_summary_only_for_its_source(tmp_path):
    _write_summary(tmp_path, "frame", traffic.source_hash())
    assert traffic.load_summary("frame", str(tmp_path))["workload"] == "frame"
    _write_summary(tmp_path, "stress", "0" * 64)  # another kernel source
    assert traffic.load_summary("stress", str(tmp_path)) is None
    assert traffic.load_summary("coded", str(tmp_path)) is None  # none written


def test_kernel_names():
    assert traffic.kernel_name("void (anonymous namespace)::k_rans<2, 1>(RansDesc const*, unsigned int const*)") \
        == "k_rans<2, 1>"
    assert traffic.kernel_name("(anonymous namespace)::k_attached(FrameDesc const*)") == "k_attached"


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("workload,kernel", [("batched", "k_attached"), ("coded", "k_attached"),
                                             ("frame", "k_attached"), ("stress", "k_attached"),
                                             ("encode", "k_enc_tracks")])
def test_committed_summaries_parse(workload, kernel):
    """Every committed traffic summary carries its JSON line and the kernels'
    calibrated bytes (whether it is current is checked by load_summary)."""
    fn = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    lines = [l for l in open(fn) if l.startswith("traffic-json: ")]
    assert len(lines) == 1
    s = json.loads(lines[0][len("traffic-json: "):])
    assert s["workload"] == workload and len(s["source_sha256"]) == 64
    assert s["kernels"][kernel]["traffic_bytes"] > 0


def test_encode_bytes_and_roofline(monkeypatch):
    # 20 B in per track, 30 B in and 10 B out per attached cluster, 22 B in and 10 B out per unattached one,
    # 15 B per header written and the bin counts
    assert bench.encode_bytes(2, 10, 5, 3) == 20 * 2 + 40 * 10 + 32 * 5 + 15 * 3 + 4 * 5472
    summ = {"frames": 64, "kernels": {"k_enc_tracks": {"traffic_bytes": 1e6, "dispatches": 4},
                                      "k_rad_scatter": {"traffic_bytes": 2e6, "dispatches": 48},
                                      "k_attached": {"traffic_bytes": 9e9, "dispatches": 4}}}
    monkeypatch.setattr(traffic, "load_summary", lambda w: summ)
    r = bench.roofline("encode", 4e8, 0.2, "encode")
    assert r["kernel"] == "tmd_encode (all kernels)" and r["achieved"] == 2000.0
    assert r["traffic"] == 1e6 + 12 * 2e6   # per call: twelve scatter passes

"""Run by tests/test_sanitizers.py in a child process whose oracle library is
an AddressSanitizer + UndefinedBehaviorSanitizer build: decodes and encodes a
set of frames and prints one digest line per result."""
import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import physgen as pg  # noqa: E402
import synth  # noqa: E402

NBIN = 36 * 152


def garbage(seed, nt=50, na=3000, nu=9000):
    rng = np.random.default_rng(seed)
    fr = {
        "trk_ncls": rng.integers(0, 256, nt).astype(np.uint8),
        "trk_sec0": rng.integers(0, 256, nt).astype(np.uint8),
        "trk_row0": rng.integers(0, 256, nt).astype(np.uint8),
        "trk_pad0": rng.integers(0, 65536, nt).astype(np.uint16),
        "trk_time0": rng.integers(0, 2**32, nt, dtype=np.uint64).astype(np.uint32),
        "trk_qpt": rng.integers(-32768, 32768, nt).astype(np.int16),
        "trk_snp": rng.integers(-32768, 32768, nt).astype(np.int16),
        "trk_tgl": rng.integers(-32768, 32768, nt).astype(np.int16),
        "cls_row_diff": rng.integers(-128, 128, na).astype(np.int8),
        "cls_sec_diff": rng.integers(0, 256, na).astype(np.uint8),
        "cls_pad_res": rng.integers(-32768, 32768, na).astype(np.int16),
        "cls_time_res": rng.integers(-32768, 32768, na).astype(np.int16),
        "cls_qtot": rng.integers(0, 65536, na).astype(np.uint16),
        "cls_qmax": rng.integers(0, 65536, na).astype(np.uint16),
        "un_count": rng.integers(0, 3, NBIN).astype(np.uint32),
        "un_time_diff": rng.integers(0, 2**32, nu, dtype=np.uint64).astype(np.uint32),
        "un_pad_diff": rng.integers(0, 65536, nu).astype(np.uint16),
        "un_qtot": rng.integers(0, 65536, nu).astype(np.uint16),
        "un_qmax": rng.integers(0, 65536, nu).astype(np.uint16),
    }
    return fr


def digest(d, status):
    h = hashlib.sha256()
    for k in sorted(d):
        h.update(k.encode())
        h.update(np.ascontiguousarray(d[k]).tobytes())
    h.update(str(status).encode())
    return h.hexdigest()


def main():
    cases = [("tiny", synth.make_frame(synth.spec_for("tiny")), 0.5),
             ("stress2", synth.make_frame(synth.spec_for("stress", collisions=1)), 0.5)]
    for s in range(3):
        cases.append((f"garbage{s}", garbage(100 + s), 5.0))
    for name, fr, bz in cases:
        out, st = oracle.decode(fr, bz=bz)
        print(f"decode {name} {digest(out, st)}", flush=True)
    phys = pg.generate(seed=7, n_tracks=60, n_un=500, bz=0.5)
    enc, nsplit = oracle.encode(phys, bz=0.5)
    print(f"encode phys {digest(enc, nsplit)}", flush=True)
    for name, fr, _ in cases[:3]:
        blob = oracle.rans_encode(fr)
        back = oracle.rans_decode(blob, oracle.frame_sizes(fr))
        same = all(np.array_equal(fr[k], back[k]) for k, _ in oracle.RANS_ARRAYS)
        bad = 0
        for cut in (0, 16, blob.size // 3, blob.size - 1):
            try:
                oracle.rans_decode(blob[:cut], oracle.frame_sizes(fr))
            except ValueError:
                bad += 1
        print(f"rans {name} {blob.size} {same} {bad}", flush=True)


if __name__ == "__main__":
    main()

"""Autotuner of the attached decode's schedule.

The attached decode has two scheduling knobs (tmd_set_schedule), neither of
which changes a result:
  - tracks per wave (64..128): above 64, the tracks that start last are each
    decoded after a track of the same wave that ends earlier, in the same lane
    (length bucketing across the lanes: more of a wave's lanes busy per row
    step, fewer waves);
  - persistent waves per SIMD (0 = one workgroup per wave of work; n > 0 = a
    grid of n waves per SIMD pulling the waves of work from per-XCD counters).
Which setting is fastest depends on the device and on the frame mix (track
count per frame against the SIMD count, number of frames).  `choose` times
the candidate settings on the caller's own plan and buffers and keeps the
fastest; `tuned` looks the choice up in a JSON cache keyed by the device and a
shape class of the frames, and tunes (and stores) on a miss.

    from paper_2411_02206_amd import autotune
    setting, info = autotune.tuned(plan, ins, outs, ws, stream)
"""
import json
import math
import os
import time

CANDIDATES = [(64, 0), (72, 0), (76, 0), (80, 0), (84, 0), (64, 2), (72, 2), (76, 2), (80, 2), (76, 3)]
DEFAULT = (64, 0)


def cache_path():
    return os.environ.get("TMD_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "tmd", "autotune.json")


def shape_class(shapes):
    """Frames are tuned alike when they agree in the number of frames and,
    on a log2 scale, in the mean and largest track counts."""
    n = len(shapes)
    tracks = [s[0] for s in shapes] or [0]
    mean = sum(tracks) / len(tracks)
    lg = lambda v: int(round(math.log2(v))) if v > 0 else -1  # noqa: E731
    return f"f{n}-t{lg(mean)}-m{lg(max(tracks))}"


def device_key():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|cu{p.multi_processor_count}"


def load_cache(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store_cache(cache, path=None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(timings):
    """The fastest setting; ties go to the earlier candidate."""
    best = None
    for setting, ms in timings:
        if best is None or ms < best[1]:
            best = (setting, ms)
    return best[0]


def choose(plan, ins, outs, ws, stream=None, candidates=CANDIDATES, reps=3, timer=None):
    """Time every candidate on this plan (median of `reps` decodes after one
    warm-up) and leave the plan set to the fastest.  Returns (setting,
    [(setting, ms), ...]).  timer(setting) may replace the measurement
    (tests)."""
    timings = []
    for setting in candidates:
        plan.set_schedule(*setting)
        if timer is not None:
            ms = timer(setting)
        else:
            ms = _measure(plan, ins, outs, ws, stream, reps)
        timings.append((tuple(setting), ms))
    best = pick(timings)
    plan.set_schedule(*best)
    return best, timings


def _measure(plan, ins, outs, ws, stream, reps):
    import torch
    stream = stream or torch.cuda.current_stream()
    plan.decode(ins, outs, ws, stream)
    ev = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.decode(ins, outs, ws, stream)
        b.record(stream)
        ev.append((a, b))
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in ev)
    return t[len(t) // 2]


def tuned(plan, ins, outs, ws, stream=None, path=None, candidates=CANDIDATES, reps=3, device=None,
          timer=None):
    """Set the plan to the cached choice for its device and shape class, or
    tune, store and set it.  Returns (setting, info)."""
    device = device or device_key()
    key = f"{device}::{shape_class(plan.shapes)}"
    cache = load_cache(path)
    hit = cache.get(key)
    if hit is not None:
        setting = tuple(hit["setting"])
        plan.set_schedule(*setting)
        return setting, {"key": key, "cache": "hit", "timings_ms": hit.get("timings_ms")}
    t0 = time.perf_counter()
    setting, timings = choose(plan, ins, outs, ws, stream, candidates, reps, timer)
    entry = {"setting": list(setting), "timings_ms": {f"{a}x{b}": round(ms, 4) for (a, b), ms in timings},
             "tuned_s": round(time.perf_counter() - t0, 2)}
    cache = load_cache(path)  # (another process may have stored meanwhile)
    cache[key] = entry
    store_cache(cache, path)
    return setting, {"key": key, "cache": "miss", "timings_ms": entry["timings_ms"]}

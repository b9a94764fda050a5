"""Host logic of the schedule autotuner (no GPU): shape classes, choice of
the fastest setting with ties to the earlier candidate, the JSON cache (hit
after a miss, one entry per device and shape class)."""
from paper_2411_02206_amd import autotune


class FakePlan:
    def __init__(self, shapes):
        self.shapes = shapes
        self.settings = []

    def set_schedule(self, tpw, persist):
        self.settings.append((tpw, persist))


def test_shape_class():
    a = autotune.shape_class([(200000, 1, 1)])
    assert a == autotune.shape_class([(210000, 5, 5)])
    assert a != autotune.shape_class([(100000, 1, 1)])
    assert a != autotune.shape_class([(200000, 1, 1)] * 2)
    assert autotune.shape_class([(0, 0, 0)]) == "f1-t-1-m-1"


def test_pick_and_ties():
    assert autotune.pick([((64, 0), 2.0), ((80, 0), 1.5), ((72, 2), 1.5)]) == (80, 0)


def test_tuned_caches(tmp_path):
    path = str(tmp_path / "cache.json")
    plan = FakePlan([(200000, 10, 10)])
    cost = {(64, 0): 3.0, (80, 0): 2.0, (80, 2): 2.5}
    calls = []

    def timer(s):
        calls.append(s)
        return cost[s]
    s, info = autotune.tuned(plan, None, None, None, path=path, candidates=list(cost), device="dev", timer=timer)
    assert s == (80, 0) and info["cache"] == "miss" and len(calls) == 3
    assert plan.settings[-1] == (80, 0)
    plan2 = FakePlan([(190000, 1, 1)])
    s2, info2 = autotune.tuned(plan2, None, None, None, path=path, candidates=list(cost), device="dev", timer=timer)
    assert s2 == (80, 0) and info2["cache"] == "hit" and len(calls) == 3
    assert plan2.settings == [(80, 0)]
    s3, info3 = autotune.tuned(FakePlan([(190000, 1, 1)]), None, None, None, path=path, candidates=list(cost),
                               device="other", timer=timer)
    assert info3["cache"] == "miss" and len(calls) == 6
    assert len(autotune.load_cache(path)) == 2

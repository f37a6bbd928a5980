"""The autotuner's choice rule (host logic, no GPU): the lone cycle's time
first, the back-to-back time among candidates within 1 % of the best lone
time."""
from paper_2603_01122_amd import tune


def test_pick_prefers_latency_then_throughput():
    times = {"a": (1.000, 2.0), "b": (1.009, 1.5), "c": (1.2, 1.0)}
    assert tune.pick(times) == "b"          # within 1 % of the best lone time, faster back to back
    times["b"] = (1.011, 1.5)
    assert tune.pick(times) == "a"          # outside the window: latency decides
    assert tune.pick({"x": [0.5, 0.7]}) == "x"   # lists (as read back from JSON) work too

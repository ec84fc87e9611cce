"""CPU checks of the seeded input generators' stream shapes (no GPU)."""
from __future__ import annotations

import workload


def test_served_stream_outliers():
    ps = workload.served(2, 40, 0.05)
    out = [p for p in ps if p.name.endswith("-outlier")]
    assert len(out) == 2  # round(40 x 0.05)
    for p in out:
        assert p.n_props == 5 and len(p.traces) == 1024
        assert sum(p.positive) == 512
        assert all(16 <= len(t) <= 64 for t in p.traces)
        assert 9 <= p.cost_bound <= 15  # planted U{6..12} + 3
    again = workload.served(2, 40, 0.05)
    assert [p.name for p in again] == [p.name for p in ps]
    assert all(a.traces == b.traces for a, b in zip(again, ps) if a.name.endswith("-outlier"))


def test_served_stream_without_outliers_is_the_batched_mix():
    a = workload.served(2, 24, 0.0)
    b = workload.batched(2, 24)
    assert [p.name for p in a] == [p.name for p in b]
    assert all(x.traces == y.traces and x.positive == y.positive for x, y in zip(a, b))

"""GPU: the stored level sets, compared with the oracle's as sets.

* Per-level digests (LTLF_FLAG_DIGEST, computed on the device from the stored
  rows) equal the digests the tests compute from the oracle's exported levels
  with their own code (tests/digest.py), under every generation kernel.
* Levels that span several generation launches (a 256 MiB workspace: the
  deferral list holds ~2.5e5 records, so level 9 of the medium problem, with
  ~1e6 candidates, runs as several launches with table growth between them)
  export exactly the oracle's sorted CM sets, under every kernel.

Bar: bit-exact sets (sorted canonical rows) and equal 64-bit digests.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_2504_18943_amd as m
import workload
from tests import digest

pytestmark = pytest.mark.gpu

KERNELS = {"lane": m.FLAG_KERNEL_LANE, "group": m.FLAG_KERNEL_GROUP, "wave": m.FLAG_KERNEL_WAVE}


def oracle_digests(o, p):
    return [0] + [digest.level_digest(o.export_level(c), p.lengths) for c in range(1, o.levels_done + 1)]


def sorted_rows(a):
    return a[np.lexsort(a.T[::-1])] if len(a) else a


@pytest.mark.parametrize("kernel", sorted(KERNELS))
def test_level_digests_match_oracle(synth, kernel):
    for p, b in ((workload.tiny(1), 8), (workload.tiny(2), 8), (workload.medium(1), 7), (workload.large(1), 5)):
        print(f"[digest] {p.name} bound {b} kernel {kernel}", flush=True)
        o = oracle.solve(p, cost_bound=b, exhaust=True)
        want = oracle_digests(o, p)
        r = synth.solve(p, cost_bound=b, flags=m.FLAG_EXHAUST | m.FLAG_DIGEST | KERNELS[kernel])
        assert (r.status, r.levels_done, r.level_counts) == (o.status, o.levels_done, o.level_counts), p.name
        assert r.level_digests[: o.levels_done + 1] == want, p.name
        assert all(d == 0 for d in r.level_digests[o.levels_done + 1:])


def test_digests_off_without_the_flag(synth):
    r = synth.solve(workload.tiny(3), cost_bound=6, flags=m.FLAG_EXHAUST)
    assert r.levels_done == 6 and not any(r.level_digests)


@pytest.fixture(scope="module")
def medium9():
    p = workload.medium(1)
    o = oracle.solve(p, cost_bound=9, exhaust=True)
    sets = {c: sorted_rows(o.export_level(c)) for c in range(1, o.levels_done + 1)}
    return p, o, sets, oracle_digests(o, p)


@pytest.mark.parametrize("kernel", sorted(KERNELS))
def test_multi_launch_levels_equal_oracle_sets(medium9, kernel):
    p, o, sets, want = medium9
    assert o.levels_done == 9
    s = m.Synthesizer(device=0, workspace_bytes=256 << 20)
    try:
        print(f"[digest] medium seed 1 to cost 9, 256 MiB workspace, kernel {kernel}", flush=True)
        r = s.solve(p, cost_bound=9, flags=m.FLAG_EXHAUST | m.FLAG_DIGEST | KERNELS[kernel])
        print(f"[digest]   {r.gen_launches} generation launches, {r.deferred} deferred", flush=True)
        assert (r.status, r.min_cost, r.levels_done, r.overflow_level) == \
            (o.status, o.min_cost, o.levels_done, o.overflow_level)
        assert r.level_counts == o.level_counts
        if kernel == "lane":  # one launch per level would be 9 (8 with candidates past the atoms)
            assert r.gen_launches >= 12, r.gen_launches
        for c in range(1, 10):
            got = sorted_rows(s.export_level(c))
            assert got.shape == sets[c].shape, c
            assert np.array_equal(got, sets[c]), f"level {c} differs"
        assert r.level_digests[:10] == want
    finally:
        s.close()

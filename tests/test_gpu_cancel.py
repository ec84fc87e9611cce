"""GPU tests of cancellation (ltlf_ctx_cancel): a run stops between two levels
with status CANCELLED and exact counts for the levels it completed; a
request that finds no run in progress stops the context's next run before
its first level; the context stays usable."""
from __future__ import annotations

import threading
import time

import pytest

import oracle
import paper_2504_18943_amd as m
import workload

pytestmark = pytest.mark.gpu


def test_pending_cancel_stops_the_next_run_before_its_first_level(synth):
    p = workload.tiny(2)
    synth.load(p)
    synth.cancel()
    r = synth.run(8, flags=m.FLAG_EXHAUST)
    assert r.status == m.CANCELLED and r.status_name == "CANCELLED"
    assert r.levels_done == 0 and not any(r.level_counts) and r.formula == ""
    # the request was used up: the next run is complete and exact
    o = oracle.solve(p, cost_bound=8, exhaust=True)
    r = synth.run(8, flags=m.FLAG_EXHAUST)
    assert (r.status, r.min_cost, r.levels_done, r.level_counts) == (o.status, o.min_cost, o.levels_done,
                                                                     o.level_counts)


def test_cancel_during_a_run_keeps_completed_levels_exact():
    p = workload.large(1)
    s = m.Synthesizer(device=0, workspace_bytes=40 << 30)
    try:
        s.load(p)
        full = s.run(9, flags=m.FLAG_EXHAUST)
        assert full.levels_done == 9
        print("[cancel] large seed 1 to cost 9, cancelled from another thread", flush=True)
        out = {}
        t = threading.Thread(target=lambda: out.setdefault("r", s.run(9, flags=m.FLAG_EXHAUST)))
        t.start()
        time.sleep(0.004)
        s.cancel()
        t.join()
        r = out["r"]
        if r.status == m.CANCELLED:
            assert r.levels_done < 9
            assert r.level_counts[: r.levels_done + 1] == full.level_counts[: r.levels_done + 1]
            assert not any(r.level_counts[r.levels_done + 1:])
            assert r.checked_level == r.levels_done
        else:  # the run ended first: the request waits for the next run
            assert (r.status, r.level_counts) == (full.status, full.level_counts)
            again = s.run(9, flags=m.FLAG_EXHAUST)
            assert again.status == m.CANCELLED and again.levels_done == 0
        after = s.run(9, flags=m.FLAG_EXHAUST)
        assert (after.status, after.level_counts) == (full.status, full.level_counts)
    finally:
        s.close()


def test_cancel_before_a_batch_cancels_every_problem(synth):
    ps = [workload.tiny(1), workload.tiny(2), workload.medium(1)]
    synth.cancel()
    rs = synth.solve_batch(ps, [8, 8, 8])
    for r in rs:
        assert r.status == m.CANCELLED and r.levels_done == 0 and not any(r.level_counts)
    # nothing left pending: the next batch is complete and exact
    rs = synth.solve_batch(ps, [8, 8, 8])
    for p, r in zip(ps, rs):
        o = oracle.solve(p, cost_bound=8)
        assert (r.status, r.min_cost, r.levels_done, r.level_counts) == (o.status, o.min_cost, o.levels_done,
                                                                         o.level_counts)

"""GPU tests of the request server (ltlf_server_*): results equal solving
each request alone (and the oracle), whatever arrives while others run.

Bar: per request, status, minimal cost, levels_done and |U_c| of every
stored level identical to ltlf_solve on the same problem and to the oracle;
the witness separates and costs the minimal cost.
"""
from __future__ import annotations

import pytest

import oracle
import paper_2504_18943_amd as m
import workload
from oracle import evaluator as ev
from tests import digest

pytestmark = pytest.mark.gpu


def same(r, a, p):
    assert (r.status, r.min_cost, r.levels_done, r.overflow_level, r.level_counts, r.level_digests) == \
        (a.status, a.min_cost, a.levels_done, a.overflow_level, a.level_counts, a.level_digests), p.name
    assert any(r.level_digests), p.name
    if r.status == m.ltlf.OK:
        assert ev.separates(r.formula, p.traces, p.positive), (p.name, r.formula)
        assert ev.cost(r.formula) == r.min_cost, (p.name, r.formula)


def drain(srv, tickets, limit=10000):
    out = {}
    for _ in range(limit):
        for t in list(tickets):
            if t in out:
                continue
            r = srv.poll(t)
            if r is not None:
                out[t] = r
        if len(out) == len(tickets):
            return out
        srv.step()
    raise AssertionError("requests did not finish")


def test_arrivals_while_running_match_alone_and_oracle():
    s = m.Synthesizer(device=0, workspace_bytes=4 << 30)
    ps = [workload.medium(1), workload.tiny(1), workload.medium(2), workload.tiny(2),
          workload.large(1), workload.tiny(3), workload.medium(3), workload.tiny(4)]
    bounds = [p.cost_bound for p in ps]
    bounds[4] = 5  # the large problem: its oracle is cheap to this bound
    D = m.FLAG_DIGEST
    alone = [s.solve(p, cost_bound=b, flags=D) for p, b in zip(ps, bounds)]
    srv = m.Server(s, max_resident=8)
    print("[server] staggered arrivals", flush=True)
    tickets = [srv.submit(ps[0], bounds[0], flags=D), srv.submit(ps[1], bounds[1], flags=D)]
    srv.step()
    tickets += [srv.submit(ps[2], bounds[2], flags=D), srv.submit(ps[3], bounds[3], flags=D)]
    srv.step()
    srv.step()
    tickets += [srv.submit(p, b, flags=D) for p, b in zip(ps[4:], bounds[4:])]
    got = drain(srv, tickets)
    srv.close()
    for p, b, t, a in zip(ps, bounds, tickets, alone):
        same(got[t], a, p)
        o = oracle.solve(p, cost_bound=b)
        assert (got[t].status, got[t].min_cost, got[t].level_counts[: o.levels_done + 1]) == \
            (o.status, o.min_cost, o.level_counts[: o.levels_done + 1]), p.name
        want = [0] + [digest.level_digest(o.export_level(c), p.lengths) for c in range(1, o.levels_done + 1)]
        assert got[t].level_digests[: o.levels_done + 1] == want, p.name
    s.close()


def test_large_levels_move_to_the_large_region():
    """A request given the minimum reservation reaches levels over 2^20
    candidates: it is restarted in the large region and still reports
    exactly the oracle's levels, while a small request runs beside it."""
    s = m.Synthesizer(device=0, workspace_bytes=2 << 30)
    p = workload.medium(1)
    srv = m.Server(s, max_resident=4)
    print("[server] large region", flush=True)
    t = srv.submit(p, 9, flags=m.FLAG_EXHAUST | m.FLAG_DIGEST, reserve_bytes=16 << 20)
    t2 = srv.submit(workload.tiny(5), 8, flags=m.FLAG_EXHAUST)
    got = drain(srv, [t, t2])
    srv.close()
    o = oracle.solve(p, cost_bound=9, exhaust=True)
    assert (got[t].status, got[t].min_cost, got[t].levels_done) == (o.status, o.min_cost, o.levels_done)
    assert got[t].level_counts == o.level_counts
    assert got[t].level_digests == [0] + [digest.level_digest(o.export_level(c), p.lengths) for c in range(1, 10)]
    o2 = oracle.solve(workload.tiny(5), cost_bound=8, exhaust=True)
    assert got[t2].level_counts == o2.level_counts
    s.close()


def test_overflow_of_the_large_region_is_exact():
    """A request larger than the large region: its stored levels, minimal
    cost and the overflow are reported exactly (the oracle's counts for
    every stored level)."""
    s = m.Synthesizer(device=0, workspace_bytes=256 << 20)
    p = workload.medium(1)
    srv = m.Server(s, max_resident=2)
    print("[server] overflow of the large region", flush=True)
    t = srv.submit(p, 11, flags=m.FLAG_EXHAUST)
    t2 = srv.submit(workload.tiny(6), 7)
    got = drain(srv, [t, t2])
    srv.close()
    r = got[t]
    assert r.overflow_level > 0 and r.levels_done == r.overflow_level - 1
    assert r.status == m.ltlf.OK and r.min_cost == 6
    o = oracle.solve(p, cost_bound=min(r.levels_done, 9), exhaust=True)
    assert r.level_counts[: o.levels_done + 1] == o.level_counts[: o.levels_done + 1]
    o2 = oracle.solve(workload.tiny(6), cost_bound=7)
    assert (got[t2].status, got[t2].min_cost) == (o2.status, o2.min_cost)
    s.close()


def test_lookahead_in_the_large_region():
    """A row limit overflows the level below the minimum: in the server the
    request moves to the large region, whose look-ahead finds the minimum one
    level past the overflow, as a solo run and the oracle do (and stops at
    the overflow with LTLF_FLAG_NO_LOOKAHEAD)."""
    p = workload.tiny(1)
    full = oracle.solve(p)
    c = full.min_cost - 1
    cap = sum(full.level_counts[1:c]) + full.level_counts[c] - 1
    s = m.Synthesizer(device=0, workspace_bytes=1 << 30)
    s.set_row_limit(cap)
    try:
        print(f"[server] look-ahead in the large region, row limit {cap}", flush=True)
        srv = m.Server(s, max_resident=4)
        t1 = srv.submit(p)
        t2 = srv.submit(p, flags=m.FLAG_NO_LOOKAHEAD)
        t3 = srv.submit(workload.tiny(2), 7)
        got = drain(srv, [t1, t2, t3])
        srv.close()
        for t, fl in ((t1, 0), (t2, m.FLAG_NO_LOOKAHEAD)):
            a = s.solve(p, flags=fl)
            o = oracle.solve(p, max_rows=cap, lookahead=not fl)
            r = got[t]
            key = lambda x: (x.status, x.min_cost, x.levels_done, x.overflow_level, x.checked_level)  # noqa: E731
            assert key(r) == key(a) == key(o), (fl, r, a, o)
        assert got[t1].status == m.ltlf.OK and got[t1].min_cost == full.min_cost
        assert got[t2].status == m.ltlf.CAPACITY
        assert ev.separates(got[t1].formula, p.traces, p.positive) and ev.cost(got[t1].formula) == full.min_cost
    finally:
        s.set_row_limit(0)
        s.close()


def test_cancel_pending_invalid():
    s = m.Synthesizer(device=0, workspace_bytes=1 << 30)
    srv = m.Server(s, max_resident=2)
    print("[server] cancel / pending / invalid", flush=True)
    ps = [workload.medium(1), workload.tiny(1), workload.tiny(2), workload.tiny(3)]
    ts = [srv.submit(p, 9 if i == 0 else None, flags=m.FLAG_EXHAUST if i == 0 else 0) for i, p in enumerate(ps)]
    assert srv.poll(ts[0]) is None  # nothing has run yet
    srv.cancel(ts[3])  # still queued (two resident at most)
    srv.step()
    srv.cancel(ts[0])  # resident
    with pytest.raises(m.LtlfError) as e:
        srv.poll(ts[0])
    assert e.value.status == m.ltlf.EINVAL
    bad = workload.Problem(n_props=2, traces=[[1], []], positive=[1, 0], cost_bound=4)
    with pytest.raises(m.LtlfError) as e:
        srv.submit(bad)
    assert e.value.status == m.ltlf.EINVAL
    got = drain(srv, ts[1:3])
    q, r, free = srv.load()
    assert (q, r) == (0, 0) and free > 0
    srv.close()
    for p, t in zip(ps[1:3], ts[1:3]):
        o = oracle.solve(p)
        assert (got[t].status, got[t].min_cost, got[t].level_counts[: o.levels_done + 1]) == \
            (o.status, o.min_cost, o.level_counts[: o.levels_done + 1])
    # the context works normally afterwards
    p = workload.tiny(7)
    r = s.solve(p, cost_bound=7, flags=m.FLAG_EXHAUST)
    assert r.level_counts[:8] == oracle.solve(p, cost_bound=7, exhaust=True).level_counts[:8]
    s.close()


def test_large_jobs_run_together_and_keep_their_levels():
    """Several requests whose levels outgrow the small pool: each moves into
    the large area with its stored levels (no level is enumerated twice), and
    they run there at the same time, each on its own worker.  Every result
    equals the request solved alone (status, cost, levels, counts, digests)."""
    s = m.Synthesizer(device=0, workspace_bytes=24 << 30)
    ps = [workload.medium(1), workload.medium(2), workload.medium(3), workload.medium(4)]
    D = m.FLAG_EXHAUST | m.FLAG_DIGEST
    alone = [s.solve(p, cost_bound=10, flags=D) for p in ps]
    srv = m.Server(s, max_resident=8)
    print("[server] concurrent large jobs", flush=True)
    tickets = [srv.submit(p, 10, flags=D) for p in ps]
    tickets.append(srv.submit(workload.tiny(3), 8, flags=D))
    got = drain(srv, tickets)
    srv.close()
    for p, t, a in zip(ps, tickets, alone):
        same(got[t], a, p)
        assert got[t].levels_done == 10
    s.close()


def test_whole_area_taken_with_stored_levels_while_serving(capfd, monkeypatch):
    """A served request that comes to need the whole large area (batched
    problem 113 in a 100 GiB workspace, at its level 10) takes it with its
    stored levels while tiny requests keep arriving and finishing; every
    result equals the problem solved alone, sets included."""
    big = workload.batched(1, 114)[113]
    monkeypatch.setenv("LTLF_TRACE", "1")
    s = m.Synthesizer(device=0, workspace_bytes=100 << 30)
    try:
        D = m.FLAG_DIGEST
        smalls = [workload.tiny(i) for i in range(1, 7)]
        srv = m.Server(s, max_resident=8)
        print("[server] whole area with stored levels", flush=True)
        tickets = [srv.submit(big, flags=D)]
        ps = [big]
        for i, p in enumerate(smalls):  # arrivals while the large request runs
            for _ in range(3 + i):
                srv.step()
            tickets.append(srv.submit(p, flags=D))
            ps.append(p)
        out = drain(srv, tickets)
        trace = capfd.readouterr().err
        promoted = trace.count("takes the whole area with its stored levels")
        print(f"[server]   promotions: {promoted}", flush=True)
        assert promoted == 1
        srv.close()
        for t, p in zip(tickets, ps):
            same(out[t], s.solve(p, flags=D), p)
    finally:
        s.close()

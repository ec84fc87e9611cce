"""GPU: the paper's 7+7 example (7 positive and 7 negative traces of length 6
over {a, b}; the paper's tool finds a size-16 formula) solved to its minimum
under the paper's grammar {p, not, and, X, F, U} with unit costs and bound 16.

Bar: the solve ends OK with a witness that separates and costs the minimal
cost; the minimal cost is 16, the size of the printed formula (which
separates, pinned on the CPU): every level the oracle reaches in seconds (to
cost 13) has the oracle's count and set (digest), the oracle finds nothing
below 14, and levels 14 and 15, beyond the oracle's reach, hold no separating
formula on the GPU.
"""
from __future__ import annotations

import time

import pytest

import oracle
import paper_2504_18943_amd as m
from oracle import evaluator as ev
from tests import digest
from tests import paper_fixtures as pf

pytestmark = pytest.mark.gpu

UNIT_PAPER = (1, 1, 1, 0, 1, 0, 1)  # not, X, F, (G off), and, (or off), U
ORACLE_BOUND = 13


def test_seven_seven_minimum_under_the_paper_grammar():
    p = pf.spec_problem("seven_seven", 16)
    s = m.Synthesizer(device=0, workspace_bytes=16 << 30)
    try:
        s.solve(p, cost_bound=8, op_cost=UNIT_PAPER)  # warm-up
        a = time.perf_counter()
        r = s.solve(p, cost_bound=16, op_cost=UNIT_PAPER, flags=m.FLAG_DIGEST)
        ms = (time.perf_counter() - a) * 1e3
        print(f"[7+7] status {r.status_name} min cost {r.min_cost} formula {r.formula!r} "
              f"counts {r.level_counts[1:]} candidates {r.candidates} {ms:.1f} ms", flush=True)
        assert r.status == m.ltlf.OK and r.overflow_level == 0
        assert r.min_cost == 16
        assert ev.separates(r.formula, p.traces, p.positive)
        assert ev.cost(r.formula) == r.min_cost
        o = oracle.solve(p, op_cost=UNIT_PAPER, cost_bound=ORACLE_BOUND, exhaust=True)
        assert o.status == oracle.NOT_FOUND and r.min_cost > ORACLE_BOUND
        assert r.level_counts[: ORACLE_BOUND + 1] == o.level_counts
        for c in range(1, ORACLE_BOUND + 1):
            assert r.level_digests[c] == digest.level_digest(o.export_level(c), p.lengths), c
    finally:
        s.close()

"""Kernel autotuning (ltlf_autotune, ltlf_ctx_set_tuning) on the GPU.

The tuning only chooses among generation kernels whose results are
identical, so the bar is: every class gets an applicable kernel that was the
fastest measured, and runs with a tuned (or forced) table stay equal to the
oracle (status, minimal cost, levels, |U_c| per level, witness valid).
"""
from __future__ import annotations

import pytest

import oracle
import paper_2504_18943_amd as m
import workload
from oracle import evaluator as ev
from paper_2504_18943_amd import ltlf as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def synth():
    s = m.Synthesizer(device=0, workspace_bytes=64 << 30)
    yield s
    s.close()


def check(s, p, bound, exhaust=True):
    r = s.solve(p, cost_bound=bound, flags=m.FLAG_EXHAUST if exhaust else 0)
    o = oracle.solve(p, cost_bound=bound, exhaust=exhaust)
    assert (r.status, r.min_cost, r.levels_done, r.overflow_level) == \
        (o.status, o.min_cost, o.levels_done, o.overflow_level), (p.name, r, o)
    assert r.level_counts[: o.levels_done + 1] == o.level_counts[: o.levels_done + 1], p.name
    if r.status == L.OK:
        assert ev.separates(r.formula, p.traces, p.positive) and ev.cost(r.formula) == r.min_cost


def test_autotune_table_and_parity(synth):
    print("[tune] autotune", flush=True)
    table = synth.autotune()
    print("[tune]", table, flush=True)
    assert [e["chunks"] for e in table] == [1, 2, 4, 8, 10, 16, 24, 32, 38, 48, 64, 96, 128, 256, 328]
    for e in table:
        ns = e["ns_per_candidate"]
        assert ns[e["kernel"]] is not None and ns[e["kernel"]] > 0, e
        # the fastest, or the built-in choice within 5% of it
        assert ns[e["kernel"]] <= 1.05 * min(v for v in ns.values() if v is not None), e
        assert e["candidates"] > 0
        if e["chunks"] == 1:
            assert ns["group"] is None  # groups need two chunks or more
        if e["chunks"] > 64:
            assert ns["group"] is None and ns["lane"] is None and e["kernel"] == "wave"
    for p, b in [(workload.tiny(1), 7), (workload.tiny(2), 7), (workload.medium(2), 6)]:
        check(synth, p, b)
    synth.set_tuning(None)


def test_forced_table_parity(synth):
    """A table that names the wave kernel for every width, then the group
    kernel: both still give the oracle's result."""
    for flag in (m.FLAG_KERNEL_WAVE, m.FLAG_KERNEL_GROUP):
        t = L.ltlf_tuning()
        t.n_classes = 2
        t.chunks[0], t.kernel[0] = 1, flag
        t.chunks[1], t.kernel[1] = 400, flag
        synth.set_tuning(t)
        try:
            for p, b in [(workload.tiny(3), 7), (workload.medium(3), 6)]:
                check(synth, p, b)
        finally:
            synth.set_tuning(None)


def test_invalid_tables_rejected(synth):
    t = L.ltlf_tuning()
    t.n_classes = 1
    t.chunks[0], t.kernel[0] = 4, 0x40
    with pytest.raises(m.LtlfError):
        synth.set_tuning(t)
    t.kernel[0], t.chunks[0] = m.FLAG_KERNEL_WAVE, 0
    with pytest.raises(m.LtlfError):
        synth.set_tuning(t)
    t.n_classes = 17
    with pytest.raises(m.LtlfError):
        synth.set_tuning(t)

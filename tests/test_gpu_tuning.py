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
from tests import digest

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
        # the wave kernel's pair tile: the fastest side, or the built-in 16 within 5% of it
        wt = e["ns_wave_tile"]
        assert e["wave_tile"] in (8, 16, 32) and all(v > 0 for v in wt.values()), e
        assert wt[e["wave_tile"]] <= 1.05 * min(wt.values()), e
        assert ns["wave"] == wt[e["wave_tile"]], e
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


def test_wave_tiles_parity(synth):
    """Tables that name the wave kernel with pair tiles of side 8 and 32 for
    every width: the oracle's result, counts and sets (digests); and past an
    overflow of the level below the minimum, the look-ahead (which plans with
    the same tile) finds the oracle's minimum."""
    for tile in (8, 32):
        t = L.ltlf_tuning()
        t.n_classes = 2
        for i, ch in enumerate((1, 400)):
            t.chunks[i], t.kernel[i], t.wave_tile[i] = ch, m.FLAG_KERNEL_WAVE, tile
        synth.set_tuning(t)
        try:
            print(f"[tune] wave tile {tile}", flush=True)
            for p, b in [(workload.tiny(1), 8), (workload.medium(3), 8)]:
                r = synth.solve(p, cost_bound=b, flags=m.FLAG_EXHAUST | m.FLAG_DIGEST)
                o = oracle.solve(p, cost_bound=b, exhaust=True)
                assert (r.status, r.min_cost, r.levels_done) == (o.status, o.min_cost, o.levels_done), (p.name, r, o)
                assert r.level_counts[: o.levels_done + 1] == o.level_counts[: o.levels_done + 1], p.name
                for c in range(1, o.levels_done + 1):
                    assert r.level_digests[c] == digest.level_digest(o.export_level(c), p.lengths), (p.name, c)
            p = workload.tiny(1)
            full = oracle.solve(p, cost_bound=p.cost_bound + 2)
            c = full.min_cost - 1
            assert full.status == oracle.OK and full.level_counts[c] >= 2
            cap = sum(full.level_counts[1:c]) + full.level_counts[c] - 1
            synth.set_row_limit(cap)
            try:
                r = synth.solve(p, cost_bound=p.cost_bound + 2)
            finally:
                synth.set_row_limit(0)
            o = oracle.solve(p, cost_bound=p.cost_bound + 2, max_rows=cap)
            assert (r.status, r.min_cost, r.overflow_level, r.checked_level) == \
                (o.status, o.min_cost, o.overflow_level, o.checked_level), (tile, r, o)
            assert r.overflow_level == c and r.status == L.OK and r.min_cost == full.min_cost
            assert ev.separates(r.formula, p.traces, p.positive) and ev.cost(r.formula) == r.min_cost
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
    t.chunks[0], t.wave_tile[0] = 4, 12
    with pytest.raises(m.LtlfError):
        synth.set_tuning(t)
    t.wave_tile[0] = 0
    t.n_classes = 17
    with pytest.raises(m.LtlfError):
        synth.set_tuning(t)

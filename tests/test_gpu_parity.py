"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar (integer/bit work, so exact): status, minimal cost, levels_done,
overflow level, |U_c| for every stored level, and the set of canonical CMs of
every stored level must be identical; the returned witness must separate the
specification under the definitional evaluator and cost exactly the minimal
cost (several witnesses can be correct, so only those properties are checked).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_2504_18943_amd as m
import workload
from oracle import evaluator as ev
from tests import paper_fixtures as pf

pytestmark = pytest.mark.gpu

OP_INDEX = {"!": 0, "X": 1, "F": 2, "G": 3, "&": 4, "|": 5, "U": 6}


def sorted_rows(a: np.ndarray) -> np.ndarray:
    if len(a) == 0:
        return a
    return a[np.lexsort(a.T[::-1])]


def compare(synth, p, bound, op_cost=oracle.UNIT_ALL, atom_cost=1, exhaust=False, flags=0,
            row_limit=0, check_sets=True):
    print(f"[parity] {p.name or 'problem'} bound={bound} ops={op_cost} atom={atom_cost} "
          f"exhaust={exhaust} flags={flags:#x} row_limit={row_limit}", flush=True)
    synth.set_row_limit(row_limit)
    fl = flags | (m.FLAG_EXHAUST if exhaust else 0)
    r = synth.solve(p, cost_bound=bound, op_cost=op_cost, atom_cost=atom_cost, flags=fl)
    synth.set_row_limit(0)
    o = oracle.solve(p, op_cost=op_cost, atom_cost=atom_cost, cost_bound=bound, exhaust=exhaust,
                     max_rows=row_limit, lookahead=not (flags & m.FLAG_NO_LOOKAHEAD))
    assert (r.status, r.min_cost, r.levels_done, r.overflow_level, r.checked_level) == \
        (o.status, o.min_cost, o.levels_done, o.overflow_level, o.checked_level), (r, o)
    assert r.level_counts[: o.levels_done + 1] == o.level_counts[: o.levels_done + 1]
    if check_sets:
        for c in range(1, o.levels_done + 1):
            g = sorted_rows(synth.export_level(c))
            w = sorted_rows(o.export_level(c))
            assert g.shape == w.shape, f"level {c}: {g.shape} vs {w.shape}"
            assert np.array_equal(g, w), f"level {c} sets differ"
    if r.status == m.ltlf.OK:
        kappa = {k: op_cost[i] for k, i in OP_INDEX.items()}
        assert ev.separates(r.formula, p.traces, p.positive), r.formula
        assert ev.cost(r.formula, atom_cost, kappa) == r.min_cost, r.formula
    return r, o


@pytest.mark.parametrize("seed", range(1, 17))
def test_tiny_plain(synth, seed):
    p = workload.tiny(seed)
    compare(synth, p, p.cost_bound)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_tiny_exhaustive(synth, seed):
    compare(synth, workload.tiny(seed), 8, exhaust=True)


@pytest.mark.parametrize("seed", [1, 2])
def test_tiny_exhaustive_wave(synth, seed):
    """One-chunk rows through the wave kernel (63 of 64 lanes past the row)."""
    compare(synth, workload.tiny(seed), 8, exhaust=True, flags=m.FLAG_KERNEL_WAVE)


@pytest.mark.parametrize("seed", [1, 2])
def test_large_exhaustive(synth, seed):
    """The large configuration (1024 traces, ~41,000 bits per CM: 328 chunks,
    six 64-chunk steps per row) to cost 5, every level compared."""
    compare(synth, workload.large(seed), 5, exhaust=True)


def test_large_weak_hash(synth):
    """Wide rows with every probe meeting an equal tag: the wave kernel's
    verification passes and the wave verification kernel carry the work."""
    compare(synth, workload.large(3), 4, exhaust=True, flags=m.FLAG_WEAK_HASH)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_medium_plain(synth, seed):
    p = workload.medium(seed)
    compare(synth, p, p.cost_bound)


KERNELS = pytest.mark.parametrize("kflag", [0, m.FLAG_KERNEL_LANE, m.FLAG_KERNEL_GROUP, m.FLAG_KERNEL_WAVE],
                                  ids=["default", "lane", "group", "wave"])


@KERNELS
def test_medium_exhaustive_to_8(synth, kflag):
    compare(synth, workload.medium(1), 8, exhaust=True, flags=kflag)


@pytest.mark.parametrize("ops", [oracle.UNIT_ALL, oracle.UNIT_PAPER], ids=["all", "paper"])
def test_paper_small_spec(synth, ops):
    r, _ = compare(synth, pf.spec_problem("small_spec", 8), 8, op_cost=ops)
    assert r.min_cost == 4


def test_paper_seven_seven_prefix(synth):
    """The paper's 7+7 example: every level up to 10 identical (no separator yet)."""
    r, _ = compare(synth, pf.spec_problem("seven_seven", 10), 10)
    assert r.status == m.ltlf.NOT_FOUND


@pytest.mark.parametrize("costs", [((2, 1, 3, 1, 2, 2, 3), 1), ((1, 1, 1, 1, 1, 1, 1), 2),
                                   ((1, 0, 1, 0, 1, 0, 1), 1), ((0, 1, 1, 0, 1, 1, 0), 1)],
                         ids=["mixed", "atom2", "paper", "no-not-no-U"])
def test_nonunit_costs(synth, costs):
    ops, ac = costs
    compare(synth, workload.tiny(5), 9, op_cost=ops, atom_cost=ac, exhaust=True)


@pytest.mark.parametrize("seed", [1, 2])
def test_weak_hash_forces_collisions(synth, seed):
    """Every candidate lands in a few slots with one tag: the verify and defer
    paths carry all the work; the sets must not change."""
    compare(synth, workload.tiny(seed), 5, exhaust=True, flags=m.FLAG_WEAK_HASH)


@KERNELS
@pytest.mark.parametrize("seed", [2, 3])
def test_weak_hash_wide_rows(synth, seed, kflag):
    """The same stress on 40-word rows, for each generation kernel."""
    compare(synth, workload.medium(seed), 5, exhaust=True, flags=m.FLAG_WEAK_HASH | kflag)


@pytest.mark.parametrize("problem", ["tiny", "medium"])
@pytest.mark.parametrize("kflag", [0, m.FLAG_KERNEL_GROUP, m.FLAG_KERNEL_WAVE], ids=["default", "group", "wave"])
def test_row_limit_matches_oracle_capacity(synth, problem, kflag):
    p = workload.tiny(3) if problem == "tiny" else workload.medium(3)
    full = oracle.solve(p, cost_bound=7, exhaust=True)
    cap = sum(full.level_counts[:5]) + 3
    r, o = compare(synth, p, 7, exhaust=True, row_limit=cap, flags=kflag)
    assert r.overflow_level == 5


def test_row_limit_check_only_level_finds_min(synth):
    p = workload.tiny(1)
    full = oracle.solve(p)
    cap = sum(full.level_counts[: full.min_cost]) + 5
    r, o = compare(synth, p, p.cost_bound, row_limit=cap)
    assert r.status == m.ltlf.OK and r.min_cost == full.min_cost


LOOKAHEAD_CASES = [
    # (problem, op_cost, atom_cost)
    ("tiny1", oracle.UNIT_ALL, 1),
    ("tiny5", oracle.UNIT_ALL, 1),
    ("unary-root", oracle.UNIT_ALL, 1),
    ("medium2", oracle.UNIT_ALL, 1),
    ("tiny2", (2, 1, 3, 1, 2, 2, 3), 1),   # unary operators of cost 2 and 3 over stored levels
    ("tiny3", (1, 0, 1, 0, 1, 1, 0), 1),   # X, G, U disabled
    ("tiny14", (1, 1, 1, 1, 1, 1, 1), 2),  # atoms cost 2; minimum X & p1 ! X p1
]


def lookahead_problem(name):
    if name == "unary-root":  # minimum G ! & p0 p1: a cost-1 operator over the overflowed level
        return workload.custom(2, [[1, 2, 1], [2, 0]], [[3, 0], [0, 3], [1, 3]], 6, name="unary-root")
    if name.startswith("medium"):
        return workload.medium(int(name[6:]))
    return workload.tiny(int(name[4:]))


@pytest.mark.parametrize("case", LOOKAHEAD_CASES, ids=[c[0] + f"-{i}" for i, c in enumerate(LOOKAHEAD_CASES)])
@pytest.mark.parametrize("kflag", [0, m.FLAG_KERNEL_GROUP, m.FLAG_KERNEL_WAVE], ids=["default", "group", "wave"])
def test_lookahead_past_overflow(synth, case, kflag):
    """The level below the minimum overflows: the minimum is still found,
    in the next level, by the look-ahead (status, cost, checked level equal
    to the oracle's; the witness separates and costs the minimum)."""
    name, ops, ac = case
    p = lookahead_problem(name)
    full = oracle.solve(p, op_cost=ops, atom_cost=ac, cost_bound=p.cost_bound + 2)  # levels up to the minimum
    want = full.min_cost
    assert full.status == oracle.OK and want >= ac + 1
    c = want - 1
    if full.level_counts[c] < 2:
        pytest.skip("the level below the minimum has fewer than two rows")
    cap = sum(full.level_counts[1:c]) + full.level_counts[c] - 1
    r, o = compare(synth, p, p.cost_bound + 2, op_cost=ops, atom_cost=ac, row_limit=cap, flags=kflag)
    assert r.overflow_level == c and r.status == m.ltlf.OK and r.min_cost == want
    assert r.checked_level == want
    r, o = compare(synth, p, p.cost_bound + 2, op_cost=ops, atom_cost=ac, row_limit=cap,
                   flags=kflag | m.FLAG_NO_LOOKAHEAD)
    assert r.status == m.ltlf.CAPACITY and r.checked_level == c


@pytest.mark.parametrize("kflag", [0, m.FLAG_KERNEL_WAVE], ids=["default", "wave"])
def test_lookahead_without_solution_is_capacity(synth, kflag):
    """Overflow two levels below the minimum: the look-ahead checks the next
    level in full and finds nothing, so the run reports CAPACITY with every
    level up to overflow + 1 checked."""
    p = workload.tiny(1)
    full = oracle.solve(p, cost_bound=p.cost_bound)
    c = full.min_cost - 2
    cap = sum(full.level_counts[1:c]) + full.level_counts[c] - 1
    r, o = compare(synth, p, p.cost_bound, row_limit=cap, flags=kflag)
    assert r.status == m.ltlf.CAPACITY and r.overflow_level == c and r.checked_level == c + 1


def test_lookahead_over_the_atoms_level(synth):
    """The atoms' level itself overflows: the look-ahead's operands are the
    atoms."""
    p = workload.custom(2, [[0, 1], [1]], [[2, 1], [3]], 4, name="not-p1")
    full = oracle.solve(p, cost_bound=4, exhaust=True)
    assert full.min_cost == 2
    r, o = compare(synth, p, 4, row_limit=1)
    assert r.overflow_level == 1 and r.status == m.ltlf.OK and r.min_cost == 2


def test_edge_single_position(synth):
    p = workload.custom(1, [[1]], [], 4, name="one-position")
    r, _ = compare(synth, p, 4, exhaust=True)
    assert r.min_cost == 1


def test_edge_contradiction_not_found(synth):
    tr = [1, 3, 0, 2]
    p = workload.custom(2, [tr, [1]], [tr], 6, name="contradiction")
    r, _ = compare(synth, p, 6)
    assert r.status == m.ltlf.NOT_FOUND and r.levels_done == 6


def test_edge_only_negatives(synth):
    p = workload.custom(2, [], [[1, 2, 3], [0, 1]], 5, name="only-negatives")
    compare(synth, p, 5)


def test_edge_32_props(synth):
    rng = np.random.Generator(np.random.PCG64(5))
    trs = [[int(x) for x in rng.integers(0, 2**32, size=int(rng.integers(1, 6)), dtype=np.uint64)]
           for _ in range(6)]
    p = workload.custom(32, trs[:3], trs[3:], 3, name="32-props")
    compare(synth, p, 3, exhaust=True)


def test_edge_long_traces_cross_words(synth):
    """Segments far longer than a word: F, G, U and X carries cross words."""
    rng = np.random.Generator(np.random.PCG64(9))
    trs = [[int(x) for x in rng.integers(0, 4, size=n)] for n in (300, 97, 1, 64, 33)]
    p = workload.custom(2, trs[:2], trs[2:], 5, name="long")
    compare(synth, p, 5, exhaust=True)


@pytest.mark.parametrize("shape", [(8, 8, 2, 6), (16, 16, 3, 9), (20, 20, 8, 16), (30, 30, 16, 24),
                                   (40, 40, 40, 64), (48, 48, 40, 64), (60, 60, 60, 64), (90, 90, 60, 64)],
                         ids=["rows-1q", "rows-2q", "rows-5q", "rows-16q", "rows-33q", "rows-40q", "rows-60q",
                              "rows-90q"])
@KERNELS
def test_edge_row_widths(synth, shape, kflag):
    """Row widths across the lane kernel's LDS limits (256-lane tiles up to
    ~37 chunks, 128-lane tiles up to ~67 under the lane flag), the group
    sizes (4..64 lanes per candidate) and past them (wave kernel)."""
    npos, nneg, lo, hi = shape
    p = workload.make_problem(21, 3, npos, nneg, lo, hi, 5, 5, q_range=(0.3, 0.7), name=f"wide{hi}")
    compare(synth, p, 4, exhaust=True, flags=kflag)


def test_repeat_runs_identical(synth):
    p = workload.tiny(7)
    a = synth.solve(p, cost_bound=7, flags=m.FLAG_EXHAUST)
    sets_a = [sorted_rows(synth.export_level(c)) for c in range(1, a.levels_done + 1)]
    b = synth.solve(p, cost_bound=7, flags=m.FLAG_EXHAUST)
    sets_b = [sorted_rows(synth.export_level(c)) for c in range(1, b.levels_done + 1)]
    assert a.level_counts == b.level_counts
    for x, y in zip(sets_a, sets_b):
        assert np.array_equal(x, y)


def test_formula_of_rows(synth):
    """Every stored representative's formula re-evaluates to its exported CM
    and costs its level."""
    p = workload.tiny(2)
    r = synth.solve(p, cost_bound=5, flags=m.FLAG_EXHAUST)
    for c in range(1, r.levels_done + 1):
        rows = synth.export_level(c)
        for i in range(len(rows)):
            f = synth.formula_of(c, i)
            assert ev.cost(f) == c
            want = ev.canonical_words(ev.characteristic_matrix(f, p.traces))
            assert [int(x) for x in rows[i]] == want


def test_invalid_arguments(synth):
    bad = workload.Problem(n_props=2, traces=[[1], []], positive=[1, 0], cost_bound=4)
    with pytest.raises(m.LtlfError) as e:
        synth.load(bad)
    assert e.value.status == m.ltlf.EINVAL
    bad2 = workload.Problem(n_props=2, traces=[[4]], positive=[1], cost_bound=4)
    with pytest.raises(m.LtlfError):
        synth.load(bad2)
    synth.load(workload.tiny(1))
    with pytest.raises(m.LtlfError):
        synth.run(0)
    with pytest.raises(m.LtlfError):
        synth.run(2000)
    with pytest.raises(m.LtlfError):
        synth.run(4, atom_cost=0)


def test_formula_buffer_too_small(synth):
    import ctypes
    from paper_2504_18943_amd import ltlf as L
    p = workload.tiny(1)
    synth.load(p)
    res = L.ltlf_result()
    buf = ctypes.create_string_buffer(3)
    res.formula = ctypes.cast(buf, ctypes.c_char_p)
    res.formula_cap = 3
    st = L.ltlf_run(synth._ctx, oracle.UNIT_ALL, 1, 10, 0, synth._stream(), res)
    assert st == L.EBUFSZ
    assert res.formula_len > 3 and res.min_cost == 7


def test_wide_rows_kernels_agree_beyond_the_oracle():
    """40-chunk rows (the lane kernel's 128-lane tiles by default): up to cost
    11 (~6e6 CMs at the top level) the lane, group and wave kernels, three
    independent generators, must give identical level counts, and identical
    CM sets for every level up to 9; levels up to 7 also equal the oracle."""
    p = workload.make_problem(22, 3, 48, 48, 40, 64, 9, 9, q_range=(0.3, 0.7), name="wide40")
    s = m.Synthesizer(device=0, workspace_bytes=16 << 30)
    try:
        runs = {}
        for name, fl in (("lane", m.FLAG_KERNEL_LANE), ("group", m.FLAG_KERNEL_GROUP), ("wave", m.FLAG_KERNEL_WAVE)):
            print(f"[parity] wide40 bound 11 kernel {name}", flush=True)
            r = s.solve(p, cost_bound=11, flags=m.FLAG_EXHAUST | fl)
            assert r.levels_done == 11 and r.overflow_level == 0, (name, r)
            runs[name] = (r, [sorted_rows(s.export_level(c)) for c in range(1, 10)])
        base_r, base_sets = runs["lane"]
        assert base_r.level_counts[11] > 1_000_000
        for name, (r, sets) in runs.items():
            assert (r.status, r.min_cost, r.level_counts) == (base_r.status, base_r.min_cost, base_r.level_counts), name
            for c, (a, b) in enumerate(zip(sets, base_sets), start=1):
                assert np.array_equal(a, b), (name, c)
        o = oracle.solve(p, cost_bound=7, exhaust=True)
        assert base_r.level_counts[:8] == o.level_counts[:8]
        for c in range(1, 8):
            assert np.array_equal(base_sets[c - 1], sorted_rows(o.export_level(c))), c
    finally:
        s.close()

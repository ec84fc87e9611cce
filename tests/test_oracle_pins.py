"""Pins of the CPU oracle to facts fixed by the paper and by the definitions.

Nothing here compares the oracle with itself: every expected value is a value
the paper prints (tests/golden/), a closed form, a brute-force enumeration of
syntax trees evaluated from the quantifier definitions, or an invariant.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workload
from oracle import brute
from oracle import evaluator as ev
from tests import paper_fixtures as pf


def bits_str(vec):
    return "".join("1" if b else "0" for b in vec)


# ------------------------------------------------------------- paper values --
def test_bitwise_example_evaluator():
    d = pf.load()["bitwise_example"]
    tr = pf.trace_masks(d["trace"], d["props"])
    for f, want in d["cs"].items():
        assert bits_str(ev.vector(pf.formula_tokens(f, d["props"]), tr)) == want


def test_bitwise_example_oracle_levels(oracle_lib):
    """The oracle's level sets over the single trace abcaa contain the printed
    characteristic sequences at the right cost."""
    d = pf.load()["bitwise_example"]
    tr = pf.trace_masks(d["trace"], d["props"])
    p = workload.custom(3, [tr], [], 2)
    r = oracle.solve(p, cost_bound=2, exhaust=True)
    lv1 = {tuple(int(x) for x in row) for row in r.export_level(1)}
    lv2 = {tuple(int(x) for x in row) for row in r.export_level(2)}
    enc = lambda s: tuple(ev.canonical_words([[c == "1" for c in s]]))  # noqa: E731
    assert enc(d["cs"]["a"]) in lv1
    assert enc(d["cs"]["X a"]) in lv2
    assert enc(d["cs"]["! a"]) in lv2


def test_squeegee_facts():
    d = pf.load()["squeegee"]
    tr = pf.trace_masks(d["trace"], d["props"])
    for fact in d["facts"]:
        f = pf.formula_tokens(fact["formula"], d["props"])
        assert ev.holds(f, tr, fact["pos"]) == fact["holds"], fact
        assert ev.vector(f, tr)[fact["pos"]] == fact["holds"], fact


@pytest.mark.parametrize("ops", [oracle.UNIT_ALL, oracle.UNIT_PAPER])
def test_small_spec_min_size_4(oracle_lib, ops):
    d = pf.load()["small_spec"]
    p = pf.spec_problem("small_spec", 8)
    f = pf.formula_tokens(d["formula"], d["props"])
    assert ev.separates(f, p.traces, p.positive)
    assert ev.cost(f) == d["min_size"]
    r = oracle.solve(p, op_cost=ops)
    assert r.status == oracle.OK and r.min_cost == d["min_size"]
    assert ev.separates(r.witness, p.traces, p.positive)
    assert ev.cost(r.witness) == d["min_size"]
    assert brute.min_separating_cost(p.n_props, p.traces, p.positive, 4, op_cost=ops) == 4


def test_small_spec_paper_grammar_unique_separator():
    """Under the printed grammar (p, not, and, X, F, U) the size-4 separators
    all have the CM of not(b U a)."""
    d = pf.load()["small_spec"]
    p = pf.spec_problem("small_spec", 4)
    by_cost, mincost = brute.level_sets(p.n_props, p.traces, 4, op_cost=oracle.UNIT_PAPER)
    want = tuple(bool(x) for x in p.positive)
    seps = [cm for cm in by_cost[4] if tuple(cs[0] for cs in cm) == want]
    target = ev.characteristic_matrix(pf.formula_tokens(d["formula"], d["props"]), p.traces)
    assert seps == [target]


def test_seven_seven_formula_separates():
    d = pf.load()["seven_seven"]
    p = pf.spec_problem("seven_seven", 16)
    f = pf.formula_tokens(d["formula"], d["props"])
    assert ev.cost(f) == d["size"] == 16
    assert ev.separates(f, p.traces, p.positive)


def test_seven_seven_no_small_separator(oracle_lib):
    """Consistent with the paper's size-16 minimum: nothing of cost <= 9
    separates (under either operator set)."""
    p = pf.spec_problem("seven_seven", 9)
    for ops in (oracle.UNIT_ALL, oracle.UNIT_PAPER):
        r = oracle.solve(p, op_cost=ops)
        assert r.status == oracle.NOT_FOUND and r.levels_done == 9


# ------------------------------------------------ the paper's log-step F ----
def _paper_F(word: int) -> int:
    """The paper's branch-free F on one 64-bit characteristic sequence:
    six rounds of cs |= cs << 2^k (position 0 in the most significant bit)."""
    m = (1 << 64) - 1
    for s in (1, 2, 4, 8, 16, 32):
        word = (word | (word << s)) & m
    return word


@pytest.mark.parametrize("seed", range(6))
def test_oracle_F_equals_paper_log_step(oracle_lib, seed):
    """A trace of length n <= 64 stored as the top n bits of a word: the
    doubling rounds give the same F as the oracle's level-2 set contains."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.integers(1, 65))
    tr = [int(x) for x in rng.integers(0, 2, size=n)]
    word = sum(tr[k] << (63 - k) for k in range(n))
    fw = _paper_F(word)
    want = [bool((fw >> (63 - k)) & 1) for k in range(n)]
    assert want == ev.vector("F p0", tr)
    p = workload.custom(1, [tr], [], 2)
    r = oracle.solve(p, cost_bound=2, exhaust=True)
    lv = {tuple(int(x) for x in row) for row in r.export_level(2)} | \
         {tuple(int(x) for x in row) for row in r.export_level(1)}
    assert tuple(ev.canonical_words([want])) in lv


def test_F_is_linear_disjunction():
    """F phi = phi or X phi or ... or X^(n-1) phi (the paper's argument)."""
    rng = np.random.Generator(np.random.PCG64(7))
    for _ in range(20):
        n = int(rng.integers(1, 12))
        tr = [int(x) for x in rng.integers(0, 4, size=n)]
        disj = "p0"
        for k in range(1, n):
            disj = "| " + disj + " " + " ".join(["X"] * k) + " p0"
        assert ev.vector("F p0", tr) == ev.vector(disj, tr)


# --------------------------------------------- brute force vs the oracle ----
CASES = [
    # (seed, props, traces, len_lo, len_hi, max_cost, op_cost, atom_cost)
    (1, 2, 5, 1, 5, 6, oracle.UNIT_ALL, 1),
    (2, 2, 6, 2, 6, 6, oracle.UNIT_ALL, 1),
    (3, 1, 4, 1, 8, 7, oracle.UNIT_ALL, 1),
    (4, 3, 4, 1, 4, 5, oracle.UNIT_ALL, 1),
    (5, 2, 5, 2, 5, 6, oracle.UNIT_PAPER, 1),
    (6, 2, 5, 1, 6, 8, (2, 1, 3, 1, 2, 2, 3), 1),
    (7, 2, 4, 1, 5, 8, (1, 1, 1, 1, 1, 1, 1), 2),
    (8, 1, 3, 1, 3, 6, (1, 0, 1, 0, 1, 1, 0), 1),
]


@pytest.mark.parametrize("case", CASES, ids=[f"case{c[0]}" for c in CASES])
def test_oracle_levels_equal_brute_force(oracle_lib, case):
    seed, props, nt, lo, hi, K, ops, ac = case
    p = workload.random_small(seed, props, nt, lo, hi)
    r = oracle.solve(p, op_cost=ops, atom_cost=ac, cost_bound=K, exhaust=True)
    U = brute.unique_levels(p.n_props, p.traces, K, op_cost=ops, atom_cost=ac)
    for c in range(1, K + 1):
        got = {tuple(int(x) for x in row) for row in r.export_level(c)}
        assert got == U[c], f"level {c}"
        assert r.level_counts[c] == len(U[c])
    want = brute.min_separating_cost(p.n_props, p.traces, p.positive, K, op_cost=ops, atom_cost=ac)
    if want is None:
        assert r.status == oracle.NOT_FOUND
    else:
        assert r.status == oracle.OK and r.min_cost == want


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_every_stored_cm_matches_its_formula(oracle_lib, seed):
    """Each representative's derivation, re-evaluated from the definitions,
    gives the stored CM, costs exactly its level, and no CM repeats."""
    p = workload.tiny(seed)
    r = oracle.solve(p, cost_bound=6, exhaust=True)
    seen = set()
    for c in range(1, r.levels_done + 1):
        rows = r.export_level(c)
        forms = r.formulas_of_level(c)
        assert len(forms) == len(rows) == r.level_counts[c]
        for row, f in zip(rows, forms):
            key = tuple(int(x) for x in row)
            assert key not in seen
            seen.add(key)
            assert ev.cost(f) == c
            assert tuple(ev.canonical_words(ev.characteristic_matrix(f, p.traces))) == key


@pytest.mark.parametrize("seed", range(1, 17))
def test_tiny_planted_bound_and_witness(oracle_lib, seed):
    p = workload.tiny(seed)
    assert ev.separates(workload.to_prefix(p.planted), p.traces, p.positive)
    r = oracle.solve(p)
    assert r.status == oracle.OK
    assert r.min_cost <= p.planted_cost
    assert ev.separates(r.witness, p.traces, p.positive)
    assert ev.cost(r.witness) == r.min_cost


def test_algebraic_duplicates_absorbed(oracle_lib):
    """not not p, F F p, G G p, G = not F not, F = true U p, p U p: none of
    these may add a new class; their CMs are in the sets of their cheaper
    equivalents."""
    p = workload.random_small(11, 2, 6, 2, 7)
    r = oracle.solve(p, cost_bound=5, exhaust=True)
    allcms = {}
    for c in range(1, 6):
        for row in r.export_level(c):
            allcms[tuple(int(x) for x in row)] = c
    cm = lambda f: tuple(ev.canonical_words(ev.characteristic_matrix(f, p.traces)))  # noqa: E731
    assert allcms[cm("! ! p0")] == 1
    assert allcms[cm("F F p0")] == 2
    assert allcms[cm("G G p1")] == 2
    assert cm("G p0") == cm("! F ! p0")
    assert allcms[cm("U p0 p0")] == 1
    assert cm("& p0 p1") == cm("& p1 p0")
    assert allcms[cm("& p0 p1")] == 3


def test_capacity_levels_below_overflow_are_exact(oracle_lib):
    p = workload.tiny(3)
    full = oracle.solve(p, cost_bound=7, exhaust=True)
    cap = sum(full.level_counts[:5]) + 3
    r = oracle.solve(p, cost_bound=7, exhaust=True, max_rows=cap)
    assert r.overflow_level == 5
    assert r.levels_done == 4
    assert r.level_counts[:5] == full.level_counts[:5]
    # level 5 is checked without storing it, level 6 by the look-ahead
    if full.min_cost and full.min_cost <= 6:
        assert r.status == oracle.OK and r.min_cost == full.min_cost
    else:
        assert r.status == oracle.CAPACITY and r.checked_level == 6


def test_capacity_still_finds_min_cost_in_overflow_level(oracle_lib):
    """Check-only candidates of the overflowing level are still tested."""
    p = workload.tiny(1)  # min cost 7
    full = oracle.solve(p)
    assert full.min_cost == 7
    cap = sum(full.level_counts[:7]) + 5  # levels 1..6 fit, level 7 does not
    r = oracle.solve(p, max_rows=cap)
    assert r.status == oracle.OK and r.min_cost == 7 and r.overflow_level == 7
    assert ev.separates(r.witness, p.traces, p.positive) and ev.cost(r.witness) == 7


def test_invalid_inputs(oracle_lib):
    good = workload.tiny(1)
    bad_len = workload.Problem(n_props=2, traces=[[1, 2], []], positive=[1, 0], cost_bound=5)
    assert oracle.solve(bad_len).status == oracle.EINVAL
    bad_letter = workload.Problem(n_props=2, traces=[[4]], positive=[1], cost_bound=5)
    assert oracle.solve(bad_letter).status == oracle.EINVAL
    assert oracle.solve(good, cost_bound=0).status == oracle.EINVAL
    assert oracle.solve(good, atom_cost=0).status == oracle.EINVAL


def test_contradictory_spec_not_found(oracle_lib):
    """The same trace in P and in N can never be separated."""
    tr = [1, 3, 0, 2]
    p = workload.custom(2, [tr, [1]], [tr], 6)
    r = oracle.solve(p)
    assert r.status == oracle.NOT_FOUND and r.levels_done == 6


def _kappa(ops):
    return {k: ops[i] for i, k in enumerate(("!", "X", "F", "G", "&", "|", "U"))}


@pytest.mark.parametrize("case", CASES, ids=[f"case{c[0]}" for c in CASES])
def test_lookahead_past_overflow_equals_brute_force(oracle_lib, case):
    """Overflow forced at every level c in turn: the result must be the
    brute-force minimum whenever it is at most c + 1 (level c checked
    without storing, level c + 1 by the look-ahead), else CAPACITY with
    every candidate up to c + 1 tested."""
    seed, props, nt, lo, hi, K, ops, ac = case
    p = workload.random_small(seed, props, nt, lo, hi)
    full = oracle.solve(p, op_cost=ops, atom_cost=ac, cost_bound=K, exhaust=True)
    want = brute.min_separating_cost(p.n_props, p.traces, p.positive, K, op_cost=ops, atom_cost=ac)
    outer_found = 0
    for c in range(1, K):
        if full.level_counts[c] == 0 or (want is not None and want < c):
            continue
        cap = sum(full.level_counts[1:c]) + full.level_counts[c] - 1
        if cap == 0:  # 0 means no limit
            continue
        r = oracle.solve(p, op_cost=ops, atom_cost=ac, cost_bound=K, max_rows=cap)
        assert r.overflow_level == c and r.levels_done == c - 1, (c, r)
        assert r.checked_level == c + 1 or (want == c and r.checked_level == c), (c, r)
        if want is not None and want <= c + 1:
            assert r.status == oracle.OK and r.min_cost == want, (c, r)
            assert ev.separates(r.witness, p.traces, p.positive), r.witness
            assert ev.cost(r.witness, ac, _kappa(ops)) == want, r.witness
            outer_found += want == c + 1
            # without the look-ahead the same run stops at the overflowed level
            plain = oracle.solve(p, op_cost=ops, atom_cost=ac, cost_bound=K, max_rows=cap, lookahead=False)
            assert plain.checked_level == c
            assert plain.status == (oracle.OK if want == c else oracle.CAPACITY)
        else:
            assert r.status == oracle.CAPACITY, (c, r)
    if want is not None and want >= 2 and full.level_counts[want - 1] > 0:
        assert outer_found == 1


def test_lookahead_finds_unary_root_over_unstored_level(oracle_lib):
    """A minimal formula whose root is a cost-1 unary operator over a formula
    of the overflowed level (the regenerated-operand path)."""
    # one positive trace where p0 and p1 never hold together; negatives where
    # they do at the first position or later: ! F & p0 p1 costs 5
    p = workload.custom(2, [[1, 2, 1], [2, 0]], [[3, 0], [0, 3], [1, 3]], 6)
    want = brute.min_separating_cost(p.n_props, p.traces, p.positive, 6)
    full = oracle.solve(p, cost_bound=6, exhaust=True)
    assert full.min_cost == want
    c = want - 1
    cap = sum(full.level_counts[1:c]) + full.level_counts[c] - 1
    r = oracle.solve(p, cost_bound=6, max_rows=cap)
    assert r.status == oracle.OK and r.min_cost == want and r.overflow_level == c
    assert ev.separates(r.witness, p.traces, p.positive)
    assert ev.cost(r.witness) == want
    root, rest = r.witness.split(" ", 1)
    assert root in ("!", "X", "F", "G") and ev.cost(rest) == c, r.witness

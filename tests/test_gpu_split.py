"""Divide-and-conquer synthesis (ltlf_solve_split) on the GPU.

The recombined formula is not minimal, so there is no oracle value for it;
the bar is: the formula separates the specification under the definitional
evaluator, its cost is the reported cost, and, where the split is one level
deep, that cost is the recombination's cost over the oracle's minimal costs
of the four parts (so every part was solved minimally).
"""
from __future__ import annotations

import pytest

import oracle
import paper_2504_18943_amd as m
import workload
from oracle import evaluator as ev

pytestmark = pytest.mark.gpu

OPS = ("!", "X", "F", "G", "&", "|", "U")


@pytest.fixture(scope="module")
def synth():
    s = m.Synthesizer(device=0, workspace_bytes=8 << 30)
    yield s
    s.close()


def halves(v):
    h = (len(v) + 1) // 2
    return v[:h], v[h:]


def part(p, pos, neg, name):
    return workload.custom(p.n_props, [p.traces[i] for i in pos], [p.traces[i] for i in neg], p.cost_bound,
                           name=name)


def check_formula(p, r, op_cost=oracle.UNIT_ALL, atom_cost=1):
    assert r.status == m.ltlf.OK, r
    assert ev.separates(r.formula, p.traces, p.positive), r.formula
    assert ev.cost(r.formula, atom_cost, dict(zip(OPS, op_cost))) == r.cost, r.formula


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_one_split_recombines_minimal_parts(synth, seed):
    p = workload.tiny(seed)
    print(f"[split] {p.name} one level", flush=True)
    r = synth.solve_split(p, max_traces=len(p.traces) - 1)
    check_formula(p, r)
    assert (r.depth, r.parts_split, r.parts_solved) == (1, 1, 4)
    P = [i for i, lab in enumerate(p.positive) if lab]
    N = [i for i, lab in enumerate(p.positive) if not lab]
    (P1, P2), (N1, N2) = halves(P), halves(N)
    mins = [oracle.solve(part(p, a, b, f"{p.name}/{k}")).min_cost
            for k, (a, b) in enumerate([(P1, N1), (P1, N2), (P2, N1), (P2, N2)])]
    assert all(mins)
    assert r.cost == 3 + sum(mins)  # (phi11 & phi12) | (phi21 & phi22)
    assert r.max_part_cost == max(mins)


def test_recursive_split_of_a_medium_problem(synth):
    p = workload.medium(1)
    print(f"[split] {p.name} max_traces 8", flush=True)
    r = synth.solve_split(p, max_traces=8)
    check_formula(p, r)
    # 64 traces, 32 + 32: three rounds of four-way splits before any solve
    assert r.parts_split == 1 + 4 + 16 and r.parts_solved == 64 and r.depth == 1


def test_split_after_capacity(synth):
    """The whole problem overflows a small row limit; its parts fit."""
    p = workload.tiny(1)
    full = oracle.solve(p)
    assert full.min_cost == 7
    cap = sum(full.level_counts[1:5]) + full.level_counts[5] // 2
    print(f"[split] {p.name} row limit {cap}", flush=True)
    synth.set_row_limit(cap)
    try:
        alone = synth.solve(p)
        r = synth.solve_split(p)
    finally:
        synth.set_row_limit(0)
    assert alone.status == m.ltlf.CAPACITY and alone.checked_level == 6
    check_formula(p, r)
    assert r.parts_split >= 1 and r.depth >= 2


def test_paper_grammar_writes_or_as_de_morgan(synth):
    """Without | in the grammar, the recombination's disjunction is
    ! & ! a ! b."""
    p = workload.tiny(2)
    print(f"[split] {p.name} paper grammar", flush=True)
    r = synth.solve_split(p, max_traces=len(p.traces) - 1, op_cost=oracle.UNIT_PAPER)
    check_formula(p, r, op_cost=oracle.UNIT_PAPER)
    assert "|" not in r.formula and r.formula.startswith("! & !")


def test_positives_only_split_is_a_disjunction(synth):
    p = workload.custom(2, [[1, 0], [2, 2], [3], [0, 1]], [], 6, name="positives-only")
    print(f"[split] {p.name}", flush=True)
    r = synth.solve_split(p, max_traces=2)
    check_formula(p, r)
    assert r.formula.startswith("|") and r.parts_split == 1 and r.parts_solved == 2


def test_unsplittable_contradiction_not_found(synth):
    tr = [1, 3, 0]
    p = workload.custom(2, [tr], [tr], 6, name="contradiction")
    print(f"[split] {p.name}", flush=True)
    r = synth.solve_split(p, max_traces=1)
    assert r.status == m.ltlf.NOT_FOUND and r.formula == ""


def test_split_rejects_grammar_without_conjunction(synth):
    p = workload.tiny(1)
    with pytest.raises(m.LtlfError):
        synth.solve_split(p, op_cost=(0, 1, 1, 1, 0, 1, 1))


def test_no_split_needed_is_the_minimal_solve(synth):
    """Without a trace limit and with a solvable part, the recursion ends at
    the root: one part, no split, the minimal cost of the plain solve."""
    p = workload.tiny(4)
    print(f"[split] {p.name} unsplit", flush=True)
    r = synth.solve_split(p)
    o = oracle.solve(p)
    assert (r.parts_solved, r.parts_split, r.depth) == (1, 0, 1)
    assert r.cost == o.min_cost and r.max_part_cost == o.min_cost
    check_formula(p, r)

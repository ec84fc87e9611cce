"""Exhaustive syntactic enumeration for tiny inputs -- TEST INFRASTRUCTURE ONLY.

Enumerates every formula tree of cost <= K (no semantic deduplication, no
pruning), computes its characteristic matrix with the quantifier definitions
of :mod:`oracle.evaluator`, and derives from that, by definition:

* ``mincost[cm]`` = the least cost of any tree whose CM is cm;
* ``U_c = {cm : mincost[cm] == c}``;
* the least cost of a separating tree.

Trees are grouped by cost; a tree of cost c is an atom (c = atom cost), a
unary operator over any tree of cost c - k, or a binary operator over any
pair of trees whose costs sum to c - k.  Only the CM of each tree is kept
(with multiplicity collapsed), which is exact because the CM of op(f, g) is a
function of the CMs of f and g (compositionality of the satisfaction
relation).
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Set, Tuple

from . import evaluator as ev

OPS = ("!", "X", "F", "G", "&", "|", "U")


def _cm_of_atom(p: int, traces) -> tuple:
    return tuple(tuple(bool((x >> p) & 1) for x in tr) for tr in traces)


def level_sets(n_props: int, traces: Sequence[Sequence[int]], max_cost: int,
               op_cost=(1, 1, 1, 1, 1, 1, 1), atom_cost: int = 1):
    """Returns (by_cost, mincost): by_cost[c] = set of CMs of all trees of
    cost exactly c; mincost maps each CM to its least tree cost."""
    kappa = dict(zip(OPS, op_cost))
    by_cost: Dict[int, Set[tuple]] = {c: set() for c in range(max_cost + 1)}
    if atom_cost <= max_cost:
        for p in range(n_props):
            by_cost[atom_cost].add(_cm_of_atom(p, traces))
    for c in range(1, max_cost + 1):
        for op in ("!", "X", "F", "G"):
            k = kappa[op]
            if k == 0 or c - k < 1:
                continue
            for cm in by_cost[c - k]:
                by_cost[c].add(tuple(tuple(ev.apply_unary(op, cs)) for cs in cm))
        for op in ("&", "|", "U"):
            k = kappa[op]
            if k == 0:
                continue
            for i in range(1, c - k):
                j = c - k - i
                if j < 1:
                    continue
                for a in by_cost[i]:
                    for b in by_cost[j]:
                        by_cost[c].add(tuple(tuple(ev.apply_binary(op, x, y))
                                             for x, y in zip(a, b)))
    mincost: Dict[tuple, int] = {}
    for c in range(1, max_cost + 1):
        for cm in by_cost[c]:
            if cm not in mincost:
                mincost[cm] = c
    return by_cost, mincost


def unique_levels(n_props, traces, max_cost, op_cost=(1, 1, 1, 1, 1, 1, 1), atom_cost=1):
    """U_c as sets of canonical word tuples, c = 1..max_cost."""
    _, mincost = level_sets(n_props, traces, max_cost, op_cost, atom_cost)
    out: Dict[int, Set[Tuple[int, ...]]] = {c: set() for c in range(1, max_cost + 1)}
    for cm, c in mincost.items():
        out[c].add(tuple(ev.canonical_words(cm)))
    return out


def min_separating_cost(n_props, traces, positive, max_cost, op_cost=(1, 1, 1, 1, 1, 1, 1),
                        atom_cost=1):
    _, mincost = level_sets(n_props, traces, max_cost, op_cost, atom_cost)
    want = tuple(bool(x) for x in positive)
    best = None
    for cm, c in mincost.items():
        if tuple(cs[0] for cs in cm) == want and (best is None or c < best):
            best = c
    return best

"""Recursive LTLf evaluator written from the satisfaction relation itself.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The satisfaction relation ``tr, i |= phi`` of the paper's section
"Synthesising linear temporal logic formulae from examples", over finite,
non-empty traces; each clause below is the quantifier definition, not a
recurrence:

* ``p``      : p holds in the i-th letter;
* ``not f``  : not (tr, i |= f);
* ``f and g``, ``f or g``: the Boolean connectives;
* ``X f``    : i+1 < n and tr, i+1 |= f        (strong next: false at the
  last position; fixed by the paper's worked bit example);
* ``F f``    : some j in [i, n) with tr, j |= f  (reflexive);
* ``G f``    : every j in [i, n) has tr, j |= f  (the dual of F);
* ``f U g``  : some j in [i, n) with tr, j |= g and tr, k |= f for all k in
  [i, j)  (reflexive until: g now suffices).

Separation (same section): phi separates (P, N) iff tr, 0 |= phi for every
tr in P and not for any tr in N.

Formulas are given as prefix token strings (``"! U p1 p0"``) or as nested
tuples ``('!', ('U', ('p', 1), ('p', 0)))``; this module has its own parser.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

UNARY = {"!", "X", "F", "G"}
BINARY = {"&", "|", "U"}


def parse(s: str):
    toks = s.split()
    pos = 0

    def node():
        nonlocal pos
        if pos >= len(toks):
            raise ValueError("truncated formula")
        t = toks[pos]
        pos += 1
        if t[0] == "p" and t[1:].isdigit():
            return ("p", int(t[1:]))
        if t in UNARY:
            return (t, node())
        if t in BINARY:
            a = node()
            b = node()
            return (t, a, b)
        raise ValueError(f"unknown token {t!r}")

    f = node()
    if pos != len(toks):
        raise ValueError("trailing tokens")
    return f


def as_tree(f):
    return parse(f) if isinstance(f, str) else f


def cost(f, atom_cost: int = 1, op_cost: Dict[str, int] | None = None) -> int:
    f = as_tree(f)
    if f[0] == "p":
        return atom_cost
    c = 1 if op_cost is None else op_cost[f[0]]
    return c + sum(cost(g, atom_cost, op_cost) for g in f[1:])


def holds(f, tr: Sequence[int], i: int) -> bool:
    """tr, i |= f, straight from the definitions (exponential; tiny inputs)."""
    f = as_tree(f)
    n = len(tr)
    if not (0 <= i < n):
        return False
    k = f[0]
    if k == "p":
        return bool((tr[i] >> f[1]) & 1)
    if k == "!":
        return not holds(f[1], tr, i)
    if k == "&":
        return holds(f[1], tr, i) and holds(f[2], tr, i)
    if k == "|":
        return holds(f[1], tr, i) or holds(f[2], tr, i)
    if k == "X":
        return i + 1 < n and holds(f[1], tr, i + 1)
    if k == "F":
        return any(holds(f[1], tr, j) for j in range(i, n))
    if k == "G":
        return all(holds(f[1], tr, j) for j in range(i, n))
    if k == "U":
        return any(holds(f[2], tr, j) and all(holds(f[1], tr, m) for m in range(i, j))
                   for j in range(i, n))
    raise ValueError(k)


def vector(f, tr: Sequence[int]) -> List[bool]:
    """[tr, i |= f for i in range(len(tr))], the same definitions evaluated
    bottom-up over the parse tree (children's truth vectors are reused)."""
    f = as_tree(f)
    n = len(tr)
    k = f[0]
    if k == "p":
        return [bool((x >> f[1]) & 1) for x in tr]
    a = vector(f[1], tr)
    if k in UNARY:
        return apply_unary(k, a)
    b = vector(f[2], tr)
    return apply_binary(k, a, b)


def apply_unary(k: str, a: Sequence[bool]) -> List[bool]:
    n = len(a)
    if k == "!":
        return [not x for x in a]
    if k == "X":
        return [i + 1 < n and a[i + 1] for i in range(n)]
    if k == "F":
        return [any(a[j] for j in range(i, n)) for i in range(n)]
    if k == "G":
        return [all(a[j] for j in range(i, n)) for i in range(n)]
    raise ValueError(k)


def apply_binary(k: str, a: Sequence[bool], b: Sequence[bool]) -> List[bool]:
    n = len(a)
    if k == "&":
        return [x and y for x, y in zip(a, b)]
    if k == "|":
        return [x or y for x, y in zip(a, b)]
    if k == "U":
        return [any(b[j] and all(a[m] for m in range(i, j)) for j in range(i, n))
                for i in range(n)]
    raise ValueError(k)


def separates(f, traces: Sequence[Sequence[int]], positive: Sequence[int]) -> bool:
    f = as_tree(f)
    return all(vector(f, tr)[0] == bool(lab) for tr, lab in zip(traces, positive))


def characteristic_matrix(f, traces: Sequence[Sequence[int]]) -> Tuple[Tuple[bool, ...], ...]:
    """The CM: one characteristic sequence per trace, in trace order."""
    f = as_tree(f)
    return tuple(tuple(vector(f, tr)) for tr in traces)


def canonical_words(cm: Sequence[Sequence[bool]]) -> List[int]:
    """Canonical packing: trace by trace, positions 0..n-1 as consecutive bits,
    least significant first, in 64-bit words, tail zero-padded."""
    bits = [b for cs in cm for b in cs]
    nw = (len(bits) + 63) // 64
    out = [0] * nw
    for g, b in enumerate(bits):
        if b:
            out[g >> 6] |= 1 << (g & 63)
    return out

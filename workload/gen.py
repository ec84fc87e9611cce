"""Seeded synthetic LTLf synthesis problems.

This module only produces inputs: example traces, their labels and the
planted formula that labels them.  It is shared by the tests, the benchmark
and the smoke check, and deliberately contains none of the enumeration,
deduplication or bit-parallel operator code that the library and the oracle
implement (each of those has its own).  The small recursive labeller below is
used for nothing but attaching labels to freshly drawn traces.

A trace is a list of integers, one per position; bit p of an entry is set iff
atomic proposition p holds at that position (the paper's traces are strings
over the powerset of the alphabet).  Formulas are nested tuples:
``('p', i)``, ``('!', f)``, ``('X', f)``, ``('F', f)``, ``('G', f)``,
``('&', f, g)``, ``('|', f, g)``, ``('U', f, g)``.

Workload recipe (all draws from ``numpy.random.Generator(PCG64(seed))`` in
the order written below):

* trace lengths are uniform integers in ``[len_lo, len_hi]``;
* each (position, proposition) bit is Bernoulli(q_p), where q_p is one fixed
  value for every proposition (``q``) or drawn per proposition uniformly from
  ``q_range``;
* the planted formula of exact unit cost c: an atom if c == 1, else a
  uniformly chosen operator among those whose arity fits (unary needs
  c >= 2, binary c >= 3); a binary operator splits its remaining cost with
  the left cost uniform in ``[1, c-2]``; the formula is redrawn while its
  rate of holding at position 0 over 1000 pilot traces is outside
  ``[0.1, 0.9]``;
* traces are then drawn one at a time and kept if their class (holds at
  position 0 or not) still has room; after 200 times the needed number of
  draws without filling both classes the formula is redrawn.

The traces are returned positives first, then negatives.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

UNARY = ("!", "X", "F", "G")
BINARY = ("&", "|", "U")


@dataclass
class Problem:
    n_props: int
    traces: List[List[int]]
    positive: List[int]
    planted: Optional[tuple] = None
    planted_cost: int = 0
    cost_bound: int = 0
    seed: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def lengths(self) -> List[int]:
        return [len(t) for t in self.traces]

    @property
    def total_positions(self) -> int:
        return sum(len(t) for t in self.traces)

    def flat_letters(self) -> np.ndarray:
        return np.array([x for t in self.traces for x in t], dtype=np.uint32)

    def arrays(self):
        """(lengths u32, letters u32, positive u8) numpy arrays."""
        return (np.array(self.lengths, dtype=np.uint32), self.flat_letters(),
                np.array(self.positive, dtype=np.uint8))


# ---------------------------------------------------------------- labelling --
def _label_vector(f, tr: Sequence[int]) -> List[bool]:
    """Truth of formula f at every position of trace tr (finite-trace LTL,
    strong next, reflexive eventually/always/until)."""
    n = len(tr)
    k = f[0]
    if k == "p":
        return [bool((x >> f[1]) & 1) for x in tr]
    a = _label_vector(f[1], tr)
    if k == "!":
        return [not v for v in a]
    if k == "X":
        return [a[i + 1] if i + 1 < n else False for i in range(n)]
    if k == "F":
        return [any(a[i:]) for i in range(n)]
    if k == "G":
        return [all(a[i:]) for i in range(n)]
    b = _label_vector(f[2], tr)
    if k == "&":
        return [x and y for x, y in zip(a, b)]
    if k == "|":
        return [x or y for x, y in zip(a, b)]
    if k == "U":
        out = []
        for i in range(n):
            hit = False
            for j in range(i, n):
                if b[j]:
                    hit = True
                    break
                if not a[j]:
                    break
            out.append(hit)
        return out
    raise ValueError(f"unknown operator {k!r}")


def label(f, tr: Sequence[int]) -> bool:
    return _label_vector(f, tr)[0]


def formula_cost(f) -> int:
    """Unit cost = number of nodes."""
    return 1 + sum(formula_cost(g) for g in f[1:] if isinstance(g, tuple))


def to_prefix(f) -> str:
    if f[0] == "p":
        return f"p{f[1]}"
    return " ".join([f[0]] + [to_prefix(g) for g in f[1:]])


def parse_prefix(s: str):
    toks = s.split()
    pos = 0

    def go():
        nonlocal pos
        t = toks[pos]
        pos += 1
        if t.startswith("p"):
            return ("p", int(t[1:]))
        if t in UNARY:
            return (t, go())
        if t in BINARY:
            a = go()
            return (t, a, go())
        raise ValueError(f"bad token {t!r}")

    f = go()
    if pos != len(toks):
        raise ValueError("trailing tokens")
    return f


# ---------------------------------------------------------------- sampling ---
def _draw_trace(rng, n_props, q, len_lo, len_hi) -> List[int]:
    n = int(rng.integers(len_lo, len_hi + 1))
    bits = rng.random((n, n_props)) < q[None, :]
    w = (1 << np.arange(n_props, dtype=np.int64))
    return [int(v) for v in (bits.astype(np.int64) * w).sum(axis=1)]


def _draw_formula(rng, n_props, cost, ops_unary=UNARY, ops_binary=BINARY):
    if cost == 1:
        return ("p", int(rng.integers(0, n_props)))
    choices = list(ops_unary) + (list(ops_binary) if cost >= 3 else [])
    op = choices[int(rng.integers(0, len(choices)))]
    if op in ops_unary:
        return (op, _draw_formula(rng, n_props, cost - 1, ops_unary, ops_binary))
    i = int(rng.integers(1, cost - 1))  # left cost in [1, cost-2]
    return (op, _draw_formula(rng, n_props, i, ops_unary, ops_binary),
            _draw_formula(rng, n_props, cost - 1 - i, ops_unary, ops_binary))


def make_problem(seed: int, n_props: int, n_pos: int, n_neg: int, len_lo: int, len_hi: int,
                 planted_cost: int, cost_bound: int, q: float | None = None,
                 q_range: Tuple[float, float] | None = None, name: str = "") -> Problem:
    rng = np.random.Generator(np.random.PCG64(seed))
    if q_range is not None:
        qv = rng.uniform(q_range[0], q_range[1], size=n_props)
    else:
        qv = np.full(n_props, 0.5 if q is None else q)
    need = n_pos + n_neg
    for _attempt in range(1000):
        while True:
            f = _draw_formula(rng, n_props, planted_cost)
            pilot = [label(f, _draw_trace(rng, n_props, qv, len_lo, len_hi)) for _ in range(1000)]
            rate = sum(pilot) / len(pilot)
            if 0.1 <= rate <= 0.9:
                break
        pos, neg = [], []
        draws = 0
        while (len(pos) < n_pos or len(neg) < n_neg) and draws < 200 * need:
            tr = _draw_trace(rng, n_props, qv, len_lo, len_hi)
            draws += 1
            if label(f, tr):
                if len(pos) < n_pos:
                    pos.append(tr)
            elif len(neg) < n_neg:
                neg.append(tr)
        if len(pos) == n_pos and len(neg) == n_neg:
            return Problem(n_props=n_props, traces=pos + neg, positive=[1] * n_pos + [0] * n_neg,
                           planted=f, planted_cost=planted_cost, cost_bound=cost_bound,
                           seed=seed, name=name,
                           meta=dict(q=[float(x) for x in qv], len_lo=len_lo, len_hi=len_hi))
    raise RuntimeError("could not fill both classes")


# ------------------------------------------------------------ named configs --
def tiny(seed: int) -> Problem:
    """2 props, 6+6 traces, lengths 3..8, bits Bernoulli(0.5), planted cost 7, bound 10."""
    return make_problem(seed, 2, 6, 6, 3, 8, 7, 10, q=0.5, name=f"tiny/s{seed}")


def medium(seed: int) -> Problem:
    """3 props, 32+32 traces, lengths 8..32, per-prop q ~ U(0.3, 0.7), planted 11, bound 14."""
    return make_problem(seed, 3, 32, 32, 8, 32, 11, 14, q_range=(0.3, 0.7), name=f"medium/s{seed}")


def large(seed: int) -> Problem:
    """5 props, 512+512 traces, lengths 16..64, per-prop q ~ U(0.3, 0.7), planted 13, bound 16."""
    return make_problem(seed, 5, 512, 512, 16, 64, 13, 16, q_range=(0.3, 0.7), name=f"large/s{seed}")


def batched(master_seed: int = 1, count: int = 256) -> List[Problem]:
    """Mixed batch: props U{2..5}, traces per class U{8..256}, lengths 4..64,
    planted cost U{6..12}, bound planted+3; problem k uses seed 1000+k and its
    shape is drawn from the master seed."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    out = []
    for k in range(count):
        props = int(rng.integers(2, 6))
        npc = int(rng.integers(8, 257))
        pc = int(rng.integers(6, 13))
        out.append(make_problem(1000 + k, props, npc, npc, 4, 64, pc, pc + 3,
                                q_range=(0.3, 0.7), name=f"batched/{k}"))
    return out


def served(master_seed: int = 2, count: int = 128, outlier_frac: float = 0.0) -> List[Problem]:
    """Served stream: the batched mix (master seed) with round(count x
    outlier_frac) requests, at positions drawn from the master seed, replaced
    by outliers of the large configuration's size (5 props, 512+512 traces,
    lengths 16..64) with the mix's cost law (planted U{6..12}, bound
    planted+3); outlier k uses seed 5000+k."""
    out = batched(master_seed, count)
    n_out = int(round(count * outlier_frac))
    if n_out:
        rng = np.random.Generator(np.random.PCG64(master_seed + 7))
        where = sorted(int(i) for i in rng.choice(count, size=n_out, replace=False))
        for k, i in enumerate(where):
            pc = int(rng.integers(6, 13))
            out[i] = make_problem(5000 + k, 5, 512, 512, 16, 64, pc, pc + 3, q_range=(0.3, 0.7),
                                  name=f"served/{i}-outlier")
    return out


def custom(n_props: int, traces_pos: Sequence[Sequence[int]], traces_neg: Sequence[Sequence[int]],
           cost_bound: int, name: str = "") -> Problem:
    return Problem(n_props=n_props, traces=[list(t) for t in traces_pos] + [list(t) for t in traces_neg],
                   positive=[1] * len(traces_pos) + [0] * len(traces_neg), cost_bound=cost_bound,
                   name=name)


def random_small(seed: int, n_props: int, n_traces: int, len_lo: int, len_hi: int,
                 q: float = 0.5, pos_frac: float = 0.5) -> Problem:
    """Unlabelled-by-formula random problem (labels are coin flips); used for
    exhaustive checks on tiny inputs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    qv = np.full(n_props, q)
    trs = [_draw_trace(rng, n_props, qv, len_lo, len_hi) for _ in range(n_traces)]
    lab = [int(rng.random() < pos_frac) for _ in range(n_traces)]
    return Problem(n_props=n_props, traces=trs, positive=lab, cost_bound=0, seed=seed,
                   name=f"random/s{seed}")

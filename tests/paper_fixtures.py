"""Loads the worked examples of tests/golden/paper_examples.json into problems."""
from __future__ import annotations

import json
import os

from workload import custom

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_examples.json")


def load():
    with open(GOLDEN) as f:
        return json.load(f)


def letter_mask(letter: str, props) -> int:
    return sum(1 << props.index(ch) for ch in letter)


def trace_masks(trace, props):
    return [letter_mask(x, props) for x in trace]


def formula_tokens(f: str, props) -> str:
    """Replaces proposition names by p<k> tokens."""
    return " ".join(f"p{props.index(t)}" if t in props else t for t in f.split())


def spec_problem(name: str, cost_bound: int):
    d = load()[name]
    props = d["props"]
    return custom(len(props), [trace_masks(t, props) for t in d["positive"]],
                  [trace_masks(t, props) for t in d["negative"]], cost_bound, name=name)

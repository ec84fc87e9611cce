"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check."""
from .gen import (Problem, tiny, medium, large, batched, served, custom, random_small, make_problem,
                  parse_prefix, to_prefix, formula_cost, label)

__all__ = ["Problem", "tiny", "medium", "large", "batched", "served", "custom", "random_small",
           "make_problem", "parse_prefix", "to_prefix", "formula_cost", "label"]

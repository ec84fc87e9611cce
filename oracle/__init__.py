"""CPU oracle for LTLf semantic enumeration -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and its
Python binding) never imports, links or calls anything here.

Pieces:

* ``ltlf_oracle.c`` -- single-threaded bottom-up enumerator (plain C), built
  into ``liboracle.so`` by :func:`build`; wrapped by :func:`solve`.
* ``evaluator.py`` -- recursive evaluator written from the quantifier
  definitions of the satisfaction relation.
* ``brute.py`` -- exhaustive enumeration of all syntax trees up to a small
  cost, giving the level sets straight from their definition.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ltlf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_FOUND, CAPACITY, EINVAL, ENOMEM = 0, 1, 2, -1, -2
STATUS_NAMES = {0: "OK", 1: "NOT_FOUND", 2: "CAPACITY", -1: "EINVAL", -2: "ENOMEM"}

# op_cost order: not, X, F, G, and, or, U
OPS = ("!", "X", "F", "G", "&", "|", "U")
UNIT_ALL = (1, 1, 1, 1, 1, 1, 1)
# the grammar printed in the paper: p, not, and, X, F, U
UNIT_PAPER = (1, 1, 1, 0, 1, 0, 1)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Deriv(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint8), ("left", ctypes.c_uint32), ("right", ctypes.c_uint32)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("min_cost", ctypes.c_uint32),
                ("levels_done", ctypes.c_uint32), ("overflow_level", ctypes.c_uint32),
                ("checked_level", ctypes.c_uint32), ("witness_outer", ctypes.c_uint32),
                ("witness_kind", ctypes.c_uint64), ("witness_id", ctypes.c_uint64),
                ("witness_der", _Deriv), ("candidates", ctypes.c_uint64),
                ("seconds", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.oracle_create.restype = ctypes.c_void_p
        L.oracle_destroy.argtypes = [ctypes.c_void_p]
        L.oracle_solve.restype = ctypes.c_int
        L.oracle_solve.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(_Result)]
        L.oracle_level_count.restype = ctypes.c_uint64
        L.oracle_level_count.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
        L.oracle_level_start.restype = ctypes.c_uint64
        L.oracle_level_start.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
        L.oracle_canon_words.restype = ctypes.c_uint64
        L.oracle_canon_words.argtypes = [ctypes.c_void_p]
        L.oracle_export_level.restype = ctypes.c_uint64
        L.oracle_export_level.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                          ctypes.c_uint64]
        L.oracle_witness.restype = ctypes.c_uint64
        L.oracle_witness.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Result), ctypes.c_char_p,
                                     ctypes.c_uint64]
        L.oracle_formula_of.restype = ctypes.c_uint64
        L.oracle_formula_of.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_char_p,
                                        ctypes.c_uint64]
        _lib = L
    return _lib


@dataclass
class OracleResult:
    status: int
    min_cost: int
    levels_done: int
    overflow_level: int
    checked_level: int
    level_counts: List[int]
    witness: str
    candidates: int
    seconds: float
    _handle: Optional["Oracle"] = field(default=None, repr=False)

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))

    def export_level(self, c: int) -> np.ndarray:
        return self._handle.export_level(c)

    def formulas_of_level(self, c: int) -> List[str]:
        return self._handle.formulas_of_level(c)


class Oracle:
    """One oracle context (holds the enumerated levels of the last solve)."""

    def __init__(self):
        self._L = _load()
        self._h = self._L.oracle_create()
        self._res = _Result()
        self._keep = None

    def __del__(self):
        try:
            if self._h:
                self._L.oracle_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def solve(self, problem, op_cost=UNIT_ALL, atom_cost: int = 1,
              cost_bound: Optional[int] = None, max_rows: int = 0,
              exhaust: bool = False, lookahead: bool = True) -> OracleResult:
        """lookahead: after a level that overflowed max_rows with no
        separating candidate, test the next level too (the library's
        default)."""
        lengths, letters, positive = problem.arrays()
        bound = int(cost_bound if cost_bound is not None else problem.cost_bound)
        oc = np.array(op_cost, dtype=np.uint32)
        self._keep = (lengths, letters, positive, oc)
        st = self._L.oracle_solve(self._h, problem.n_props, len(problem.traces),
                                  lengths.ctypes.data, letters.ctypes.data, positive.ctypes.data,
                                  atom_cost, oc.ctypes.data, bound, max_rows,
                                  (1 if exhaust else 0) | (2 if lookahead else 0),
                                  ctypes.byref(self._res))
        counts = [int(self._L.oracle_level_count(self._h, c)) for c in range(bound + 1)] \
            if st >= 0 else []
        buf = ctypes.create_string_buffer(1 << 16)
        self._L.oracle_witness(self._h, ctypes.byref(self._res), buf, len(buf))
        r = self._res
        return OracleResult(status=int(r.status), min_cost=int(r.min_cost),
                            levels_done=int(r.levels_done), overflow_level=int(r.overflow_level),
                            checked_level=int(r.checked_level), level_counts=counts, witness=buf.value.decode(),
                            candidates=int(r.candidates), seconds=float(r.seconds), _handle=self)

    def export_level(self, c: int) -> np.ndarray:
        n = int(self._L.oracle_level_count(self._h, c))
        cw = int(self._L.oracle_canon_words(self._h))
        out = np.zeros((n, cw), dtype=np.uint64)
        if n:
            got = self._L.oracle_export_level(self._h, c, out.ctypes.data, out.size)
            assert got == n
        return out

    def formulas_of_level(self, c: int) -> List[str]:
        n = int(self._L.oracle_level_count(self._h, c))
        s = int(self._L.oracle_level_start(self._h, c))
        buf = ctypes.create_string_buffer(1 << 16)
        out = []
        for q in range(n):
            self._L.oracle_formula_of(self._h, s + q, buf, len(buf))
            out.append(buf.value.decode())
        return out


def solve(problem, op_cost=UNIT_ALL, atom_cost: int = 1, cost_bound: Optional[int] = None,
          max_rows: int = 0, exhaust: bool = False, lookahead: bool = True) -> OracleResult:
    return Oracle().solve(problem, op_cost=op_cost, atom_cost=atom_cost, cost_bound=cost_bound,
                          max_rows=max_rows, exhaust=exhaust, lookahead=lookahead)

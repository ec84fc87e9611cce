"""Python binding of the C ABI in include/ltlf.h (argument marshalling only).

The functions named ``ltlf_*`` mirror the C entry points one to one.  Every
step of the synthesis runs in libltlf.so; nothing here computes on the data.
PyTorch supplies device memory (the workspace tensor) and the stream.
:class:`Synthesizer` bundles a context, a torch workspace and the current
stream for convenience.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libltlf.so")

OK, NOT_FOUND, CAPACITY, PENDING, CANCELLED = 0, 1, 2, 3, 4
EINVAL, ENOMEM, EDEVICE, EBUFSZ, ESTATE = -1, -2, -3, -4, -5
STATUS_NAMES = {0: "OK", 1: "NOT_FOUND", 2: "CAPACITY", 3: "PENDING", 4: "CANCELLED", -1: "EINVAL", -2: "ENOMEM",
                -3: "EDEVICE", -4: "EBUFSZ", -5: "ESTATE"}
FLAG_EXHAUST = 0x1
FLAG_PROFILE = 0x2
FLAG_KERNEL_LANE = 0x4  # one candidate per lane (default where it fits)
FLAG_KERNEL_GROUP = 0x8  # one candidate per lane group (rows of 2..64 chunks)
FLAG_KERNEL_WAVE = 0x10  # one candidate per wavefront (any row width)
FLAG_NO_LOOKAHEAD = 0x20  # stop at an overflowed level (no check of the next one)
FLAG_DIGEST = 0x40  # per-level digests of the stored sets (ltlf_result.level_digests)
FLAG_WEAK_HASH = 0x100  # test hook: 6-bit hashes, every probe meets an equal tag

OP_NAMES = ("!", "X", "F", "G", "&", "|", "U")  # index = ltlf_op


class LtlfError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        msg = f"{where}: {STATUS_NAMES.get(status, status)}"
        super().__init__(msg + (f" ({detail})" if detail else ""))
        self.status = status


class ltlf_spec(ctypes.Structure):
    _fields_ = [("n_props", ctypes.c_uint32), ("n_traces", ctypes.c_uint32),
                ("lengths", ctypes.POINTER(ctypes.c_uint32)),
                ("letters", ctypes.POINTER(ctypes.c_uint32)),
                ("positive", ctypes.POINTER(ctypes.c_uint8))]


class ltlf_costs(ctypes.Structure):
    _fields_ = [("atom_cost", ctypes.c_uint32), ("op_cost", ctypes.c_uint32 * 7)]


class ltlf_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("min_cost", ctypes.c_uint32),
                ("levels_done", ctypes.c_uint32), ("overflow_level", ctypes.c_uint32),
                ("level_counts", ctypes.POINTER(ctypes.c_uint64)),
                ("level_counts_len", ctypes.c_uint32),
                ("formula", ctypes.c_char_p), ("formula_cap", ctypes.c_uint64),
                ("formula_len", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
                ("unique_total", ctypes.c_uint64), ("deferred", ctypes.c_uint64),
                ("row_bytes", ctypes.c_uint32), ("gen_launches", ctypes.c_uint32),
                ("verify_launches", ctypes.c_uint32), ("checked_level", ctypes.c_uint32),
                ("enum_ms", ctypes.c_double), ("gen_ms", ctypes.c_double),
                ("verify_ms", ctypes.c_double), ("dead_rows", ctypes.c_uint64),
                ("level_digests", ctypes.POINTER(ctypes.c_uint64))]


TUNE_CLASSES = 16


class ltlf_tuning(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_uint32), ("chunks", ctypes.c_uint32 * TUNE_CLASSES),
                ("kernel", ctypes.c_uint32 * TUNE_CLASSES), ("bound", ctypes.c_uint32 * TUNE_CLASSES),
                ("candidates", ctypes.c_uint64 * TUNE_CLASSES),
                ("ns_per_candidate", (ctypes.c_double * 3) * TUNE_CLASSES),
                ("wave_tile", ctypes.c_uint32 * TUNE_CLASSES),
                ("ns_wave_tile", (ctypes.c_double * 3) * TUNE_CLASSES)]


class ltlf_split_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("depth", ctypes.c_uint32),
                ("parts_solved", ctypes.c_uint32), ("parts_split", ctypes.c_uint32),
                ("max_part_cost", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("cost", ctypes.c_uint64), ("formula", ctypes.c_char_p),
                ("formula_cap", ctypes.c_uint64), ("formula_len", ctypes.c_uint64),
                ("enum_ms", ctypes.c_double)]


_lib = None


def load_library() -> ctypes.CDLL:
    """Loads libltlf.so from the package directory; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libltlf.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.ltlf_status_str.restype = ctypes.c_char_p
    L.ltlf_status_str.argtypes = [i32]
    L.ltlf_ctx_last_error.restype = ctypes.c_char_p
    L.ltlf_ctx_last_error.argtypes = [vp]
    L.ltlf_ctx_create.restype = i32
    L.ltlf_ctx_create.argtypes = [i32, u64, ctypes.POINTER(vp)]
    L.ltlf_ctx_set_workspace.restype = i32
    L.ltlf_ctx_set_workspace.argtypes = [vp, vp, u64]
    L.ltlf_ctx_cancel.restype = i32
    L.ltlf_ctx_cancel.argtypes = [vp]
    L.ltlf_ctx_set_row_limit.restype = i32
    L.ltlf_ctx_set_row_limit.argtypes = [vp, u64]
    L.ltlf_ctx_destroy.restype = None
    L.ltlf_ctx_destroy.argtypes = [vp]
    L.ltlf_load.restype = i32
    L.ltlf_load.argtypes = [vp, ctypes.POINTER(ltlf_spec), vp]
    L.ltlf_run.restype = i32
    L.ltlf_run.argtypes = [vp, ctypes.POINTER(ltlf_costs), u32, u32, vp, ctypes.POINTER(ltlf_result)]
    L.ltlf_solve.restype = i32
    L.ltlf_solve.argtypes = [vp, ctypes.POINTER(ltlf_spec), ctypes.POINTER(ltlf_costs), u32, u32, vp,
                             ctypes.POINTER(ltlf_result)]
    L.ltlf_solve_static.restype = i32
    L.ltlf_solve_static.argtypes = [vp, ctypes.POINTER(ltlf_spec), ctypes.POINTER(ltlf_costs), u32, u32, vp,
                                    ctypes.POINTER(ltlf_result)]
    L.ltlf_solve_batch.restype = i32
    L.ltlf_solve_batch.argtypes = [vp, u32, ctypes.POINTER(ltlf_spec), ctypes.POINTER(ltlf_costs),
                                   ctypes.POINTER(u32), u32, vp, ctypes.POINTER(ltlf_result)]
    L.ltlf_autotune.restype = i32
    L.ltlf_autotune.argtypes = [vp, vp, ctypes.POINTER(ltlf_tuning)]
    L.ltlf_ctx_set_tuning.restype = i32
    L.ltlf_ctx_set_tuning.argtypes = [vp, ctypes.POINTER(ltlf_tuning)]
    L.ltlf_solve_split.restype = i32
    L.ltlf_solve_split.argtypes = [vp, ctypes.POINTER(ltlf_spec), ctypes.POINTER(ltlf_costs), u32, u32, u32, vp,
                                   ctypes.POINTER(ltlf_split_result)]
    L.ltlf_server_create.restype = i32
    L.ltlf_server_create.argtypes = [vp, u32, ctypes.POINTER(vp)]
    L.ltlf_server_submit.restype = i32
    L.ltlf_server_submit.argtypes = [vp, ctypes.POINTER(ltlf_spec), ctypes.POINTER(ltlf_costs), u32, u32, u64,
                                     ctypes.POINTER(u64)]
    L.ltlf_server_step.restype = i32
    L.ltlf_server_step.argtypes = [vp, vp, ctypes.POINTER(u32)]
    L.ltlf_server_poll.restype = i32
    L.ltlf_server_poll.argtypes = [vp, u64, ctypes.POINTER(ltlf_result)]
    L.ltlf_server_cancel.restype = i32
    L.ltlf_server_cancel.argtypes = [vp, u64]
    L.ltlf_server_load.restype = i32
    L.ltlf_server_load.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u64)]
    L.ltlf_server_destroy.restype = None
    L.ltlf_server_destroy.argtypes = [vp]
    L.ltlf_export_level.restype = i32
    L.ltlf_export_level.argtypes = [vp, u32, u64, u64, vp, u64, ctypes.POINTER(u64),
                                    ctypes.POINTER(u64)]
    L.ltlf_formula_of.restype = i32
    L.ltlf_formula_of.argtypes = [vp, u32, u64, ctypes.c_char_p, u64, ctypes.POINTER(u64)]
    _lib = L
    return L


# ---------------------------------------------------------- C entry points --
def ltlf_status_str(status: int) -> str:
    return load_library().ltlf_status_str(status).decode()


def ltlf_ctx_last_error(ctx) -> str:
    return load_library().ltlf_ctx_last_error(ctx).decode()


def ltlf_ctx_create(device: int, hbm_budget_bytes: int):
    h = ctypes.c_void_p()
    st = load_library().ltlf_ctx_create(device, hbm_budget_bytes, ctypes.byref(h))
    return st, h


def ltlf_ctx_set_workspace(ctx, dev_ptr: int, nbytes: int) -> int:
    return load_library().ltlf_ctx_set_workspace(ctx, ctypes.c_void_p(dev_ptr), nbytes)


def ltlf_ctx_cancel(ctx) -> int:
    return load_library().ltlf_ctx_cancel(ctx)


def ltlf_ctx_set_row_limit(ctx, max_rows: int) -> int:
    return load_library().ltlf_ctx_set_row_limit(ctx, max_rows)


def ltlf_ctx_destroy(ctx) -> None:
    load_library().ltlf_ctx_destroy(ctx)


def _spec(n_props, lengths, letters, positive):
    lengths = np.ascontiguousarray(lengths, dtype=np.uint32)
    letters = np.ascontiguousarray(letters, dtype=np.uint32)
    positive = np.ascontiguousarray(positive, dtype=np.uint8)
    sp = ltlf_spec(n_props, len(lengths),
                   lengths.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                   letters.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                   positive.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return sp, (lengths, letters, positive)


def _costs(op_cost: Sequence[int], atom_cost: int):
    c = ltlf_costs()
    c.atom_cost = atom_cost
    for i, v in enumerate(op_cost):
        c.op_cost[i] = v
    return c


def ltlf_load(ctx, n_props, lengths, letters, positive, stream: int = 0) -> int:
    sp, keep = _spec(n_props, lengths, letters, positive)
    return load_library().ltlf_load(ctx, ctypes.byref(sp), ctypes.c_void_p(stream))


def ltlf_run(ctx, op_cost, atom_cost, cost_bound, flags, stream, res: ltlf_result) -> int:
    c = _costs(op_cost, atom_cost)
    return load_library().ltlf_run(ctx, ctypes.byref(c), cost_bound, flags, ctypes.c_void_p(stream),
                                   ctypes.byref(res))


def ltlf_solve(ctx, n_props, lengths, letters, positive, op_cost, atom_cost, cost_bound, flags,
               stream, res: ltlf_result) -> int:
    sp, keep = _spec(n_props, lengths, letters, positive)
    c = _costs(op_cost, atom_cost)
    return load_library().ltlf_solve(ctx, ctypes.byref(sp), ctypes.byref(c), cost_bound, flags,
                                     ctypes.c_void_p(stream), ctypes.byref(res))


def ltlf_solve_static(ctx, n_props, lengths, letters, positive, op_cost, atom_cost, cost_bound, flags,
                      stream, res: ltlf_result) -> int:
    sp, keep = _spec(n_props, lengths, letters, positive)
    c = _costs(op_cost, atom_cost)
    return load_library().ltlf_solve_static(ctx, ctypes.byref(sp), ctypes.byref(c), cost_bound, flags,
                                            ctypes.c_void_p(stream), ctypes.byref(res))


def ltlf_solve_batch(ctx, problems, op_cost, atom_cost, bounds, flags, stream, results) -> int:
    """problems: (n_props, lengths, letters, positive) per problem; results:
    ctypes array of ltlf_result with the caller's buffers set."""
    n = len(problems)
    specs = (ltlf_spec * n)()
    keep = []
    for i, (n_props, lengths, letters, positive) in enumerate(problems):
        sp, k = _spec(n_props, lengths, letters, positive)
        specs[i] = sp
        keep.append(k)
    c = _costs(op_cost, atom_cost)
    b = (ctypes.c_uint32 * n)(*bounds)
    return load_library().ltlf_solve_batch(ctx, n, specs, ctypes.byref(c), b, flags, ctypes.c_void_p(stream),
                                           results)


def ltlf_autotune(ctx, stream, out) -> int:
    return load_library().ltlf_autotune(ctx, ctypes.c_void_p(stream), ctypes.byref(out) if out is not None else None)


def ltlf_ctx_set_tuning(ctx, tuning) -> int:
    return load_library().ltlf_ctx_set_tuning(ctx, ctypes.byref(tuning) if tuning is not None else None)


def ltlf_solve_split(ctx, n_props, lengths, letters, positive, op_cost, atom_cost, cost_bound, max_traces,
                     flags, stream, res: ltlf_split_result) -> int:
    sp, keep = _spec(n_props, lengths, letters, positive)
    c = _costs(op_cost, atom_cost)
    return load_library().ltlf_solve_split(ctx, ctypes.byref(sp), ctypes.byref(c), cost_bound, max_traces, flags,
                                           ctypes.c_void_p(stream), ctypes.byref(res))


def ltlf_server_create(ctx, max_resident: int):
    h = ctypes.c_void_p()
    st = load_library().ltlf_server_create(ctx, max_resident, ctypes.byref(h))
    return st, h


def ltlf_server_submit(srv, n_props, lengths, letters, positive, op_cost, atom_cost, cost_bound, flags,
                       reserve_bytes: int = 0):
    sp, keep = _spec(n_props, lengths, letters, positive)
    c = _costs(op_cost, atom_cost)
    t = ctypes.c_uint64()
    st = load_library().ltlf_server_submit(srv, ctypes.byref(sp), ctypes.byref(c), cost_bound, flags,
                                           reserve_bytes, ctypes.byref(t))
    return st, t.value


def ltlf_server_step(srv, stream: int = 0):
    n = ctypes.c_uint32()
    st = load_library().ltlf_server_step(srv, ctypes.c_void_p(stream), ctypes.byref(n))
    return st, n.value


def ltlf_server_poll(srv, ticket: int, res: ltlf_result) -> int:
    return load_library().ltlf_server_poll(srv, ticket, ctypes.byref(res))


def ltlf_server_cancel(srv, ticket: int) -> int:
    return load_library().ltlf_server_cancel(srv, ticket)


def ltlf_server_load(srv):
    q, r, f = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
    st = load_library().ltlf_server_load(srv, ctypes.byref(q), ctypes.byref(r), ctypes.byref(f))
    return st, q.value, r.value, f.value


def ltlf_server_destroy(srv) -> None:
    load_library().ltlf_server_destroy(srv)


def ltlf_export_level(ctx, cost: int, first: int = 0, count: int = (1 << 64) - 1):
    L = load_library()
    n, cw = ctypes.c_uint64(), ctypes.c_uint64()
    st = L.ltlf_export_level(ctx, cost, first, count, None, 0, ctypes.byref(n), ctypes.byref(cw))
    if st != OK:
        return st, None
    out = np.zeros((n.value, cw.value), dtype=np.uint64)
    if n.value:
        st = L.ltlf_export_level(ctx, cost, first, count, ctypes.c_void_p(out.ctypes.data), out.size,
                                 ctypes.byref(n), ctypes.byref(cw))
    return st, out


def ltlf_formula_of(ctx, cost: int, index: int):
    L = load_library()
    need = ctypes.c_uint64()
    buf = ctypes.create_string_buffer(4096)
    st = L.ltlf_formula_of(ctx, cost, index, buf, len(buf), ctypes.byref(need))
    if st == EBUFSZ:
        buf = ctypes.create_string_buffer(int(need.value))
        st = L.ltlf_formula_of(ctx, cost, index, buf, len(buf), ctypes.byref(need))
    return st, (buf.value.decode() if st == OK else None)


# --------------------------------------------------------------- convenience --
def _result_buffers(bound: int):
    """An ltlf_result with caller buffers for levels 0..bound and the witness."""
    counts = (ctypes.c_uint64 * (bound + 1))()
    digests = (ctypes.c_uint64 * (bound + 1))()
    fbuf = ctypes.create_string_buffer(8192)
    res = ltlf_result()
    res.level_counts = counts
    res.level_digests = digests
    res.level_counts_len = bound + 1
    res.formula = ctypes.cast(fbuf, ctypes.c_char_p)
    res.formula_cap = len(fbuf)
    return res, (counts, digests, fbuf)


def _result_of(st: int, res: "ltlf_result", bufs) -> "Result":
    counts, digests, fbuf = bufs
    return Result(status=st, min_cost=res.min_cost, levels_done=res.levels_done,
                  overflow_level=res.overflow_level, level_counts=list(counts),
                  formula=fbuf.value.decode(), candidates=res.candidates,
                  unique_total=res.unique_total, enum_ms=res.enum_ms, deferred=res.deferred,
                  row_bytes=res.row_bytes, gen_launches=res.gen_launches,
                  verify_launches=res.verify_launches, gen_ms=res.gen_ms,
                  verify_ms=res.verify_ms, dead_rows=res.dead_rows, checked_level=res.checked_level,
                  level_digests=list(digests))


@dataclass
class Result:
    status: int
    min_cost: int
    levels_done: int
    overflow_level: int
    level_counts: List[int]
    formula: str
    candidates: int
    unique_total: int
    enum_ms: float
    deferred: int = 0
    row_bytes: int = 0
    gen_launches: int = 0
    verify_launches: int = 0
    gen_ms: float = 0.0
    verify_ms: float = 0.0
    dead_rows: int = 0
    checked_level: int = 0  # no formula of this cost or less separates unless status is OK
    level_digests: List[int] = field(default_factory=list)  # with FLAG_DIGEST: digest of U_c at index c

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))


@dataclass
class SplitResult:
    """Result of divide-and-conquer synthesis: a separating formula, in
    general not a minimal one."""
    status: int
    cost: int
    formula: str
    depth: int
    parts_solved: int
    parts_split: int
    max_part_cost: int
    enum_ms: float

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))


UNIT_ALL = (1, 1, 1, 1, 1, 1, 1)


class Synthesizer:
    """A context on one device with a torch-owned workspace.

    workspace_bytes: size of the torch uint8 tensor handed to the library as
    its only device memory.
    """

    def __init__(self, device: int = 0, workspace_bytes: int = 1 << 30):
        import torch

        self._torch = torch
        self.device = device
        st, self._ctx = ltlf_ctx_create(device, 0)
        if st != OK:
            raise LtlfError(st, "ltlf_ctx_create")
        self.workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8,
                                     device=f"cuda:{device}")
        st = ltlf_ctx_set_workspace(self._ctx, self.workspace.data_ptr(), self.workspace.numel())
        if st != OK:
            raise LtlfError(st, "ltlf_ctx_set_workspace")
        self._bound = 0

    def close(self):
        if getattr(self, "_ctx", None):
            ltlf_ctx_destroy(self._ctx)
            self._ctx = None
        # the workspace tensor goes with the context, even if this object
        # stays referenced (e.g. by a traceback)
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self) -> int:
        return self._torch.cuda.current_stream(self.device).cuda_stream

    def set_row_limit(self, max_rows: int) -> None:
        st = ltlf_ctx_set_row_limit(self._ctx, max_rows)
        if st != OK:
            raise LtlfError(st, "ltlf_ctx_set_row_limit")

    def load(self, problem) -> None:
        lengths, letters, positive = problem.arrays()
        st = ltlf_load(self._ctx, problem.n_props, lengths, letters, positive, self._stream())
        if st != OK:
            raise LtlfError(st, "ltlf_load", ltlf_ctx_last_error(self._ctx))

    def run(self, cost_bound: int, op_cost=UNIT_ALL, atom_cost: int = 1, flags: int = 0) -> Result:
        res, bufs = _result_buffers(cost_bound)
        st = ltlf_run(self._ctx, op_cost, atom_cost, cost_bound, flags, self._stream(), res)
        if st < 0:
            raise LtlfError(st, "ltlf_run", ltlf_ctx_last_error(self._ctx))
        self._bound = cost_bound
        return _result_of(st, res, bufs)

    def cancel(self) -> None:
        """Asks the running (or next) run of this context to stop between two
        levels (ltlf_ctx_cancel; may be called from another thread)."""
        st = ltlf_ctx_cancel(self._ctx)
        if st != OK:
            raise LtlfError(st, "ltlf_ctx_cancel")

    def solve(self, problem, cost_bound: Optional[int] = None, op_cost=UNIT_ALL, atom_cost: int = 1,
              flags: int = 0) -> Result:
        self.load(problem)
        return self.run(int(cost_bound if cost_bound is not None else problem.cost_bound),
                        op_cost=op_cost, atom_cost=atom_cost, flags=flags)

    def solve_static(self, problem, cost_bound: Optional[int] = None, op_cost=UNIT_ALL, atom_cost: int = 1,
                     flags: int = 0) -> Result:
        """ltlf_solve on the library's static 64 MiB workspace (no device
        allocation; see include/ltlf.h)."""
        bound = int(cost_bound if cost_bound is not None else problem.cost_bound)
        res, bufs = _result_buffers(bound)
        lengths, letters, positive = problem.arrays()
        st = ltlf_solve_static(self._ctx, problem.n_props, lengths, letters, positive, op_cost, atom_cost, bound,
                               flags, self._stream(), res)
        if st < 0:
            raise LtlfError(st, "ltlf_solve_static", ltlf_ctx_last_error(self._ctx))
        return _result_of(st, res, bufs)

    def autotune(self) -> List[dict]:
        """Measures the generation kernels per row-width class and keeps the
        fastest in the context (ltlf_autotune in include/ltlf.h).  Returns one
        entry per class: chunks, chosen kernel, cost bound and candidates of
        the timed runs, ns per candidate of lane / group / wave (None where a
        kernel does not apply; wave with its chosen tile), the wave kernel's
        pair-tile side and its ns per candidate with sides 8, 16, 32."""
        t = ltlf_tuning()
        st = ltlf_autotune(self._ctx, self._stream(), t)
        if st != OK:
            raise LtlfError(st, "ltlf_autotune", ltlf_ctx_last_error(self._ctx))
        self._tuning = t
        names = {FLAG_KERNEL_LANE: "lane", FLAG_KERNEL_GROUP: "group", FLAG_KERNEL_WAVE: "wave"}
        return [{"chunks": t.chunks[i], "kernel": names[t.kernel[i]], "bound": t.bound[i],
                 "candidates": t.candidates[i],
                 "ns_per_candidate": {n: (round(t.ns_per_candidate[i][j], 4) if t.ns_per_candidate[i][j] else None)
                                      for j, n in enumerate(("lane", "group", "wave"))},
                 "wave_tile": t.wave_tile[i],
                 "ns_wave_tile": {w: round(t.ns_wave_tile[i][j], 4) for j, w in enumerate((8, 16, 32))}}
                for i in range(t.n_classes)]

    def set_tuning(self, tuning: Optional["ltlf_tuning"]) -> None:
        """Installs a tuning table (None: the built-in kernel choice)."""
        st = ltlf_ctx_set_tuning(self._ctx, tuning)
        if st != OK:
            raise LtlfError(st, "ltlf_ctx_set_tuning")

    def solve_split(self, problem, cost_bound: Optional[int] = None, max_traces: int = 0,
                    op_cost=UNIT_ALL, atom_cost: int = 1, flags: int = 0) -> SplitResult:
        """Divide-and-conquer synthesis (ltlf_solve_split in include/ltlf.h)."""
        bound = int(cost_bound if cost_bound is not None else problem.cost_bound)
        res = ltlf_split_result()
        fbuf = ctypes.create_string_buffer(1 << 20)
        res.formula = ctypes.cast(fbuf, ctypes.c_char_p)
        res.formula_cap = len(fbuf)
        lengths, letters, positive = problem.arrays()
        st = ltlf_solve_split(self._ctx, problem.n_props, lengths, letters, positive, op_cost, atom_cost, bound,
                              max_traces, flags, self._stream(), res)
        if st < 0:
            raise LtlfError(st, "ltlf_solve_split", ltlf_ctx_last_error(self._ctx))
        return SplitResult(status=st, cost=res.cost, formula=fbuf.value.decode(), depth=res.depth,
                           parts_solved=res.parts_solved, parts_split=res.parts_split,
                           max_part_cost=res.max_part_cost, enum_ms=res.enum_ms)

    def solve_batch(self, problems, cost_bounds=None, op_cost=UNIT_ALL, atom_cost: int = 1,
                    flags: int = 0) -> List[Result]:
        """All problems in one ltlf_solve_batch call (see include/ltlf.h)."""
        bounds = [int(b) for b in (cost_bounds if cost_bounds is not None else
                                   [p.cost_bound for p in problems])]
        n = len(problems)
        results = (ltlf_result * n)()
        bufs = []
        for i in range(n):
            r, b = _result_buffers(bounds[i])
            results[i] = r
            bufs.append(b)
        st = ltlf_solve_batch(self._ctx, [(p.n_props,) + tuple(p.arrays()) for p in problems], op_cost,
                              atom_cost, bounds, flags, self._stream(), results)
        if st != OK:
            raise LtlfError(st, "ltlf_solve_batch", ltlf_ctx_last_error(self._ctx))
        return [_result_of(results[i].status, results[i], bufs[i]) for i in range(n)]

    def export_level(self, cost: int, first: int = 0, count: int = (1 << 64) - 1) -> np.ndarray:
        st, out = ltlf_export_level(self._ctx, cost, first, count)
        if st != OK:
            raise LtlfError(st, "ltlf_export_level")
        return out

    def formula_of(self, cost: int, index: int) -> str:
        st, f = ltlf_formula_of(self._ctx, cost, index)
        if st != OK:
            raise LtlfError(st, "ltlf_formula_of")
        return f


class Server:
    """A request loop on a Synthesizer's context (see ltlf_server_* in
    include/ltlf.h): submit, step, poll.  The Synthesizer must not be used for
    anything else while the server exists."""

    def __init__(self, synth: "Synthesizer", max_resident: int = 256):
        self._synth = synth
        st, self._srv = ltlf_server_create(synth._ctx, max_resident)
        if st != OK:
            raise LtlfError(st, "ltlf_server_create", ltlf_ctx_last_error(synth._ctx))
        self._bounds = {}

    def submit(self, problem, cost_bound: Optional[int] = None, op_cost=UNIT_ALL, atom_cost: int = 1,
               flags: int = 0, reserve_bytes: int = 0) -> int:
        b = int(cost_bound if cost_bound is not None else problem.cost_bound)
        lengths, letters, positive = problem.arrays()
        st, t = ltlf_server_submit(self._srv, problem.n_props, lengths, letters, positive, op_cost, atom_cost,
                                   b, flags, reserve_bytes)
        if st != OK:
            raise LtlfError(st, "ltlf_server_submit")
        self._bounds[t] = b
        return t

    def step(self) -> int:
        st, n = ltlf_server_step(self._srv, self._synth._stream())
        if st != OK:
            raise LtlfError(st, "ltlf_server_step", ltlf_ctx_last_error(self._synth._ctx))
        return n

    def poll(self, ticket: int) -> Optional[Result]:
        """The result if the request finished (the ticket is then released), else None."""
        b = self._bounds.get(ticket, 0)
        res, bufs = _result_buffers(b)
        st = ltlf_server_poll(self._srv, ticket, res)
        if st == PENDING:
            return None
        if st < 0:
            raise LtlfError(st, "ltlf_server_poll")
        del self._bounds[ticket]
        return _result_of(st, res, bufs)

    def cancel(self, ticket: int) -> None:
        st = ltlf_server_cancel(self._srv, ticket)
        if st != OK:
            raise LtlfError(st, "ltlf_server_cancel")
        self._bounds.pop(ticket, None)

    def load(self):
        """(queued, resident, free workspace bytes)."""
        st, q, r, f = ltlf_server_load(self._srv)
        if st != OK:
            raise LtlfError(st, "ltlf_server_load")
        return q, r, f

    def close(self) -> None:
        if getattr(self, "_srv", None):
            ltlf_server_destroy(self._srv)
            self._srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

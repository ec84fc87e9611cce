"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad arguments before touching a device."""
from __future__ import annotations

import ctypes
import subprocess
import os
import re

import pytest

import paper_2504_18943_amd as m
from paper_2504_18943_amd import ltlf as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ltlf.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ltlf_[a-z_]+)\s*\(", src)))


def test_status_values_match_header():
    src = open(HEADER).read()
    for name, val in (("LTLF_OK", 0), ("LTLF_NOT_FOUND", 1), ("LTLF_CAPACITY", 2), ("LTLF_PENDING", 3),
                      ("LTLF_CANCELLED", 4)):
        assert re.search(rf"\b{name} = {val},", src), name
    assert L.CANCELLED == 4 and L.STATUS_NAMES[4] == "CANCELLED"
    assert re.search(r"#define LTLF_FLAG_DIGEST 0x40u", src) and L.FLAG_DIGEST == 0x40


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ["ltlf_ctx_create", "ltlf_ctx_set_workspace", "ltlf_ctx_set_row_limit", "ltlf_ctx_cancel",
                 "ltlf_ctx_destroy", "ltlf_load", "ltlf_run", "ltlf_solve",
                 "ltlf_export_level", "ltlf_formula_of", "ltlf_status_str"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = m.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_mirrors_every_entry_point():
    for name in declared_functions():
        assert callable(getattr(m, name)), name


def test_status_strings():
    for st in (0, 1, 2, 3, 4, -1, -2, -3, -4, -5):
        assert m.ltlf_status_str(st)
    assert m.ltlf_status_str(99) == "unknown status"
    assert m.ltlf_status_str(4) == "cancelled"


def test_null_arguments_rejected_without_device():
    lib = m.load_library()
    assert lib.ltlf_ctx_create(0, 0, None) == L.EINVAL
    assert lib.ltlf_load(None, None, None) == L.EINVAL
    res = L.ltlf_result()
    c = L.ltlf_costs()
    assert lib.ltlf_run(None, ctypes.byref(c), 5, 0, None, ctypes.byref(res)) == L.EINVAL
    assert lib.ltlf_ctx_set_workspace(None, None, 0) == L.EINVAL
    assert lib.ltlf_ctx_set_row_limit(None, 5) == L.EINVAL
    assert lib.ltlf_ctx_cancel(None) == L.EINVAL
    n, cw = ctypes.c_uint64(), ctypes.c_uint64()
    assert lib.ltlf_export_level(None, 1, 0, 1, None, 0, ctypes.byref(n), ctypes.byref(cw)) == L.EINVAL
    sres = L.ltlf_split_result()
    assert lib.ltlf_solve_split(None, None, ctypes.byref(c), 5, 0, 0, None, ctypes.byref(sres)) == L.EINVAL
    assert lib.ltlf_autotune(None, None, None) == L.EINVAL
    assert lib.ltlf_ctx_set_tuning(None, None) == L.EINVAL
    lib.ltlf_ctx_destroy(None)  # no-op


def test_struct_layouts_match_header():
    # ltlf_costs: 8 uint32; ltlf_spec: 2 uint32 + 3 pointers
    assert ctypes.sizeof(L.ltlf_costs) == 32
    assert ctypes.sizeof(L.ltlf_spec) == 8 + 3 * ctypes.sizeof(ctypes.c_void_p)
    assert ctypes.sizeof(L.ltlf_result) == 4 * 4 + 8 * 8 + 4 * 4 + 3 * 8 + 8 + 8


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Sizes and field offsets of the result structs as gcc lays them out
    from the header, against the binding's ctypes declarations."""
    fields = {"ltlf_result": [f for f, _ in L.ltlf_result._fields_],
              "ltlf_split_result": [f for f, _ in L.ltlf_split_result._fields_],
              "ltlf_tuning": [f for f, _ in L.ltlf_tuning._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ltlf.h"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for st, fs in fields.items():
        cls = getattr(L, st)
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in fs:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, f"{st}.{f}"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError):
        L.load_library()

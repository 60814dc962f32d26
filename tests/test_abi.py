"""CPU checks of the C ABI: the library loads, exports every function that
include/ccmi.h declares, the ctypes structs match the C layout, and host-side
argument validation rejects bad calls before any device work."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_1409_2065_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccmi.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cc_[A-Za-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = _declared_functions()
    for must in ["cc_problem_create", "cc_solve", "cc_solve_path", "cc_get_U", "cc_get_labels",
                 "cc_get_fused_edges", "cc_build_knn_weights", "cc_problem_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []
    assert set(names) == set(_lib.SIGNATURES), "binding must cover exactly the header"
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (cc_[A-Za-z_]+)\b", out))
    assert set(names) <= exported


def test_struct_layout_matches_c():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "ccmi.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(cc_solve_opts), sizeof(cc_solve_info),
         offsetof(cc_solve_opts, max_iter), offsetof(cc_solve_opts, record_objective),
         offsetof(cc_solve_info, gamma), offsetof(cc_solve_info, seconds));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        got = list(map(int, subprocess.run([exe], capture_output=True, text=True).stdout.split()))
    O, I = _lib.SolveOpts, _lib.SolveInfo
    assert got == [C.sizeof(O), C.sizeof(I), O.max_iter.offset, O.record_objective.offset,
                   I.gamma.offset, I.seconds.offset]


def test_defaults_and_strings():
    lib = _lib.load()
    o = _lib.default_opts()
    assert o.struct_size == C.sizeof(_lib.SolveOpts)
    assert o.eta == 1e-2 and o.tol == 1e-6 and o.warm_start == 1
    assert lib.cc_status_string(_lib.CC_ERR_NUMERIC) == b"CC_ERR_NUMERIC"
    assert lib.cc_version() >= 100


def test_host_validation_rejects_before_device_work():
    lib = _lib.load()
    h = C.c_void_p()
    # n = 0
    st = lib.cc_problem_create(0, 3, 0, C.c_void_p(16), 3, None, 3, 0, None, None, None, 1, None, C.byref(h))
    assert st == _lib.CC_ERR_INVALID_ARG
    assert b"n >= 1" in lib.cc_last_error_message()
    # ldx < p
    st = lib.cc_problem_create(4, 3, 0, C.c_void_p(16), 2, None, 3, 0, None, None, None, 1, None, C.byref(h))
    assert st == _lib.CC_ERR_INVALID_ARG
    # unknown precision
    st = lib.cc_problem_create(4, 3, 0, C.c_void_p(16), 3, None, 3, 0, None, None, None, 7, None, C.byref(h))
    assert st == _lib.CC_ERR_INVALID_ARG
    # kNN: k >= n
    ne = C.c_int64()
    st = lib.cc_build_knn_weights(5, 2, 0, C.c_void_p(16), 2, None, 2, 5, 0.5, 0, C.c_void_p(16),
                                  C.c_void_p(16), C.c_void_p(16), 25, C.byref(ne), None, None)
    assert st == _lib.CC_ERR_INVALID_ARG
    # solve on a NULL problem
    assert lib.cc_solve(None, 1.0, None, None) == _lib.CC_ERR_INVALID_ARG
    # opts with a wrong struct_size
    o = _lib.default_opts()
    o.struct_size = 3
    assert lib.cc_solve(C.c_void_p(8), 1.0, C.byref(o), None) == _lib.CC_ERR_INVALID_ARG

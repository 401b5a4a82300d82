"""Host-side checks of the C ABI (no GPU needed, no compute calls).

The library must load, export every entry point that include/qdot.h
declares, and the ctypes structures of the binding must have the same size
and field offsets as the C structures (checked with a probe compiled by
gcc from the header itself).
"""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2105_00115_amd as q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qdot.h")


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(q.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"QDOT_API\s+[\w\s\*]+?\b(qdot\w*)\s*\(", text)))


def test_header_declares_the_expected_entry_points():
    names = declared_functions()
    for must in ("qdot", "qdot_async", "qdot_create", "qdot_destroy", "qdot_cg",
                 "qdot_power", "qdot_fp64_dot_async", "qdot_classes_async"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = C.CDLL(q.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    # and the binding covers exactly the declared ABI
    assert sorted(n for n, _, _ in q.SIGNATURES) == declared_functions()


def test_binding_loads():
    L = q.lib()
    assert L.qdot_last_error(None) == b"null handle"
    # argument checks run on the host before any device work
    assert L.qdot_destroy(None) == q.OK
    assert L.qdot_create(None, 0) == q.E_INVAL


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "qdot.h"
#define P(T, F) printf(#T "." #F " %zu\n", offsetof(T, F))
int main(void) {
  printf("qdot_result %zu\n", sizeof(qdot_result));
  printf("qdot_options %zu\n", sizeof(qdot_options));
  printf("qdot_csr %zu\n", sizeof(qdot_csr));
  printf("qdot_cg_result %zu\n", sizeof(qdot_cg_result));
  printf("qdot_tune %zu\n", sizeof(qdot_tune));
  printf("qdot_cg_system %zu\n", sizeof(qdot_cg_system));
  printf("qdot_solver_tune %zu\n", sizeof(qdot_solver_tune));
  P(qdot_result, value); P(qdot_result, count); P(qdot_result, n_zero);
  P(qdot_result, e_min); P(qdot_result, e_max); P(qdot_result, n_bins);
  P(qdot_result, t); P(qdot_result, part); P(qdot_result, bound_rel);
  P(qdot_result, bound_abs); P(qdot_result, flags); P(qdot_result, status);
  P(qdot_csr, n); P(qdot_csr, nnz); P(qdot_csr, rowptr); P(qdot_csr, col); P(qdot_csr, val);
  P(qdot_cg_result, iters); P(qdot_cg_result, status); P(qdot_cg_result, relres_est);
  P(qdot_cg_result, relres_true);
  P(qdot_cg_system, A); P(qdot_cg_system, b); P(qdot_cg_system, x); P(qdot_cg_system, rtol);
  P(qdot_cg_system, qtol); P(qdot_cg_system, maxit); P(qdot_cg_system, use_qdot);
  return 0;
}
"""


def test_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "probe.c"
    exe = tmp_path / "probe"
    src.write_text(PROBE)
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    types = {"qdot_result": q.QdotResult, "qdot_options": q.QdotOptions,
             "qdot_csr": q.QdotCsr, "qdot_cg_result": q.QdotCgResult,
             "qdot_tune": q.QdotTune, "qdot_cg_system": q.QdotCgSystem,
             "qdot_solver_tune": q.QdotSolverTune}
    for k, v in got.items():
        if "." in k:
            t, f = k.split(".")
            assert getattr(types[t], f).offset == int(v), k
        else:
            assert C.sizeof(types[k]) == int(v), k


def test_header_has_no_torch_or_hip_types():
    text = open(HEADER).read()
    assert "torch" not in text.lower().replace("pytorch", "")
    assert "hipStream_t" not in re.sub(r"/\*.*?\*/", "", text, flags=re.S)

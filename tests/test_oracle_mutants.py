"""The pins must catch plausible oracle mistakes.

Each case plants one mistake (a dropped term, a wrong sign or index, a
transposed operand, an off-by-one window) in a temporary copy of the oracle's
C source, builds it, points the oracle module at it, and checks that at least
one pin of ``test_oracle.py`` fails.  Everything runs on the CPU.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle as T

SRC = os.path.join(os.path.dirname(oracle.__file__), "spc5_oracle.c")

MUTANTS = {
    "o1_sign": ("double p = values[k] * x[colidx[k]];\n            s = s + p;",
                "double p = values[k] * x[colidx[k]];\n            s = s - p;"),
    "o1_index": ("double p = values[k] * x[colidx[k]];",
                 "double p = values[k] * x[colidx[k] > 0 ? colidx[k] - 1 : 0];"),
    "o1_dropped_term": ("for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {\n            double p = values[k] * x[colidx[k]];",
                        "for (int64_t k = rowptr[i] + 1; k < rowptr[i + 1]; ++k) {\n            double p = values[k] * x[colidx[k]];"),
    "o2_transposed": ("double p = values[k] * ybar[i];",
                      "double p = values[k] * ybar[colidx[k] % nrows];"),
    "o3_window_wide": ("(int64_t)colidx[cur[i]] < anchor + c",
                       "(int64_t)colidx[cur[i]] <= anchor + c"),
    "o3_bit_shift": ("m |= 1u << (colidx[cur[i]] - anchor);",
                     "m |= 1u << (colidx[cur[i]] - anchor + (c > 1 ? 1 : 0));"),
    "o3_anchor_max": ("(anchor < 0 || colidx[cur[i]] < anchor)",
                      "(anchor < 0 || colidx[cur[i]] > anchor)"),
    "o4_col_offset": ("colidx[fill[row]] = blk_col[b] + k;",
                      "colidx[fill[row]] = blk_col[b] + k + (k > 0);"),
    "o5_packed_order": ("oracle_csr_spmv(nrows, rowptr, colidx, values, x, y);",
                        "oracle_csr_spmv(nrows, rowptr, colidx, packed, x, y);"),
    "o5_top_bit": ("oracle_spc5_to_csr(nrows, r, c, blk_ptr",
                   "oracle_spc5_to_csr(nrows, r, c > 1 ? c - 1 : c, blk_ptr"),
    "o1par_sign": ("double q = values[k] * x[colidx[k]];\n                s = s + q;",
                   "double q = values[k] * x[colidx[k]];\n                s = s - q;"),
    "o1par_split": ("hi = nrows * (t + 1) / nt;",
                    "hi = nrows * (t + 1) / nt - (t + 1 < nt ? 1 : 0);"),
    "o6_row": ("vbar[v] = ybar[p * r + i] * x[blk_col[b] + k];",
               "vbar[v] = ybar[p * r] * x[blk_col[b] + k];"),
}


def _pins():
    cases = T.edge_cases()
    A_tiny = T.tiny_cases()
    yield lambda: [T.test_csr_spmv_vs_dense_and_scipy(a) for a in A_tiny[10:20]]
    yield lambda: [T.test_csr_spmv_par_bitwise(a, n) for a in cases[:12] for n in (2, 3)]
    yield lambda: T.test_csr_spmv_unit_vectors_give_columns()
    yield lambda: [T.test_transpose_vs_dense(a) for a in A_tiny[::3]]
    yield lambda: T.test_transpose_adjoint_and_unit_rows()
    yield lambda: [T.test_round_trip_and_invariants(a, rc) for a in cases[:12]
                   for rc in [(1, 8), (2, 4), (4, 4), (3, 5)]]
    yield lambda: [T.test_block_count_is_minimum_cover(rc, 0) for rc in [(1, 4), (4, 4)]]
    yield lambda: [T.test_laplacian_closed_forms(N) for N in (8, 16)]
    yield lambda: T.test_fig3_expand_golden()
    yield lambda: [T.test_spc5_product_equals_csr_definition_bitwise(a, rc) for a in cases[:12]
                   for rc in [(1, 8), (2, 4), (4, 4)]]
    yield lambda: [T.test_values_grad_by_exact_central_difference(rc) for rc in [(2, 4)]]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor must be unique"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O3", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(mpath)])
    monkeypatch.setattr(oracle, "_LIB", str(lib))
    monkeypatch.setattr(oracle, "_lib", None)
    monkeypatch.setattr(oracle, "build", lambda force=False: str(lib))
    caught = False
    for pin in _pins():
        try:
            with np.errstate(all="ignore"):
                pin()
        except Exception:
            caught = True
            break
    monkeypatch.setattr(oracle, "_lib", None)
    assert caught, f"no pin caught mutant {name}"

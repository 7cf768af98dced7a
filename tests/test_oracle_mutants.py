"""The pins must catch plausible oracle mistakes.  Each case plants one
mistake in a copy of the oracle's C source (a wrong sign, a dropped term, a
wrong or transposed index, a wrong comparison), builds that copy with gcc,
swaps it in for the real oracle and checks that at least one pin fails.
CPU only: the mistakes are planted in the oracle, never in GPU code."""
import ctypes
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_analysis as T_an
from tests import test_oracle_dot as T_dot
from tests import test_oracle_solvers as T_sol
from tests import test_oracle_spmv as T_spmv

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()

MUTANTS = {
    "spmv_sign": ("s += vals[k] * x[col_idx[k]];", "s -= vals[k] * x[col_idx[k]];",
                  [T_spmv.test_paper_5x5_products, T_spmv.test_against_scipy_csr]),
    "spmv_index": ("s += vals[k] * x[col_idx[k]];",
                   "s += vals[k] * x[k - row_ptr[i]];",
                   [T_spmv.test_paper_5x5_products, T_spmv.test_against_scipy_csr]),
    "spmv_drop_last": ("for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)\n"
                       "            s += vals[k] * x[col_idx[k]];",
                       "for (int32_t k = row_ptr[i]; k < row_ptr[i + 1] - 1; ++k)\n"
                       "            s += vals[k] * x[col_idx[k]];",
                       [T_spmv.test_paper_5x5_products]),
    "spmv_f32_index": ("s += (double)vals[k] * (double)x[col_idx[k]];\n        y[i] = s;",
                       "s += (double)vals[k] * (double)x[k % 5];\n        y[i] = s;",
                       [T_spmv.test_f32_storage_is_widened_exactly]),
    "dot_shift": ("double p = a[i] * b[i];", "double p = a[i] * b[i > 0 ? i - 1 : 0];",
                  [T_dot.test_fsum_correctly_rounded_reference]),
    "dot_compensation_sign": ("c += (s - t) + p;", "c -= (s - t) + p;",
                              [T_dot.test_ill_conditioned_sums_match_fsum]),
    "cg_direction": ("p[i] = r[i] + beta * p[i];", "p[i] = r[i] + beta * r[i];",
                     [T_sol.test_cg_matches_direct_solve,
                      T_sol.test_cg_finite_termination_k_eigenvalues]),
    "cg_update": ("x[i] += alpha * p[i];", "x[i] += alpha * r[i];",
                  [T_sol.test_cg_matches_direct_solve,
                   T_sol.test_cg_finite_termination_k_eigenvalues]),
    "pagerank_teleport": ("y[i] = d * s + tele;", "y[i] = d * s;",
                          [T_sol.test_pagerank_mass_identity]),
    "pagerank_no_feedback": ("memcpy(x_inout, y, sizeof(double) * (size_t)rows);", "",
                             [T_sol.test_pagerank_cycle_several_steps_closed_form]),
    "abs_f32_drops_x": ("s += fabs((double)vals[k]) * fabs((double)x[col_idx[k]]);",
                        "s += fabs((double)vals[k]);",
                        [T_spmv.test_abs_scale_f32_is_the_widened_magnitude]),
    "bins_compare": ("len > upper[b]", "len >= upper[b]",
                     [T_an.test_bins_match_searchsorted_and_stable_sort]),
    "jds_perm_direction": ("perm[order[p]] = p;", "perm[p] = order[p];",
                           [T_an.test_jds_paper_example]),
    "chunks_off_by_one": ("c_k1[m] = (e - k > chunk) ? k + chunk : e;",
                          "c_k1[m] = (e - k > chunk) ? k + chunk - 1 : e;",
                          [T_an.test_split_chunks_cover_long_rows_exactly]),
    "bfs_depth": ("level[v] = depth + 1;", "level[v] = depth + 2;",
                  [T_an.test_bfs_levels_match_scipy_distances]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, golden_dir):
    find, repl, pins = MUTANTS[name]
    assert SRC.count(find) >= 1, name
    src = SRC.replace(find, repl, 1)
    c = tmp_path / "mut.c"
    so = tmp_path / "libmut.so"
    c.write_text(src)
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(c), "-lm"])
    mut = ctypes.CDLL(str(so))
    oracle._declare(mut)
    saved = oracle.lib()
    oracle._lib = mut
    try:
        caught = 0
        for pin in pins:
            try:
                if "golden_dir" in pin.__code__.co_varnames[:pin.__code__.co_argcount]:
                    pin(golden_dir)
                else:
                    pin()
            except AssertionError:
                caught += 1
        assert caught >= 1, f"mutant {name} survived every pin"
    finally:
        oracle._lib = saved

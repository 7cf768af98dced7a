"""Pins for the oracle's CSR SpMV: values the paper's worked example fixes,
dense matvec, exact rational arithmetic, identity/permutation special cases
and the scipy CSR routine.  CPU only."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle

U64 = 2.0 ** -53


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def test_paper_5x5_products(golden_dir):
    g = _load(golden_dir, "csr_5x5.json")
    rp, ci, v = g["row_ptr"], g["col_ind"], np.array(g["val"], float)
    # the hand-written dense form agrees with numpy on the fixture itself
    dense = np.array(g["dense"], float)
    assert np.array_equal(dense @ np.array(g["x_ramp"], float), g["y_ramp"])
    assert np.array_equal(oracle.spmv_csr(rp, ci, v, g["x_ones"]), g["y_ones"])
    assert np.array_equal(oracle.spmv_csr(rp, ci, v, g["x_ramp"]), g["y_ramp"])
    # float32 storage path gives the same exact integers
    y32 = oracle.spmv_csr(rp, ci, v.astype(np.float32),
                          np.array(g["x_ramp"], np.float32))
    assert np.array_equal(y32, g["y_ramp"])
    assert oracle.cols(ci) == g["cols"]
    assert oracle.validate(rp, ci) == 0


def test_dense_matvec_tiny_with_duplicates_and_unsorted():
    for seed in range(5):
        A = gen.ragged(37, 23, seed=seed, max_len=40, dup=True, sort_cols=False)
        x = gen.vector(A.cols, seed + 100)
        dense = np.zeros((A.rows, A.cols))
        for i in range(A.rows):
            for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
                dense[i, A.col_idx[k]] += A.vals[k]
        y = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x)
        scale = np.abs(dense) @ np.abs(x)
        assert np.all(np.abs(y - dense @ x) <= 64 * U64 * scale + 1e-300)


def test_exact_rational_bound():
    """Against exact rational arithmetic: the recursive-summation error bound
    |y - exact| <= gamma_len * sum|a||x| must hold row by row."""
    A = gen.ragged(25, 40, seed=7, max_len=30, dup=True)
    x = gen.vector(A.cols, 8)
    y = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x)
    for i in range(A.rows):
        a, b = A.row_ptr[i], A.row_ptr[i + 1]
        exact = sum((Fraction(float(A.vals[k])) * Fraction(float(x[A.col_idx[k]]))
                     for k in range(a, b)), Fraction(0))
        mag = sum(abs(float(A.vals[k]) * float(x[A.col_idx[k]])) for k in range(a, b))
        n = b - a
        gamma = n * U64 / (1 - n * U64) if n else 0.0
        assert abs(Fraction(float(y[i])) - exact) <= Fraction(gamma * mag * 1.0000001)


def test_identity_and_permutation_bitwise():
    x = gen.vector(1000, 3)
    I = gen.identity(1000)
    assert np.array_equal(oracle.spmv_csr(I.row_ptr, I.col_idx, I.vals, x), x)
    P = gen.permutation(1000, 4)
    assert np.array_equal(oracle.spmv_csr(P.row_ptr, P.col_idx, P.vals, x),
                          x[P.col_idx])


def test_row_sums_with_ones_integer_exact():
    A = gen.ragged(500, 300, seed=11, max_len=120, integer_vals=True)
    S = sp.csr_matrix((A.vals, A.col_idx, A.row_ptr), shape=(A.rows, A.cols))
    y = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, np.ones(A.cols))
    assert np.array_equal(y, np.asarray(S.sum(axis=1)).ravel())


def test_against_scipy_csr():
    A = gen.ragged(3000, 2000, seed=12, max_len=300, long_rows=3, long_len=1500)
    x = gen.vector(A.cols, 13)
    S = sp.csr_matrix((A.vals, A.col_idx, A.row_ptr), shape=(A.rows, A.cols))
    y = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x)
    ref = S @ x
    mag = abs(S) @ np.abs(x)
    assert np.all(np.abs(y - ref) <= 1e-13 * mag)
    # the magnitude helper agrees with the library's |A||x|
    assert np.allclose(oracle.spmv_abs(A.row_ptr, A.col_idx, A.vals, x), mag,
                       rtol=1e-13, atol=0)


def test_integer_inputs_exact_any_order():
    A = gen.ragged(4000, 4000, seed=14, max_len=400, long_rows=2, long_len=8000,
                   integer_vals=True)
    x = gen.int_vector(A.cols, 15)
    S = sp.csr_matrix((A.vals, A.col_idx, A.row_ptr), shape=(A.rows, A.cols))
    assert np.array_equal(oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x), S @ x)


def test_empty_rows_and_empty_matrix():
    A = gen.ragged(200, 50, seed=16, empty_frac=0.5)
    x = gen.vector(A.cols, 17)
    y = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x)
    empty = np.diff(A.row_ptr) == 0
    assert empty.any()
    assert np.all(y[empty] == 0.0) and not np.any(np.signbit(y[empty]))
    E = gen.empty_matrix(10, 0)
    assert np.array_equal(oracle.spmv_csr(E.row_ptr, E.col_idx, E.vals, np.zeros(1)),
                          np.zeros(10))
    assert oracle.cols(E.col_idx) == 0


def test_f32_storage_is_widened_exactly():
    A = gen.ragged(300, 300, seed=18, max_len=100).astype(np.float32)
    x = gen.vector(A.cols, 19, dtype=np.float32)
    y32 = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x)
    y64 = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals.astype(np.float64),
                          x.astype(np.float64))
    assert np.array_equal(y32, y64)
    S = sp.csr_matrix((A.vals.astype(np.float64), A.col_idx, A.row_ptr),
                      shape=A.rows and (A.rows, A.cols))
    assert np.allclose(y32, S @ x.astype(np.float64), rtol=0,
                       atol=1e-13 * np.max(np.abs(S) @ np.abs(x.astype(np.float64))))


def test_nan_propagates():
    A = gen.ragged(50, 50, seed=20, max_len=10, empty_frac=0.0)
    x = gen.vector(A.cols, 21)
    j = int(A.col_idx[0])
    x[j] = np.nan
    y = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x)
    touches = np.array([j in A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
                        for i in range(A.rows)])
    assert np.array_equal(np.isnan(y), touches)



def test_row_parallel_product_is_the_serial_one():
    """The host-baseline product that shares rows among threads forms every
    row exactly as the serial loop does."""
    A = gen.ragged(20000, 30000, seed=31, max_len=300, long_rows=2, long_len=9000)
    x = gen.vector(A.cols, 32)
    y = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x)
    yp = oracle.spmv_csr_par(A.row_ptr, A.col_idx, A.vals, x)
    assert np.array_equal(y, yp)
    assert oracle.threads() >= 1


def test_abs_scale_f32_is_the_widened_magnitude():
    """The float32 tolerance scale: sum_k |a_ik| |x_k| of the float32 data
    widened to binary64, against the library product |A| |x| of the widened
    arrays.  Products of two float32 values are exact in binary64, so the
    two differ only by the rounding of the row sums."""
    A = gen.ragged(500, 700, seed=33, max_len=120, empty_frac=0.1).astype(np.float32)
    x = gen.vector(A.cols, 34, dtype=np.float32)
    S = sp.csr_matrix((np.abs(A.vals.astype(np.float64)), A.col_idx, A.row_ptr),
                      shape=(A.rows, A.cols))
    want = S @ np.abs(x.astype(np.float64))
    got = oracle.spmv_abs(A.row_ptr, A.col_idx, A.vals, x)
    assert got.dtype == np.float64
    lens = np.diff(A.row_ptr)
    assert np.all(np.abs(got - want) <= 2.3e-16 * lens * want)
    # a row with one entry holds that product exactly
    one = np.nonzero(lens == 1)[0]
    assert one.size
    k = A.row_ptr[one]
    assert np.array_equal(got[one], np.abs(A.vals[k].astype(np.float64)) *
                          np.abs(x[A.col_idx[k]].astype(np.float64)))

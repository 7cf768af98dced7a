"""Shared checks for the GPU parity tests (tolerances follow the stated
bounds: float64 products within 1e-12 of sum|a||x| per row, float32 within
1e-5; structure and integer work bit-exact)."""
import numpy as np

import oracle

TOL_F64 = 1e-12
TOL_F32 = 1e-5


def assert_rows_close(y, ref, mag, tol, what=""):
    y = np.asarray(y, dtype=np.float64)
    err = np.abs(y - ref)
    bad = ~(err <= tol * mag)
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(
            f"{what}: {int(bad.sum())} rows out of tolerance; first row {i}: "
            f"got {y[i]!r} want {ref[i]!r} scale {mag[i]!r}")


def check_spmv(A, x, y, tol):
    """y (device result copied to host) against the oracle, row by row."""
    ref = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x)
    # the stated scale alone: a float32 row is its binary64 sum rounded once
    # (at most 2^-24 |y| <= 2^-24 sum|a||x|), far inside 1e-5 sum|a||x|
    mag = oracle.spmv_abs(A.row_ptr, A.col_idx, A.vals, x)
    assert_rows_close(y, ref, mag, tol, A.name)
    empty = np.diff(A.row_ptr) == 0
    assert np.all(np.asarray(y)[empty] == 0)

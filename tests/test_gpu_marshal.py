"""Marshaling modes of the paper-shaped raw call on the GPU: cached device
copies (default), automatic re-upload after host writes (page protection)
and the naive per-call upload."""
import os

import numpy as np
import pytest

import gen
import paper_2001_07938_amd as L
from tests.helpers import TOL_F64, check_spmv

pytestmark = pytest.mark.gpu


@pytest.fixture
def marshal_env():
    old = os.environ.get("LILAC_MARSHAL")
    yield
    L.lilac_release_all()
    if old is None:
        os.environ.pop("LILAC_MARSHAL", None)
    else:
        os.environ["LILAC_MARSHAL"] = old




def test_protect_mode_picks_up_host_writes(marshal_env):
    os.environ["LILAC_MARSHAL"] = "protect"
    A = gen.ragged(3000, 20000, seed=1, max_len=200)
    rp, ci, vals = A.row_ptr.copy(), A.col_idx.copy(), A.vals.copy()
    x = gen.vector(A.cols, 2)
    y = np.empty(A.rows)
    L.lilac_spmv_csr(A.rows, rp, ci, vals, x, y)
    check_spmv(A, x, y, TOL_F64)
    vals *= -3.0           # a host write to the cached values: no invalidate call
    L.lilac_spmv_csr(A.rows, rp, ci, vals, x, y)
    check_spmv(gen.Csr(A.rows, A.cols, rp, ci, vals), x, y, TOL_F64)
    ci[:] = (ci + 1) % A.cols  # a structural write
    L.lilac_spmv_csr(A.rows, rp, ci, vals, x, y)
    check_spmv(gen.Csr(A.rows, A.cols, rp, ci, vals), x, y, TOL_F64)
    L.lilac_spmv_csr(A.rows, rp, ci, vals, x, y)  # unchanged: cached copy
    check_spmv(gen.Csr(A.rows, A.cols, rp, ci, vals), x, y, TOL_F64)


def test_default_mode_needs_invalidate(marshal_env):
    os.environ.pop("LILAC_MARSHAL", None)
    A = gen.ragged(2000, 5000, seed=3, max_len=100)
    vals = A.vals.copy()
    x = gen.vector(A.cols, 4)
    y = np.empty(A.rows)
    L.lilac_spmv_csr(A.rows, A.row_ptr, A.col_idx, vals, x, y)
    y0 = y.copy()
    vals[:] = 0.0
    L.lilac_spmv_csr(A.rows, A.row_ptr, A.col_idx, vals, x, y)
    assert np.array_equal(y, y0)          # stale by design
    L.lilac_invalidate(vals[100:])        # any address inside the array
    L.lilac_spmv_csr(A.rows, A.row_ptr, A.col_idx, vals, x, y)
    assert np.all(y == 0.0)


def test_naive_mode_uploads_every_call(marshal_env):
    os.environ["LILAC_MARSHAL"] = "naive"
    A = gen.ragged(2000, 5000, seed=5, max_len=100)
    vals = A.vals.copy()
    x = gen.vector(A.cols, 6)
    y = np.empty(A.rows)
    L.lilac_spmv_csr(A.rows, A.row_ptr, A.col_idx, vals, x, y)
    check_spmv(A, x, y, TOL_F64)
    vals[:] = 1.0
    L.lilac_spmv_csr(A.rows, A.row_ptr, A.col_idx, vals, x, y)
    check_spmv(gen.Csr(A.rows, A.cols, A.row_ptr, A.col_idx, vals), x, y, TOL_F64)

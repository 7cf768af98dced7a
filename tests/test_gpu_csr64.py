"""GPU parity of the handles with 64-bit row offsets (consecutive row parts,
each an ordinary handle) against the oracle, through the C ABI: small
matrices split into several parts by a lowered part bound, and one matrix
with more than 2^31 non-zeros."""
import os

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2001_07938_amd as L
from tests.helpers import TOL_F32, TOL_F64, check_spmv

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _expected_parts(row_ptr, lim):
    """First rows of the parts: greedy, each part as many whole rows as fit
    in lim non-zeros."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    rows = rp.size - 1
    firsts, r0 = [], 0
    while r0 < rows:
        firsts.append(r0)
        r1 = int(np.searchsorted(rp, rp[r0] + lim, side="right")) - 1
        r0 = r1
    return firsts


@pytest.fixture
def part_bound():
    """Sets LILAC_PART_NNZ (read when a matrix is created) for one test."""
    old = os.environ.get("LILAC_PART_NNZ")

    def set_(n):
        os.environ["LILAC_PART_NNZ"] = str(n)
    yield set_
    if old is None:
        os.environ.pop("LILAC_PART_NNZ", None)
    else:
        os.environ["LILAC_PART_NNZ"] = old


SMALL = {
    # row lengths from 0 to 20000 (long rows split into chunks inside a part)
    "ragged_long_rows": (lambda: gen.ragged(3000, 40000, seed=1, max_len=300,
                                            long_rows=3, long_len=20000), 40000),
    # gather-heavy parts (column panels)
    "random5_60": (lambda: gen.random_rows(60000, 5, 60, seed=7), 400000),
    # local columns (band layout)
    "stencil27": (lambda: gen.stencil(20, 27), 50000),
    "mostly_empty": (lambda: gen.ragged(5000, 5000, seed=3, empty_frac=0.7), 5000),
}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_csr64_parts_parity(name, part_bound):
    make, lim = SMALL[name]
    A = make()
    part_bound(lim)
    m = L.Csr64.from_gen(A, cols=A.cols)
    firsts = _expected_parts(A.row_ptr, lim)
    assert len(firsts) >= 2, name
    assert m.info() == (A.rows, A.cols, A.nnz, len(firsts))
    x = gen.vector(A.cols, 90)
    yd = torch.full((A.rows,), np.nan, dtype=torch.float64, device=DEV)
    m.spmv(_dev(x), yd)
    y = _host(yd)
    check_spmv(A, x, y, TOL_F64)
    m.spmv(_dev(x), yd)
    assert np.array_equal(_host(yd), y)
    m.destroy()
    # integer data: exact in any order
    A.vals = gen.int_vector(A.nnz, 91)
    xi = gen.int_vector(A.cols, 92)
    m = L.Csr64.from_gen(A, cols=A.cols)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    m.spmv(_dev(xi), yd)
    assert np.array_equal(_host(yd), oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, xi))
    m.destroy()
    # float32
    B = make().astype(np.float32)
    m = L.Csr64.from_gen(B, cols=B.cols)
    x32 = gen.vector(B.cols, 93, dtype=np.float32)
    yd = torch.empty(B.rows, dtype=torch.float32, device=DEV)
    m.spmv(_dev(x32), yd)
    check_spmv(B, x32, _host(yd), TOL_F32)
    m.destroy()


def test_csr64_device_inputs_inferred_cols_and_edges(part_bound):
    A = gen.random_rows(20000, 1, 40, seed=11, cols=70000)
    part_bound(100000)
    # device-resident arrays; cols inferred part by part, the largest kept
    m = L.Csr64(_dev(A.row_ptr.astype(np.int64)), _dev(A.col_idx), _dev(A.vals))
    rows, cols, nnz, nparts = m.info()
    assert (rows, nnz, nparts) == (A.rows, A.nnz, len(_expected_parts(A.row_ptr, 100000)))
    assert cols == int(A.col_idx.max()) + 1
    x = gen.vector(A.cols, 94)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    m.spmv(_dev(x), yd)
    check_spmv(A, x, _host(yd), TOL_F64)
    m.destroy()
    # no rows: no parts, the product does nothing
    E = L.Csr64(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert E.info() == (0, 0, 0, 0)
    E.spmv(None, None)
    E.destroy()
    # rows but no entries: one part, y overwritten with zeros
    Z = L.Csr64(np.zeros(301, np.int64), np.zeros(0, np.int32), np.zeros(0), cols=5)
    assert Z.info() == (300, 5, 0, 1)
    yd = torch.full((300,), np.nan, dtype=torch.float64, device=DEV)
    Z.spmv(_dev(np.ones(5)), yd)
    assert np.array_equal(_host(yd), np.zeros(300))
    Z.destroy()


def test_csr64_errors(part_bound):
    A = gen.ragged(2000, 3000, seed=12, max_len=100, long_rows=1, long_len=2500)
    part_bound(1000)
    # one row alone is longer than a part
    with pytest.raises(L.LilacError) as e:
        L.Csr64.from_gen(A)
    assert e.value.code == -7
    part_bound(10**6)
    bad = A.row_ptr.astype(np.int64).copy()
    bad[5] = bad[6] + 1  # decreasing offsets
    with pytest.raises(L.LilacError) as e:
        L.Csr64(bad, A.col_idx, A.vals)
    assert e.value.code == -2
    short = A.row_ptr.astype(np.int64).copy()
    short[-1] -= 1       # row_ptr[rows] != nnz
    with pytest.raises(L.LilacError) as e:
        L.Csr64(short, A.col_idx, A.vals)
    assert e.value.code == -2
    badcol = A.col_idx.copy()
    badcol[7] = A.cols   # column out of range in a part
    with pytest.raises(L.LilacError) as e:
        L.Csr64(A.row_ptr.astype(np.int64), badcol, A.vals, cols=A.cols)
    assert e.value.code == -2


def test_csr64_more_than_2p31_nonzeros():
    """2^22 + 16 rows of 512 entries: 2^31 + 8192 non-zeros, float32 with
    integer values (every product exact), in two parts.  Sampled rows (the
    first and last rows, those around the part boundary and a random
    sample) against the oracle computed row by row."""
    rows, k, cols = (1 << 22) + 16, 512, 1 << 22
    A = gen.strided_rows(rows, k, cols, seed=gen.BASE_SEED + 64)
    assert A.nnz == (1 << 31) + 8192
    m = L.Csr64.from_gen(A, cols=cols)
    assert m.info() == (rows, cols, A.nnz, 2)
    x = gen.int_vector(cols, 95, dtype=np.float32, lo=-8, hi=8)
    xd = _dev(x)
    yd = torch.full((rows,), np.nan, dtype=torch.float32, device=DEV)
    m.spmv(xd, yd)
    y = _host(yd)
    m.destroy()
    lim = (1 << 31) - (1 << 20)
    b = _expected_parts(A.row_ptr, lim)[1]
    rng = np.random.default_rng(96)
    sample = np.unique(np.concatenate([
        np.arange(0, 64), np.arange(b - 64, b + 64), np.arange(rows - 64, rows),
        rng.integers(0, rows, 2048)]))
    starts = A.row_ptr[sample]
    sub_rp = np.zeros(sample.size + 1, dtype=np.int32)
    sub_rp[1:] = np.cumsum(np.full(sample.size, k))
    idx = (starts[:, None] + np.arange(k)[None, :]).reshape(-1)
    ref = oracle.spmv_csr(sub_rp, A.col_idx[idx], A.vals[idx].astype(np.float64),
                          x.astype(np.float64))
    assert np.array_equal(y[sample].astype(np.float64), ref)
    assert np.all(np.isfinite(y)) and np.all(y == np.round(y))
    assert np.abs(y).max() <= k * 64

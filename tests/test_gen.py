"""Structural invariants of the seeded input generators.  CPU only."""
import numpy as np
import scipy.sparse as sp

import gen


def _check_csr(A):
    assert A.row_ptr.dtype == np.int32 and A.col_idx.dtype == np.int32
    assert A.row_ptr[0] == 0 and np.all(np.diff(A.row_ptr) >= 0)
    assert A.row_ptr[-1] == A.col_idx.size == A.vals.size
    if A.nnz:
        assert A.col_idx.min() >= 0 and A.col_idx.max() < A.cols


def test_uniform_rows_exact_16_distinct_sorted():
    A = gen.uniform_rows(512, 16, seed=1)
    _check_csr(A)
    assert np.all(np.diff(A.row_ptr) == 16)
    c = A.col_idx.reshape(512, 16)
    assert np.all(np.diff(c, axis=1) > 0)
    assert np.all((A.vals >= -1) & (A.vals < 1))
    B = gen.uniform_rows(512, 16, seed=1)
    assert np.array_equal(A.col_idx, B.col_idx) and np.array_equal(A.vals, B.vals)


def test_spd_random_symmetric_dominant():
    A = gen.spd_random(3000, 20, seed=2)
    _check_csr(A)
    S = sp.csr_matrix((A.vals, A.col_idx, A.row_ptr), shape=(A.rows, A.cols))
    assert abs(S - S.T).max() == 0
    d = S.diagonal()
    off = np.asarray(abs(S).sum(axis=1)).ravel() - np.abs(d)
    assert np.all(d - off >= 1.0 - 1e-9)
    lens = np.diff(A.row_ptr)
    assert 2 * 20 - 5 < lens.mean() < 2 * 20 + 2
    # columns sorted and distinct within rows
    for i in range(0, A.rows, 97):
        seg = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(seg) > 0)


def test_stencil_nnz_closed_forms():
    for k in (2, 3, 7, 12):
        A7 = gen.stencil(k, 7)
        A27 = gen.stencil(k, 27)
        _check_csr(A7)
        _check_csr(A27)
        assert A7.nnz == 7 * k**3 - 6 * k**2
        assert A27.nnz == (3 * k - 2) ** 3
        S = sp.csr_matrix((A7.vals, A7.col_idx, A7.row_ptr), shape=(A7.rows,) * 2)
        assert abs(S - S.T).max() == 0
        assert np.all(S.diagonal() == 6.0)


def test_random_rows_counts():
    A = gen.random_rows(5000, 5, 60, seed=3)
    _check_csr(A)
    lens = np.diff(A.row_ptr)
    assert lens.min() >= 4 and lens.max() <= 60
    assert 30 < lens.mean() < 34


def test_rmat_quadrants_and_skew():
    src, dst = gen.rmat_edges(10, 200_000, seed=4)
    top_src = src >> 9
    top_dst = dst >> 9
    q = np.bincount(top_src * 2 + top_dst, minlength=4) / src.size
    assert np.allclose(q, [0.57, 0.19, 0.19, 0.05], atol=0.01)
    G = gen.rmat_pagerank(scale=12, n_edges=60_000, seed=5)
    _check_csr(G)
    lens = np.diff(G.row_ptr)
    assert lens.max() > 20 * lens.mean()
    outdeg = np.bincount(G.col_idx, minlength=G.rows)
    assert np.allclose(G.vals, (1.0 / outdeg[G.col_idx]).astype(np.float32))
    assert G.vals.dtype == np.float32


def test_batch_specs_and_trace():
    specs = gen.batch_specs(512)
    ns = np.array([s.n for s in specs])
    assert ns.min() >= 1000 and ns.max() <= 200_000
    kinds = [s.kind for s in specs]
    assert abs(kinds.count("st7") - 171) <= 1 and abs(kinds.count("rand") - 170) <= 1
    assert 20_000 < ns.mean() < 60_000
    tr = gen.poisson_trace(10_000.0, 20_000, seed=6)
    gaps = np.diff(tr.arrival_ns) / 1e9
    assert abs(gaps.mean() - 1e-4) < 5e-6
    assert 0.08 < np.mean(tr.matrix >= 64) < 0.12
    assert 0.18 < np.mean(tr.kind) < 0.22


def test_strided_rows_exact_k_distinct_sorted_int64_offsets():
    A = gen.strided_rows(3000, 37, 1000, seed=5, chunk_rows=512)
    assert A.row_ptr.dtype == np.int64 and A.col_idx.dtype == np.int32
    assert np.array_equal(A.row_ptr, np.arange(3001) * 37)
    c = A.col_idx.reshape(3000, 37).astype(np.int64)
    assert np.all(np.diff(c, axis=1) > 0)
    assert c.min() >= 0 and c.max() < 1000
    # every row is {(a + j*s) mod cols : j < k} for one of its own entries a
    s = 1000 // 37
    for i in range(0, 3000, 97):
        row = set(c[i].tolist())
        assert any({(a + j * s) % 1000 for j in range(37)} == row for a in c[i])
    v = A.vals
    assert np.all(v == np.round(v)) and v.min() >= -8 and v.max() <= 8
    B = gen.strided_rows(3000, 37, 1000, seed=5, chunk_rows=512)
    assert np.array_equal(A.col_idx, B.col_idx) and np.array_equal(A.vals, B.vals)
    # steps that cover cols exactly
    C = gen.strided_rows(500, 16, 256, seed=6)
    c = C.col_idx.reshape(500, 16)
    assert np.all(np.diff(c, axis=1) == 16) and np.all(c[:, 0] < 16)
    # consecutive windows
    W = gen.strided_rows(400, 9, 100, seed=7, window=True)
    w = W.col_idx.reshape(400, 9)
    assert np.all(np.diff(w, axis=1) == 1) and w.min() >= 0 and w.max() < 100

"""Pins for the oracle's structure work: binning, chunk tables, the column
count, validation, JDS conversion (the paper's example) and BFS levels.
These are integer results and must match exactly.  CPU only."""
import json
import os

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import gen
import oracle

UPPER = np.array([0, 2, 4, 8, 16, 32, 64, 4096, 2**31 - 1], dtype=np.int32)


def test_bins_match_searchsorted_and_stable_sort():
    for seed in range(4):
        A = gen.ragged(5000, 3000, seed=seed, max_len=500, long_rows=4,
                       long_len=6000, empty_frac=0.2)
        bor, off, br = oracle.bins(A.row_ptr, UPPER)
        lens = np.diff(A.row_ptr)
        # first b with len <= upper[b]: searchsorted(side="left")
        ref_bin = np.minimum(np.searchsorted(UPPER, lens, side="left"), UPPER.size - 1)
        assert np.array_equal(bor, ref_bin)
        assert np.array_equal(br, np.argsort(ref_bin, kind="stable"))
        assert np.array_equal(off, np.concatenate([[0], np.cumsum(
            np.bincount(ref_bin, minlength=UPPER.size))]))


def test_bins_last_bin_catches_overflow():
    rp = np.array([0, 10, 10, 30], dtype=np.int32)
    bor, off, br = oracle.bins(rp, np.array([0, 5, 15], dtype=np.int32))
    assert list(bor) == [2, 0, 2] and list(off) == [0, 1, 1, 3] and list(br) == [1, 0, 2]
    bor, off, br = oracle.bins(rp, np.array([0, 5], dtype=np.int32))
    assert list(bor) == [1, 0, 1] and list(br) == [1, 0, 2]


def test_split_chunks_cover_long_rows_exactly():
    A = gen.ragged(3000, 50000, seed=3, long_rows=6, long_len=30000)
    t, c = 4096, 4096
    cr, c0, c1 = oracle.split_chunks(A.row_ptr, t, c)
    lens = np.diff(A.row_ptr)
    long_rows = np.nonzero(lens > t)[0]
    assert np.array_equal(np.unique(cr), long_rows)
    assert np.all(np.diff(cr) >= 0)
    assert np.all(c1 - c0 <= c) and np.all(c1 > c0)
    for r in long_rows:
        m = cr == r
        k0, k1 = c0[m], c1[m]
        assert k0[0] == A.row_ptr[r] and k1[-1] == A.row_ptr[r + 1]
        assert np.array_equal(k0[1:], k1[:-1])
        assert np.all(k1[:-1] - k0[:-1] == c)
    assert cr.size == int(np.sum(-(-lens[long_rows] // c)))


def test_cols_and_validation():
    A = gen.ragged(100, 77, seed=1)
    assert oracle.cols(A.col_idx) == int(A.col_idx.max()) + 1
    assert oracle.validate(A.row_ptr, A.col_idx, 77) == 0
    assert oracle.validate(A.row_ptr, A.col_idx, -1) == 0
    assert oracle.validate(A.row_ptr, A.col_idx, int(A.col_idx.max())) == -4
    rp = A.row_ptr.copy()
    rp[0] = 1
    assert oracle.validate(rp, A.col_idx) == -2
    rp = A.row_ptr.copy()
    i = int(np.nonzero(np.diff(rp))[0][0])
    rp[i + 1] = rp[i] - 1
    assert oracle.validate(rp, A.col_idx) == -3
    ci = A.col_idx.copy()
    ci[3] = -1
    assert oracle.validate(A.row_ptr, ci) == -4


def test_jds_paper_example(golden_dir):
    with open(os.path.join(golden_dir, "csr_5x5.json")) as f:
        c = json.load(f)
    with open(os.path.join(golden_dir, "jds_5x5.json")) as f:
        j = json.load(f)
    got = oracle.csr_to_jds(c["row_ptr"], c["col_ind"], c["val"])
    assert list(got["perm"]) == j["perm"]
    assert list(got["val"]) == j["val"]
    assert list(got["col_ind"]) == j["col_ind"]
    assert list(got["jd_ptr"]) == j["jd_ptr"]
    assert list(got["nzcnt"]) == j["nzcnt"]
    y = oracle.spmv_jds(got, c["x_ramp"])
    assert list(y) == c["y_ramp"]


def test_jds_spmv_equals_csr_bitwise():
    A = gen.ragged(2000, 1500, seed=9, max_len=300, empty_frac=0.1)
    x = gen.vector(A.cols, 10)
    J = oracle.csr_to_jds(A.row_ptr, A.col_idx, A.vals)
    assert np.array_equal(oracle.spmv_jds(J, x),
                          oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x))
    lens = np.diff(A.row_ptr)
    assert np.array_equal(np.sort(lens)[::-1], J["nzcnt"])


def test_bfs_levels_match_scipy_distances():
    for seed in range(3):
        G = gen.rmat_pagerank(scale=9, n_edges=3000, seed=seed)
        src = int(np.argmax(np.diff(G.row_ptr)))
        lvl, nlev = oracle.bfs_levels(G.row_ptr, G.col_idx, src)
        # pull CSR row v lists sources u of u->v, i.e. the transpose graph
        S = sp.csr_matrix((np.ones(G.nnz), G.col_idx, G.row_ptr),
                          shape=(G.rows, G.rows)).T.tocsr()
        dist = csg.shortest_path(S, method="D", unweighted=True, indices=src)
        ref = np.where(np.isinf(dist), -1, dist).astype(np.int32)
        assert np.array_equal(lvl, ref)
        assert nlev == ref.max() + 1

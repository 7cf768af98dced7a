"""Pins for the oracle's conjugate gradient and PageRank: direct solves,
finite termination, the zero right-hand side, A-norm monotonicity, PageRank
mass identity, a cycle's fixed point, the closed form of several steps on a
cycle from a non-uniform start, and a star's closed form.  CPU only."""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

import gen
import oracle


def _dense(A):
    return sp.csr_matrix((A.vals.astype(np.float64), A.col_idx, A.row_ptr),
                         shape=(A.rows, A.cols)).toarray()


def test_cg_matches_direct_solve():
    A = gen.spd_random(400, 12, seed=3)
    b = gen.vector(A.rows, 4)
    M = _dense(A)
    assert np.allclose(M, M.T) and np.all(np.linalg.eigvalsh(M) > 0)
    xs = sla.cho_solve(sla.cho_factor(M), b)
    x, done, hist = oracle.cg(A.row_ptr, A.col_idx, A.vals, b, 60)
    assert done == 60 or hist[done] == 0.0
    assert np.max(np.abs(x - xs)) <= 1e-11 * np.max(np.abs(xs))
    assert hist[0] == oracle.dot(b, b)


def test_cg_finite_termination_k_eigenvalues():
    for k in (1, 2, 5):
        A = gen.diag_distinct(300, k, seed=k)
        b = gen.vector(A.rows, 10 + k)
        x, done, hist = oracle.cg(A.row_ptr, A.col_idx, A.vals, b, k)
        r = b - A.vals * x
        assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b)
        assert np.max(np.abs(x - b / A.vals)) <= 1e-12 * np.max(np.abs(b / A.vals))


def test_cg_zero_rhs_stops_with_zero():
    A = gen.spd_random(200, 5, seed=5)
    x, done, hist = oracle.cg(A.row_ptr, A.col_idx, A.vals, np.zeros(A.rows), 10)
    assert done == 0 and np.all(x == 0.0)


def test_cg_a_norm_error_monotone():
    A = gen.spd_random(300, 8, seed=6)
    b = gen.vector(A.rows, 7)
    M = _dense(A)
    xs = np.linalg.solve(M, b)
    errs = []
    for it in range(0, 12):
        x, _, _ = oracle.cg(A.row_ptr, A.col_idx, A.vals, b, it)
        e = x - xs
        errs.append(float(e @ M @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))
    assert errs[-1] < 1e-6 * errs[0]


def test_pagerank_mass_identity():
    A = gen.rmat_pagerank(scale=10, n_edges=8000, seed=9)
    n = A.rows
    x = gen.vector(n, 10, dtype=np.float32, lo=0.0, hi=1.0)
    d = 0.85
    y = oracle.pagerank_step(A.row_ptr, A.col_idx, A.vals, x, d)
    # column sums of the stored weights (1/outdeg rounded to float32)
    colsum = np.bincount(A.col_idx, weights=A.vals.astype(np.float64), minlength=n)
    outdeg = np.bincount(A.col_idx, minlength=n)
    assert np.allclose(colsum[outdeg > 0], 1.0, rtol=1e-7, atol=0)
    mass = d * np.dot(colsum, x.astype(np.float64)) + (1 - d)
    assert abs(np.sum(y) - mass) <= 1e-12 * mass


def test_pagerank_cycle_fixed_point_and_star_closed_form():
    C = gen.cycle_graph(97)
    x = np.full(97, 1.0 / 97, dtype=np.float32)
    y = oracle.pagerank_step(C.row_ptr, C.col_idx, C.vals, x, 0.85)
    assert np.allclose(y, np.float64(np.float32(1.0 / 97)) * 0.85 + 0.15 / 97,
                       rtol=1e-15, atol=0)
    xx = oracle.pagerank(C.row_ptr, C.col_idx, C.vals, np.full(97, 1 / 97), 0.85, 20)
    assert np.allclose(xx, 1 / 97, rtol=1e-14, atol=0)
    n = 33
    S = gen.star_graph(n)
    x = np.full(n, 1.0 / n, dtype=np.float32)
    xf = np.float64(np.float32(1.0 / n))
    y = oracle.pagerank_step(S.row_ptr, S.col_idx, S.vals, x, 0.85)
    hub = 0.85 * (n - 1) * xf + 0.15 / n
    leaf = 0.85 * np.float64(np.float32(1.0 / (n - 1))) * xf + 0.15 / n
    assert abs(y[0] - hub) <= 1e-15 and np.allclose(y[1:], leaf, rtol=1e-15, atol=0)


def test_pagerank_cycle_several_steps_closed_form():
    """On the directed n-cycle u -> u+1 each step moves every value one
    vertex on, so from any start x0 the k-th iterate is
        x_k[v] = d^k x0[(v - k) mod n] + (1 - d^k) / n
    (the teleport terms (1-d)/n summed over d^0 .. d^(k-1)).  A start that is
    not the fixed point makes the result depend on k and on d, so an oracle
    that does not feed each step's result into the next fails here."""
    n = 61
    C = gen.cycle_graph(n)
    x0 = gen.vector(n, 44, lo=0.0, hi=1.0)
    x0 = x0 / x0.sum()
    for d in (0.5, 0.85, 0.99):
        for k in (1, 2, 7, 20):
            want = d ** k * np.roll(x0, k) + (1.0 - d ** k) / n
            got = oracle.pagerank(C.row_ptr, C.col_idx, C.vals, x0, d, k)
            assert np.allclose(got, want, rtol=1e-13, atol=0), (d, k)
        # the step count matters from this start
        one = oracle.pagerank(C.row_ptr, C.col_idx, C.vals, x0, d, 1)
        two = oracle.pagerank(C.row_ptr, C.col_idx, C.vals, x0, d, 2)
        assert not np.allclose(one, two)

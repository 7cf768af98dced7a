"""GPU parity of the CG solve (eager and graph), the fused product + dot and
PageRank against the oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2001_07938_amd as L
from tests.helpers import TOL_F32, TOL_F64, assert_rows_close

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_spmv_dot_fused():
    A = gen.ragged(30000, 30000, seed=1, max_len=300, long_rows=3, long_len=20000)
    x = gen.vector(A.cols, 2)
    w = gen.vector(A.rows, 3)
    h = L.Csr.from_gen(A)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    out = torch.empty(1, dtype=torch.float64, device=DEV)
    h.spmv_dot(_dev(x), yd, _dev(w), out)
    y = _host(yd)
    ref_y = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x)
    mag = oracle.spmv_abs(A.row_ptr, A.col_idx, A.vals, x)
    assert_rows_close(y, ref_y, mag, TOL_F64)
    ref = oracle.dot(w, y)
    assert abs(_host(out)[0] - ref) <= TOL_F64 * oracle.dot_abs(w, y)
    h.destroy()


def _cg_case(A, iters, graph):
    b = gen.vector(A.rows, 7)
    x_or, done, hist = oracle.cg(A.row_ptr, A.col_idx, A.vals, b, iters)
    h = L.Csr.from_gen(A)
    bd = _dev(b)
    xd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    rho, it = h.cg(bd, xd, iters, graph=graph, want_result=True)
    x = _host(xd)
    h.destroy()
    return x, x_or, done, it, b


@pytest.mark.parametrize("graph", [False, True])
def test_cg_matches_oracle(graph):
    A = gen.spd_random(20000, 60, seed=11)
    x, x_or, done, it, b = _cg_case(A, 75, graph)
    assert it == done
    assert np.max(np.abs(x - x_or)) <= 1e-10 * np.max(np.abs(x_or))
    S_res = b - oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x)
    assert np.linalg.norm(S_res) <= 1e-10 * np.linalg.norm(b)


def test_cg_graph_equals_eager_bitwise_and_replays():
    A = gen.spd_random(30000, 40, seed=12)
    b = gen.vector(A.rows, 13)
    h = L.Csr.from_gen(A)
    bd = _dev(b)
    x1 = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    x2 = torch.empty_like(x1)
    h.cg(bd, x1, 30, graph=False)
    outs = []
    for _ in range(3):
        h.cg(bd, x2, 30, graph=True)
        torch.cuda.synchronize()
        outs.append(x2.clone())
        _ = torch.ones(1000, device=DEV).sum().item()  # eager work in between
    for o in outs:
        assert torch.equal(o, x1)
    h.destroy()


def test_cg_guards_zero_rhs_and_early_convergence():
    A = gen.spd_random(2000, 10, seed=14)
    h = L.Csr.from_gen(A)
    bd = torch.zeros(A.rows, dtype=torch.float64, device=DEV)
    xd = torch.full((A.rows,), 7.0, dtype=torch.float64, device=DEV)
    rho, it = h.cg(bd, xd, 10, want_result=True)
    assert it == 0 and torch.all(xd == 0)
    h.destroy()
    D = gen.diag_distinct(5000, 3, seed=15)
    b = gen.vector(D.rows, 16)
    x_or, done, _ = oracle.cg(D.row_ptr, D.col_idx, D.vals, b, 20)
    h = L.Csr.from_gen(D)
    xd = torch.empty(D.rows, dtype=torch.float64, device=DEV)
    rho, it = h.cg(_dev(b), xd, 20, want_result=True)
    x = _host(xd)
    assert np.max(np.abs(x - b / D.vals)) <= 1e-12 * np.max(np.abs(b / D.vals))
    assert np.max(np.abs(x - x_or)) <= 1e-12 * np.max(np.abs(x_or))
    h.destroy()


def test_cg_full_size_spd150k():
    A = gen.spd_random()
    x, x_or, done, it, b = _cg_case(A, 75, True)
    assert it == done == 75
    assert np.max(np.abs(x - x_or)) <= 1e-10 * np.max(np.abs(x_or))


def test_pagerank_step_and_run():
    A = gen.rmat_pagerank(16, 1 << 20, seed=20)
    n = A.rows
    d = float(np.float32(0.85))
    x0 = np.full(n, 1.0 / n, dtype=np.float32)
    h = L.Csr.from_gen(A)
    # one step: per-row tolerance
    xd = _dev(x0)
    h.pagerank(d, 1, xd)
    y1 = _host(xd)
    ref = oracle.pagerank_step(A.row_ptr, A.col_idx, A.vals, x0, d)
    mag = d * oracle.spmv_abs(A.row_ptr, A.col_idx, A.vals, x0) + (1 - d) / n
    assert_rows_close(y1, ref, mag, TOL_F32)
    # twenty steps: relative L1 against the float64 oracle run
    xd = _dev(x0)
    h.pagerank(d, 20, xd)
    x20 = _host(xd)
    ref20 = oracle.pagerank(A.row_ptr, A.col_idx, A.vals, x0.astype(np.float64), d, 20)
    assert np.sum(np.abs(x20 - ref20)) <= 20 * TOL_F32 * np.sum(np.abs(ref20))
    # graph replays are deterministic
    xd2 = _dev(x0)
    h.pagerank(d, 20, xd2)
    assert torch.equal(xd, xd2)
    h.destroy()


def test_pagerank_cycle_fixed_point():
    C = gen.cycle_graph(1000)
    h = L.Csr.from_gen(C)
    x = torch.full((1000,), 1e-3, dtype=torch.float32, device=DEV)
    h.pagerank(0.85, 20, x)
    assert np.allclose(_host(x), 1e-3, rtol=1e-6, atol=0)
    h.destroy()


def test_pagerank_after_value_update():
    """The relabelled copy PageRank iterates on follows new values."""
    A = gen.rmat_pagerank(16, 1 << 20, seed=21)
    n = A.rows
    d = float(np.float32(0.85))
    x0 = np.full(n, 1.0 / n, dtype=np.float32)
    h = L.Csr.from_gen(A)
    xd = _dev(x0)
    h.pagerank(d, 3, xd)
    vals2 = (A.vals * np.float32(0.5)).astype(np.float32)
    h.update_values(vals2)
    xd = _dev(x0)
    h.pagerank(d, 3, xd)
    ref = oracle.pagerank(A.row_ptr, A.col_idx, vals2, x0.astype(np.float64), d, 3)
    assert np.sum(np.abs(_host(xd) - ref)) <= 3 * TOL_F32 * np.sum(np.abs(ref))
    h.destroy()


def _pagerank_scales(A, d, x0, iters):
    """The oracle's iterates ref_1..ref_iters (binary64) and, per element, the
    scale that carries the per-step tolerance through the iteration:
        s_k = d |A| s_{k-1} + (d |A| |x_{k-1}| + (1-d)/N),   s_0 = 0,
    i.e. each step's own row scale plus the previous scale passed through
    the matrix once more; both terms go through |A| together:
        s_k = d |A| (s_{k-1} + |x_{k-1}|) + (1-d)/N.
    A float32 run whose every step is within 1e-5 of its row scale stays
    within 1e-5 s_k."""
    n = A.rows
    vals = A.vals.astype(np.float64)
    x = x0.astype(np.float64)
    s = np.zeros(n)
    for _ in range(iters):
        s = d * oracle.spmv_abs(A.row_ptr, A.col_idx, vals, s + np.abs(x)) + (1 - d) / n
        x = oracle.pagerank(A.row_ptr, A.col_idx, A.vals, x, d, 1)
    return x, s


def test_full_size_pagerank_rmat22():
    """PageRank on the full R-MAT 2^22 graph (the relabelled hot-column
    copy, whose persistent workgroups each take many row blocks): one step
    checked row by row, and 20 steps checked element by element against
    the float64 oracle run with the per-step tolerance carried through the
    iteration, beside the relative L1 bound."""
    A = gen.rmat_pagerank()
    n = A.rows
    d = float(np.float32(0.85))
    x0 = np.full(n, 1.0 / n, dtype=np.float32)
    h = L.Csr.from_gen(A)
    # one step, every row
    xd = _dev(x0)
    h.pagerank(d, 1, xd)
    y1 = _host(xd)
    ref1 = oracle.pagerank_step(A.row_ptr, A.col_idx, A.vals, x0, d)
    mag1 = d * oracle.spmv_abs(A.row_ptr, A.col_idx, A.vals, x0) + (1 - d) / n
    assert_rows_close(y1, ref1, mag1, TOL_F32, "rmat22 one step")
    # twenty steps
    xd = _dev(x0)
    h.pagerank(d, 20, xd)
    x20 = _host(xd)
    ref, scale = _pagerank_scales(A, d, x0, 20)
    assert_rows_close(x20, ref, scale, TOL_F32, "rmat22 twenty steps")
    assert np.sum(np.abs(x20 - ref)) <= 20 * TOL_F32 * np.sum(np.abs(ref))
    h.destroy()

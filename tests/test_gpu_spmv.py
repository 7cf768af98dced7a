"""GPU parity of the CSR analysis and product against the oracle, through the
C ABI (the paper-shaped raw call and the device-resident handle)."""
import json
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


def _matrices():
    return {
        "ragged_split": lambda: gen.ragged(3000, 40000, seed=1, max_len=300,
                                           long_rows=3, long_len=20000),
        "ragged_dup_unsorted": lambda: gen.ragged(2000, 700, seed=2, max_len=150,
                                                  dup=True, sort_cols=False,
                                                  long_rows=2, long_len=9000),
        "mostly_empty": lambda: gen.ragged(5000, 5000, seed=3, empty_frac=0.7),
        "one_long_row": lambda: gen.ragged(1, 200000, seed=4, long_rows=1,
                                           long_len=150000, empty_frac=0.0),
        "uniform16": lambda: gen.uniform_rows(4096, 16),
        "stencil7": lambda: gen.stencil(20, 7),
        "stencil27": lambda: gen.stencil(12, 27),
        "rmat16": lambda: gen.rmat_pagerank(16, 1 << 20, seed=5).astype(np.float64),
        "spd_small": lambda: gen.spd_random(20000, 60, seed=6),
        "random5_60": lambda: gen.random_rows(30000, 5, 60, seed=7),
        "all_empty": lambda: gen.empty_matrix(1000, 10),
    }


MATS = _matrices()


@pytest.mark.parametrize("name", sorted(MATS))
def test_analysis_bit_exact(name):
    A = MATS[name]()
    h = L.Csr.from_gen(A)
    up = h.upper()
    bor, off, br = oracle.bins(A.row_ptr, up)
    g_off, g_br, g_cr, g_c0, g_c1 = h.analysis()
    assert np.array_equal(g_off, off)
    assert np.array_equal(g_br, br)
    inf = h.info()
    cr, c0, c1 = oracle.split_chunks(A.row_ptr, int(up[7]), inf.chunk)
    assert np.array_equal(g_cr, cr) and np.array_equal(g_c0, c0) and \
        np.array_equal(g_c1, c1)
    assert h.cols == oracle.cols(A.col_idx) and h.nnz == A.nnz
    h.destroy()


@pytest.mark.parametrize("name", sorted(MATS))
def test_spmv_f64_handle(name):
    A = MATS[name]()
    x = gen.vector(max(A.cols, 1), 11)[:A.cols]
    h = L.Csr.from_gen(A)
    xd = _dev(x) if A.cols else torch.zeros(1, dtype=torch.float64, device=DEV)
    yd = torch.full((A.rows,), np.nan, dtype=torch.float64, device=DEV)
    h.spmv(xd, yd)
    check_spmv(A, x, _host(yd), TOL_F64)
    # deterministic: a second product is bitwise identical
    y2 = torch.empty_like(yd)
    h.spmv(xd, y2)
    assert torch.equal(yd, y2)
    h.destroy()


@pytest.mark.parametrize("name", ["ragged_split", "rmat16", "stencil27",
                                  "ragged_dup_unsorted"])
def test_spmv_f32_handle(name):
    A = MATS[name]().astype(np.float32)
    x = gen.vector(A.cols, 12, dtype=np.float32)
    h = L.Csr.from_gen(A)
    yd = torch.empty(A.rows, dtype=torch.float32, device=DEV)
    h.spmv(_dev(x), yd)
    check_spmv(A, x, _host(yd), TOL_F32)
    h.destroy()


@pytest.mark.parametrize("name", ["ragged_split", "random5_60", "stencil7",
                                  "one_long_row"])
def test_integer_inputs_bitwise(name):
    """Integer values and vector: every summation order gives the same exact
    integers, so every class of row must equal the oracle bitwise."""
    A = MATS[name]()
    A.vals = gen.int_vector(A.nnz, 13)
    x = gen.int_vector(A.cols, 14)
    h = L.Csr.from_gen(A)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    h.spmv(_dev(x), yd)
    assert np.array_equal(_host(yd), oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x))
    h.destroy()


def test_identity_and_permutation_bitwise():
    x = gen.vector(100_000, 15)
    for A, ref in ((gen.identity(100_000), x),
                   (gen.permutation(100_000, 16), None)):
        h = L.Csr.from_gen(A)
        yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
        h.spmv(_dev(x), yd)
        want = x if ref is not None else x[A.col_idx]
        assert np.array_equal(_host(yd), want)
        h.destroy()


def test_paper_example_raw_call(golden_dir):
    with open(os.path.join(golden_dir, "csr_5x5.json")) as f:
        g = json.load(f)
    rp = np.array(g["row_ptr"], np.int32)
    ci = np.array(g["col_ind"], np.int32)
    v = np.array(g["val"], np.float64)
    for xs, ys in ((g["x_ones"], g["y_ones"]), (g["x_ramp"], g["y_ramp"])):
        y = np.zeros(5)
        L.lilac_spmv_csr(5, rp, ci, v, np.array(xs, np.float64), y)
        assert list(y) == ys
        y32 = np.zeros(5, np.float32)
        L.lilac_spmv_csr_f32(5, rp, ci, v.astype(np.float32),
                             np.array(xs, np.float32), y32)
        assert list(y32) == ys
    L.lilac_release_all()


def test_raw_call_device_pointers_and_cache():
    A = gen.ragged(4000, 30000, seed=21, max_len=200, long_rows=2, long_len=12000)
    x = gen.vector(A.cols, 22)
    rp, ci, v, xd = _dev(A.row_ptr), _dev(A.col_idx), _dev(A.vals), _dev(x)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    L.lilac_spmv_csr(A.rows, rp, ci, v, xd, yd)
    check_spmv(A, x, _host(yd), TOL_F64)
    # host arrays, then change values and invalidate: the cached copy updates
    y = np.empty(A.rows)
    vals = A.vals.copy()
    L.lilac_spmv_csr(A.rows, A.row_ptr, A.col_idx, vals, x, y)
    check_spmv(A, x, y, TOL_F64)
    vals *= 2.0
    L.lilac_spmv_csr(A.rows, A.row_ptr, A.col_idx, vals, x, y)  # stale copy
    check_spmv(A, x, y, TOL_F64)
    L.lilac_invalidate(vals)
    L.lilac_spmv_csr(A.rows, A.row_ptr, A.col_idx, vals, x, y)
    A2 = gen.Csr(A.rows, A.cols, A.row_ptr, A.col_idx, vals, "x2")
    check_spmv(A2, x, y, TOL_F64)
    L.lilac_release_all()


def test_invalid_csr_rejected():
    A = gen.ragged(100, 50, seed=30, empty_frac=0.0)
    bad = A.row_ptr.copy()
    bad[0] = 1
    cases = [bad]
    mono = A.row_ptr.copy()
    mono[5] = mono[4] - 1
    cases.append(mono)
    for rp in cases:
        assert oracle.validate(rp, A.col_idx) != 0
        with pytest.raises(L.LilacError) as e:
            L.Csr(rp, A.col_idx, A.vals)
        assert e.value.code == -2
    ci = A.col_idx.copy()
    ci[7] = -3
    assert oracle.validate(A.row_ptr, ci) != 0
    with pytest.raises(L.LilacError) as e:
        L.Csr(A.row_ptr, ci, A.vals)
    assert e.value.code == -2
    with pytest.raises(L.LilacError) as e:
        L.Csr(A.row_ptr, A.col_idx, A.vals, cols=int(A.col_idx.max()))
    assert e.value.code == -2


def test_plan_changes_keep_results_in_tolerance():
    A = gen.ragged(6000, 60000, seed=31, max_len=600, long_rows=4, long_len=30000)
    x = gen.vector(A.cols, 32)
    h = L.Csr.from_gen(A)
    xd = _dev(x)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    for upper, chunk in (([1, 2, 4, 8, 16, 32, 256, 2048], 1024),
                         ([4, 8, 16, 32, 64, 128, 4096, 65536], 8192),
                         ([0, 0, 0, 0, 0, 0, 0, 0], 256)):
        h.set_plan(upper=upper, chunk=chunk)
        g_off, g_br, g_cr, g_c0, g_c1 = h.analysis()
        _, off, br = oracle.bins(A.row_ptr, np.array(upper + [2**31 - 1], np.int32))
        assert np.array_equal(g_off, off) and np.array_equal(g_br, br)
        h.spmv(xd, yd)
        check_spmv(A, x, _host(yd), TOL_F64)
    h.destroy()


def test_full_size_uniform16_and_spd150k():
    """The single-product workloads at full size, every row checked."""
    A = gen.uniform_rows()
    x = gen.vector(A.cols, 41)
    h = L.Csr.from_gen(A)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    h.spmv(_dev(x), yd)
    check_spmv(A, x, _host(yd), TOL_F64)
    h.destroy()
    A = gen.spd_random()
    x = gen.vector(A.cols, 42)
    h = L.Csr.from_gen(A)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    h.spmv(_dev(x), yd)
    check_spmv(A, x, _host(yd), TOL_F64)
    h.destroy()


def test_full_size_rmat22_f32():
    A = gen.rmat_pagerank()
    x = gen.vector(A.cols, 43, dtype=np.float32, lo=0.0, hi=1.0)
    h = L.Csr.from_gen(A)
    yd = torch.empty(A.rows, dtype=torch.float32, device=DEV)
    h.spmv(_dev(x), yd)
    check_spmv(A, x, _host(yd), TOL_F32)
    inf = h.info()
    assert inf.nchunks > 0  # the hubs take the split path
    h.destroy()


def test_dot_raw_and_device():
    for n in (0, 1, 1000, 150_000, 3_000_001):
        a = gen.vector(n, 50)
        b = gen.vector(n, 51)
        ref = oracle.dot(a, b)
        mag = oracle.dot_abs(a, b)
        got = L.lilac_dot(n, a, b)
        assert abs(got - ref) <= TOL_F64 * mag
        if n:
            ad, bd = _dev(a), _dev(b)
            out = torch.empty(1, dtype=torch.float64, device=DEV)
            L.lilac_dot_dev(n, ad, bd, out)
            assert _host(out)[0] == L.lilac_dot(n, ad, bd)
            L.lilac_dot_dev(n, ad, bd, out, dtype=L.F64)
            assert _host(out)[0] == L.lilac_dot(n, ad, bd)
    assert L.lilac_dot(1 << 20, np.ones(1 << 20), np.ones(1 << 20)) == float(1 << 20)


def test_dot_f32_raw_host_and_device():
    """float32 arrays: products and sums in binary64, one final rounding."""
    for n in (0, 1, 1000, 150_000, 3_000_001):
        a = gen.vector(n, 52, dtype=np.float32)
        b = gen.vector(n, 53, dtype=np.float32)
        ref = oracle.dot(a.astype(np.float64), b.astype(np.float64))
        mag = oracle.dot_abs(a.astype(np.float64), b.astype(np.float64))
        got = L.lilac_dot_f32(n, a, b)
        assert abs(got - ref) <= TOL_F32 * (mag + abs(ref))
        if n:
            assert L.lilac_dot_f32(n, _dev(a), _dev(b)) == got
        # the device-resident form: float32 result, same single rounding
        out = torch.full((1,), 7.0, dtype=torch.float32, device=DEV)
        L.lilac_dot_dev(n, _dev(a) if n else None, _dev(b) if n else None, out)
        assert _host(out)[0] == np.float32(got)
        assert abs(float(_host(out)[0]) - ref) <= TOL_F32 * (mag + abs(ref))
    ones = np.ones(1 << 20, dtype=np.float32)
    assert L.lilac_dot_f32(1 << 20, ones, ones) == float(1 << 20)


PANEL_MATS = {
    "spd20k": lambda: gen.spd_random(20000, 60, seed=6),
    "uniform16": lambda: gen.uniform_rows(4096, 16),
    "ragged_dense_rows": lambda: gen.ragged(3000, 9000, seed=8, max_len=1000,
                                            empty_frac=0.05, sort_cols=False),
    "wide_tail_panel": lambda: gen.random_rows(5000, 150, 300, seed=9, cols=20000),
}


@pytest.mark.parametrize("name", sorted(PANEL_MATS))
def test_panel_layout_parity(name):
    A = PANEL_MATS[name]()
    x = gen.vector(A.cols, 60)
    h = L.Csr.from_gen(A, cols=A.cols)
    xd = _dev(x)
    ys = {}
    for lay in (L.LAYOUT_PANELS, L.LAYOUT_ROWS):
        h.set_layout(lay)
        inf = h.info()
        assert inf.layout == lay, (name, lay)
        yd = torch.full((A.rows,), np.nan, dtype=torch.float64, device=DEV)
        h.spmv(xd, yd)
        ys[lay] = _host(yd)
        check_spmv(A, x, ys[lay], TOL_F64)
    # integer data: both layouts exact
    A.vals = gen.int_vector(A.nnz, 61)
    xi = gen.int_vector(A.cols, 62)
    h2 = L.Csr.from_gen(A, cols=A.cols)
    h2.set_layout(L.LAYOUT_PANELS)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    h2.spmv(_dev(xi), yd)
    assert np.array_equal(_host(yd), oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, xi))
    h.destroy()
    h2.destroy()


def test_panel_layout_f32_and_fused_dot():
    A = gen.spd_random(40000, 60, seed=6)
    h = L.Csr.from_gen(A)
    assert h.info().layout == L.LAYOUT_PANELS  # chosen automatically
    x = gen.vector(A.cols, 63)
    w = gen.vector(A.rows, 64)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    out = torch.empty(1, dtype=torch.float64, device=DEV)
    h.spmv_dot(_dev(x), yd, _dev(w), out)
    y = _host(yd)
    check_spmv(A, x, y, TOL_F64)
    assert abs(_host(out)[0] - oracle.dot(w, y)) <= TOL_F64 * oracle.dot_abs(w, y)
    h.destroy()
    B = A.astype(np.float32)
    h = L.Csr.from_gen(B)
    h.set_layout(L.LAYOUT_PANELS)
    x32 = gen.vector(B.cols, 65, dtype=np.float32)
    yd = torch.empty(B.rows, dtype=torch.float32, device=DEV)
    h.spmv(_dev(x32), yd)
    check_spmv(B, x32, _host(yd), TOL_F32)
    h.destroy()


def test_panel_layout_tall_row_blocks():
    """Short scattered rows over many columns: row blocks of 4096 rows (the
    row sums take 32 KiB of LDS, panels of 16384 float64 columns, several
    rows per thread in the epilogue and the fused dot), with a partial last
    block."""
    A = gen.random_rows(120000, 3, 9, seed=13)
    h = L.Csr.from_gen(A)
    inf = h.info()
    assert inf.layout == L.LAYOUT_PANELS  # chosen automatically
    assert inf.npanels == 8               # 16384-column panels
    x = gen.vector(A.cols, 67)
    w = gen.vector(A.rows, 68)
    yd = torch.full((A.rows,), np.nan, dtype=torch.float64, device=DEV)
    out = torch.empty(1, dtype=torch.float64, device=DEV)
    h.spmv_dot(_dev(x), yd, _dev(w), out)
    y = _host(yd)
    check_spmv(A, x, y, TOL_F64)
    assert abs(_host(out)[0] - oracle.dot(w, y)) <= TOL_F64 * oracle.dot_abs(w, y)
    yd2 = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    h.spmv(_dev(x), yd2)
    assert np.array_equal(_host(yd2), y)
    h.destroy()
    A.vals = gen.int_vector(A.nnz, 69)
    xi = gen.int_vector(A.cols, 70)
    h = L.Csr.from_gen(A)
    assert h.info().layout == L.LAYOUT_PANELS
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    h.spmv(_dev(xi), yd)
    assert np.array_equal(_host(yd), oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, xi))
    h.destroy()
    B = gen.random_rows(120000, 3, 9, seed=13, dtype=np.float32)
    h = L.Csr.from_gen(B)
    inf = h.info()
    assert inf.layout == L.LAYOUT_PANELS and inf.npanels == 4  # 32768 float32 columns
    x32 = gen.vector(B.cols, 71, dtype=np.float32)
    yd = torch.empty(B.rows, dtype=torch.float32, device=DEV)
    h.spmv(_dev(x32), yd)
    check_spmv(B, x32, _host(yd), TOL_F32)
    h.destroy()


def test_panel_layout_rotated_order_many_panels():
    """Over 128 row blocks and 16 panels: each block takes the panels in a
    rotated order (blocks of one XCD start at different panels, most of
    them past the eighth), alone and in a grouped launch, with the same
    result."""
    A = gen.random_rows(110000, 200, 280, seed=23, cols=300000)
    h = L.Csr.from_gen(A)
    h.set_layout(L.LAYOUT_PANELS)
    inf = h.info()
    assert inf.layout == L.LAYOUT_PANELS and inf.npanels >= 16, inf.npanels
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    rb = max(-(-A.rows // cu), int(np.ceil(A.cols * 8 / (A.nnz / A.rows * 12))))
    assert cu != 256 or -(-A.rows // rb) >= 128
    x = gen.vector(A.cols, 72)
    xd = _dev(x)
    yd = torch.full((A.rows,), np.nan, dtype=torch.float64, device=DEV)
    h.spmv(xd, yd)
    y = _host(yd)
    check_spmv(A, x, y, TOL_F64)
    B = gen.spd_random(20000, 40, seed=24)
    hb = L.Csr.from_gen(B)
    xb = _dev(gen.vector(B.cols, 73))
    ys = [torch.empty(A.rows, dtype=torch.float64, device=DEV),
          torch.empty(B.rows, dtype=torch.float64, device=DEV)]
    L.lilac_spmv_batched([h, hb], [xd, xb], ys)
    assert np.array_equal(_host(ys[0]), y)
    h.destroy()
    hb.destroy()


def test_panel_layout_unaligned_x():
    """x starting 8 bytes past a 16-byte boundary takes the scalar staging
    path of the panel kernel."""
    A = gen.spd_random(40000, 60, seed=6)
    h = L.Csr.from_gen(A)
    x = gen.vector(A.cols, 66)
    buf = torch.empty(A.cols + 1, dtype=torch.float64, device=DEV)
    buf[1:] = torch.from_numpy(x).to(DEV)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    h.spmv(buf[1:], yd)
    check_spmv(A, x, _host(yd), TOL_F64)
    h.destroy()


HOT_MATS = {
    "ragged_long_rows": lambda: gen.ragged(3000, 40000, seed=1, max_len=300,
                                           long_rows=3, long_len=20000),
    "mostly_empty_all_hot": lambda: gen.ragged(5000, 5000, seed=3, empty_frac=0.7),
    "one_long_row": lambda: gen.ragged(1, 200000, seed=4, long_rows=1,
                                       long_len=150000, empty_frac=0.0),
    "rmat16": lambda: gen.rmat_pagerank(16, 1 << 20, seed=5).astype(np.float64),
    "random5_60": lambda: gen.random_rows(30000, 5, 60, seed=7),
    "stencil27": lambda: gen.stencil(12, 27),
    "cols_2p22": lambda: gen.random_rows(5000, 1, 20, seed=10, cols=1 << 22),
    "cols_one": lambda: gen.random_rows(3000, 1, 1, seed=11, cols=1),
    # 2^20 rows cut into blocks of at most 1536 non-empty rows: 522 blocks,
    # so the workgroups of the persistent grid (one per CU) take two or more
    # on average and run the code that moves from one block to the next
    "rmat20_by_degree": lambda: gen.relabel_by_degree(
        gen.rmat_pagerank(20, 1 << 24, seed=14)).astype(np.float64),
    # 97% empty rows: blocks end at 24576 rows (16 x 1536) long before they
    # hold 1536 non-empty ones, and most rows of a block take no row sum
    "mostly_empty_span": lambda: gen.ragged(80000, 80000, seed=15, empty_frac=0.97),
}


@pytest.mark.parametrize("name", sorted(HOT_MATS))
def test_hot_layout_parity(name):
    """Hot-column layout (columns below the LDS width staged, the rest
    gathered): float64 and float32 within tolerance, integer data exact,
    repeated calls bitwise equal."""
    A = HOT_MATS[name]()
    x = gen.vector(A.cols, 70)
    h = L.Csr.from_gen(A, cols=A.cols)
    h.set_layout(L.LAYOUT_HOT)
    assert h.info().layout == L.LAYOUT_HOT, name
    xd = _dev(x)
    yd = torch.full((A.rows,), np.nan, dtype=torch.float64, device=DEV)
    h.spmv(xd, yd)
    y = _host(yd)
    check_spmv(A, x, y, TOL_F64)
    h.spmv(xd, yd)
    assert np.array_equal(_host(yd), y)
    h.destroy()
    B = A.astype(np.float32)
    x32 = gen.vector(B.cols, 71, dtype=np.float32)
    h = L.Csr.from_gen(B, cols=B.cols)
    h.set_layout(L.LAYOUT_HOT)
    yd = torch.empty(B.rows, dtype=torch.float32, device=DEV)
    h.spmv(_dev(x32), yd)
    y32 = _host(yd)
    check_spmv(B, x32, y32, TOL_F32)
    h.spmv(_dev(x32), yd)
    assert np.array_equal(_host(yd), y32)
    h.destroy()
    # float32 integer data: every partial sum is an integer below 2^24, so
    # the product is exact whatever the order of the additions
    B.vals = gen.int_vector(B.nnz, 74).astype(np.float32)
    xi32 = gen.int_vector(B.cols, 75).astype(np.float32)
    h = L.Csr.from_gen(B, cols=B.cols)
    h.set_layout(L.LAYOUT_HOT)
    h.spmv(_dev(xi32), yd)
    want = oracle.spmv_csr(B.row_ptr, B.col_idx, B.vals.astype(np.float64),
                           xi32.astype(np.float64))
    assert np.max(np.abs(want)) < 2 ** 24
    assert np.array_equal(_host(yd).astype(np.float64), want)
    h.destroy()
    A.vals = gen.int_vector(A.nnz, 72)
    xi = gen.int_vector(A.cols, 73)
    h = L.Csr.from_gen(A, cols=A.cols)
    h.set_layout(L.LAYOUT_HOT)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    h.spmv(_dev(xi), yd)
    assert np.array_equal(_host(yd), oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, xi))
    h.destroy()


def test_hot_layout_fused_dot_unaligned_x_and_fallback():
    A = gen.ragged(20000, 60000, seed=12, max_len=200, long_rows=4, long_len=30000)
    h = L.Csr.from_gen(A, cols=A.cols)
    h.set_layout(L.LAYOUT_HOT)
    x = gen.vector(A.cols, 74)
    w = gen.vector(A.rows, 75)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    out = torch.empty(1, dtype=torch.float64, device=DEV)
    h.spmv_dot(_dev(x), yd, _dev(w), out)
    y = _host(yd)
    check_spmv(A, x, y, TOL_F64)
    assert abs(_host(out)[0] - oracle.dot(w, y)) <= TOL_F64 * oracle.dot_abs(w, y)
    # x 8 bytes past a 16-byte boundary: scalar staging of the hot columns
    buf = torch.empty(A.cols + 1, dtype=torch.float64, device=DEV)
    buf[1:] = _dev(x)
    yd2 = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    h.spmv(buf[1:], yd2)
    assert np.array_equal(_host(yd2), y)
    h.destroy()
    # no entries: the layout is not built, the product still overwrites y
    E = gen.empty_matrix(1000, 10)
    he = L.Csr.from_gen(E, cols=E.cols)
    he.set_layout(L.LAYOUT_HOT)
    assert he.info().layout == L.LAYOUT_ROWS
    yd = torch.full((1000,), np.nan, dtype=torch.float64, device=DEV)
    he.spmv(_dev(np.ones(10)), yd)
    assert np.array_equal(_host(yd), np.zeros(1000))
    he.destroy()


def test_value_updates_reach_panel_and_hot_copies():
    """The column-panel and hot-column copies hold the values too (the band
    layout reads the CSR values): new values must reach every layout, and
    the CG graph built on the old copy must not be replayed."""
    A = gen.spd_random(40000, 60, seed=6)
    x = gen.vector(A.cols, 80)
    b = gen.vector(A.rows, 81)
    bd = _dev(b)  # same right-hand side and solution arrays: same graph key
    for lay in (L.LAYOUT_PANELS, L.LAYOUT_HOT, L.LAYOUT_BAND, L.LAYOUT_ROWS):
        h = L.Csr.from_gen(A)
        h.set_layout(lay)
        assert h.info().layout == lay
        yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
        xd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
        h.spmv(_dev(x), yd)
        check_spmv(A, x, _host(yd), TOL_F64)
        h.cg(bd, xd, 20, graph=True)
        B = gen.Csr(A.rows, A.cols, A.row_ptr, A.col_idx, A.vals * 0.5, "scaled")
        h.update_values(B.vals)
        assert h.info().layout == lay
        h.spmv(_dev(x), yd)
        check_spmv(B, x, _host(yd), TOL_F64)
        h.cg(bd, xd, 20, graph=True)
        x_or, _, _ = oracle.cg(B.row_ptr, B.col_idx, B.vals, b, 20)
        assert np.max(np.abs(_host(xd) - x_or)) <= 1e-10 * np.max(np.abs(x_or))
        h.destroy()


def _band_edges(n, offset):
    """Rows i with columns i and i + offset (clipped): every row spans
    `offset` columns, so blocks are cut by span, not only by rows."""
    rows = np.repeat(np.arange(n), 2)
    cols = np.stack([np.arange(n), np.minimum(np.arange(n) + offset, n - 1)], 1).ravel()
    cols = np.where(np.arange(2 * n) % 2 == 1, np.maximum(cols, rows), cols)
    keep = np.ones(2 * n, dtype=bool)
    keep[1::2] = cols[1::2] != cols[0::2]
    rows, cols = rows[keep], cols[keep]
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    vals = gen.vector(len(cols), 90)
    return gen.Csr(n, n, rp, cols.astype(np.int32), vals, f"band{offset}")


BAND_MATS = {
    "stencil7": lambda: gen.stencil(20, 7),
    "stencil27": lambda: gen.stencil(14, 27),
    "uniform16": lambda: gen.uniform_rows(4096, 16),
    "ragged_long_rows": lambda: gen.ragged(3000, 40000, seed=1, max_len=300,
                                           long_rows=3, long_len=20000),
    "mostly_empty": lambda: gen.ragged(5000, 5000, seed=3, empty_frac=0.7),
    "span_30000": lambda: _band_edges(120000, 30000),
    "span_65000": lambda: _band_edges(120000, 65000),
}


@pytest.mark.parametrize("name", sorted(BAND_MATS))
def test_band_layout_parity(name):
    """Band layout (CSR order, packed row and column offset): float64 and
    float32 within tolerance, integer data exact, repeated calls equal."""
    A = BAND_MATS[name]()
    x = gen.vector(A.cols, 91)
    h = L.Csr.from_gen(A, cols=A.cols)
    h.set_layout(L.LAYOUT_BAND)
    assert h.info().layout == L.LAYOUT_BAND, name
    xd = _dev(x)
    yd = torch.full((A.rows,), np.nan, dtype=torch.float64, device=DEV)
    h.spmv(xd, yd)
    y = _host(yd)
    check_spmv(A, x, y, TOL_F64)
    h.spmv(xd, yd)
    assert np.array_equal(_host(yd), y)
    h.destroy()
    B = A.astype(np.float32)
    x32 = gen.vector(B.cols, 92, dtype=np.float32)
    h = L.Csr.from_gen(B, cols=B.cols)
    h.set_layout(L.LAYOUT_BAND)
    yd = torch.empty(B.rows, dtype=torch.float32, device=DEV)
    h.spmv(_dev(x32), yd)
    check_spmv(B, x32, _host(yd), TOL_F32)
    h.destroy()
    A.vals = gen.int_vector(A.nnz, 93)
    xi = gen.int_vector(A.cols, 94)
    h = L.Csr.from_gen(A, cols=A.cols)
    h.set_layout(L.LAYOUT_BAND)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    h.spmv(_dev(xi), yd)
    assert np.array_equal(_host(yd), oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, xi))
    h.destroy()


def test_layout_choice_and_band_fallback():
    """The automatic choice: scattered columns -> column panels, local
    columns -> band, tiny -> rows, and rows of consecutive columns at
    scattered offsets (local within a row, not between rows: band blocks
    of one row each) -> rows; a row spanning 65536 columns or more makes
    the band impossible (rows layout instead)."""
    win = gen.strided_rows(100000, 16, 1 << 21, seed=4, dtype=np.float64, window=True)
    win = gen.Csr(win.rows, win.cols, win.row_ptr.astype(np.int32), win.col_idx,
                  win.vals, "window16")
    cases = [(gen.spd_random(40000, 60, seed=6), L.LAYOUT_PANELS),
             (gen.stencil(30, 27), L.LAYOUT_BAND),
             (gen.stencil(30, 7), L.LAYOUT_BAND),
             (gen.random_rows(2000, 1, 4, seed=3), L.LAYOUT_ROWS),
             (win, L.LAYOUT_ROWS)]
    for A, want in cases:
        h = L.Csr.from_gen(A)
        assert h.info().layout == want, (A.name, h.info().layout)
        x = gen.vector(A.cols, 95)
        yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
        h.spmv(_dev(x), yd)
        check_spmv(A, x, _host(yd), TOL_F64)
        h.destroy()
    W = _band_edges(100000, 70000)
    h = L.Csr.from_gen(W)
    h.set_layout(L.LAYOUT_BAND)
    assert h.info().layout == L.LAYOUT_ROWS
    x = gen.vector(W.cols, 96)
    yd = torch.empty(W.rows, dtype=torch.float64, device=DEV)
    h.spmv(_dev(x), yd)
    check_spmv(W, x, _host(yd), TOL_F64)
    h.destroy()


def test_band_fused_dot_and_cg():
    A = gen.stencil(40, 7)
    h = L.Csr.from_gen(A)
    assert h.info().layout == L.LAYOUT_BAND
    x = gen.vector(A.cols, 97)
    w = gen.vector(A.rows, 98)
    yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    out = torch.empty(1, dtype=torch.float64, device=DEV)
    h.spmv_dot(_dev(x), yd, _dev(w), out)
    y = _host(yd)
    check_spmv(A, x, y, TOL_F64)
    assert abs(_host(out)[0] - oracle.dot(w, y)) <= TOL_F64 * oracle.dot_abs(w, y)
    b = gen.vector(A.rows, 99)
    xd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    h.cg(_dev(b), xd, 40, graph=True)
    x_or, _, _ = oracle.cg(A.row_ptr, A.col_idx, A.vals, b, 40)
    assert np.max(np.abs(_host(xd) - x_or)) <= 1e-10 * np.max(np.abs(x_or))
    h.destroy()

"""Grouped batched products and the autotuner on the GPU: every matrix of a
batch must equal its own single-call result bitwise, and the oracle within
tolerance."""
import numpy as np
import pytest
import torch

import gen
import paper_2001_07938_amd as L
from tests.helpers import TOL_F32, TOL_F64, check_spmv

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _batch(count, seed, dtype=np.float64, n_hi=20000):
    specs = gen.batch_specs(count, n_lo=200, n_hi=n_hi, seed=seed)
    mats = [s.build().astype(dtype) for s in specs]
    # a few matrices with split rows and empty rows
    mats.append(gen.ragged(3000, 30000, seed=seed + 1, long_rows=2,
                           long_len=20000).astype(dtype))
    mats.append(gen.empty_matrix(10, 5).astype(dtype))
    return mats


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batched_equals_single_bitwise(dtype):
    mats = _batch(40, 5, dtype)
    hs = [L.Csr.from_gen(A) for A in mats]
    xs_h = [gen.vector(max(A.cols, 1), 100 + i, dtype=dtype) for i, A in enumerate(mats)]
    xs = [_dev(x) for x in xs_h]
    ys = [torch.empty(max(A.rows, 1), dtype=hs[0].torch_dtype, device=DEV) for A in mats]
    ys1 = [torch.empty_like(y) for y in ys]
    for h, x, y in zip(hs, xs, ys1):
        h.spmv(x, y)
    for rep in range(2):
        L.lilac_spmv_batched(hs, xs, ys)
        torch.cuda.synchronize()
        for A, y, y1 in zip(mats, ys, ys1):
            assert torch.equal(y[:A.rows], y1[:A.rows]), A.name
    tol = TOL_F64 if dtype == np.float64 else TOL_F32
    for A, x, y in zip(mats, xs_h, ys):
        check_spmv(A, x[:A.cols], y[:A.rows].cpu().numpy(), tol)
    for h in hs:
        h.destroy()


def test_batched_same_matrix_twice_with_split_rows():
    A = gen.ragged(2000, 40000, seed=9, long_rows=3, long_len=25000)
    h = L.Csr.from_gen(A)
    x1, x2 = gen.vector(A.cols, 1), gen.vector(A.cols, 2)
    y1 = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    y2 = torch.empty_like(y1)
    L.lilac_spmv_batched([h, h], [_dev(x1), _dev(x2)], [y1, y2])
    torch.cuda.synchronize()
    check_spmv(A, x1, y1.cpu().numpy(), TOL_F64)
    check_spmv(A, x2, y2.cpu().numpy(), TOL_F64)
    h.destroy()


def test_mixed_dtypes_rejected():
    a = L.Csr.from_gen(gen.stencil(5, 7))
    b = L.Csr.from_gen(gen.stencil(5, 7).astype(np.float32))
    x = torch.zeros(125, dtype=torch.float64, device=DEV)
    with pytest.raises(L.LilacError):
        L.lilac_spmv_batched([a, b], [x, x], [x, x])
    a.destroy()
    b.destroy()


def test_tuner_keeps_results_in_tolerance():
    A = gen.random_rows(50000, 5, 60, seed=3)
    x = gen.vector(A.cols, 4)
    h = L.Csr.from_gen(A)
    try:
        us = h.tune()
        assert us > 0
        y = torch.empty(A.rows, dtype=torch.float64, device=DEV)
        h.spmv(_dev(x), y)
        torch.cuda.synchronize()
        check_spmv(A, x, y.cpu().numpy(), TOL_F64)
    finally:
        h.destroy()
        L.lilac_tune_clear()   # later tests expect the default plans


def test_batched_with_panel_matrices_bitwise():
    """The column-panel matrix has two panels and, on a 256-CU device, 181
    row blocks of 221 rows (enough rows to be worth a copy of x), so its
    blocks take the panels in a rotated order, in the grouped launch as in
    its own."""
    mats = [gen.spd_random(40000, 60, seed=21), gen.stencil(12, 7),
            gen.uniform_rows(4096, 16), gen.random_rows(8000, 5, 60, seed=22)]
    hs = [L.Csr.from_gen(A) for A in mats]
    assert hs[0].info().layout == L.LAYOUT_PANELS
    assert hs[0].info().npanels >= 2
    A0 = mats[0]
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    rb = max(-(-A0.rows // cu), int(np.ceil(A0.cols * 8 / (A0.nnz / A0.rows * 12))))
    assert cu != 256 or -(-A0.rows // rb) >= 128
    assert hs[1].info().layout == L.LAYOUT_ROWS
    xs = [_dev(gen.vector(A.cols, 30 + i)) for i, A in enumerate(mats)]
    ys = [torch.empty(A.rows, dtype=torch.float64, device=DEV) for A in mats]
    ys1 = [torch.empty_like(y) for y in ys]
    for h, x, y in zip(hs, xs, ys1):
        h.spmv(x, y)
    L.lilac_spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    for y, y1 in zip(ys, ys1):
        assert torch.equal(y, y1)
    for h in hs:
        h.destroy()


def test_batched_mixed_layouts_bitwise():
    """A batch holding column-panel, band, hot-column and rows matrices: one
    grouped launch per layout, each result equal to its single call."""
    mats = [gen.spd_random(40000, 60, seed=6), gen.stencil(30, 27),
            gen.stencil(25, 7), gen.random_rows(2000, 1, 4, seed=3),
            gen.rmat_pagerank(16, 1 << 20, seed=5).astype(np.float64)]
    hs = [L.Csr.from_gen(A) for A in mats]
    hs[-1].set_layout(L.LAYOUT_HOT)
    lays = [h.info().layout for h in hs]
    assert lays == [L.LAYOUT_PANELS, L.LAYOUT_BAND, L.LAYOUT_BAND, L.LAYOUT_ROWS,
                    L.LAYOUT_HOT], lays
    xs = [_dev(gen.vector(A.cols, 200 + i)) for i, A in enumerate(mats)]
    ys = [torch.empty(A.rows, dtype=torch.float64, device=DEV) for A in mats]
    ys1 = [torch.empty_like(y) for y in ys]
    for h, x, y in zip(hs, xs, ys1):
        h.spmv(x, y)
    L.lilac_spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    for A, x, y, y1 in zip(mats, xs, ys, ys1):
        assert torch.equal(y, y1), A.name
        check_spmv(A, x.cpu().numpy(), y.cpu().numpy(), TOL_F64)
    for h in hs:
        h.destroy()


def test_full_size_batched512():
    """The batched workload at full size (512 matrices, 430M non-zeros) in
    the launch the benchmark times: every row against the oracle, every
    matrix bitwise equal to its single call."""
    mats = [s.build() for s in gen.batch_specs()]
    hs = [L.Csr.from_gen(A) for A in mats]
    xs_h = [gen.vector(A.cols, 1000 + i) for i, A in enumerate(mats)]
    xs = [_dev(x) for x in xs_h]
    ys = [torch.empty(A.rows, dtype=torch.float64, device=DEV) for A in mats]
    L.lilac_spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    y1 = torch.empty(max(A.rows for A in mats), dtype=torch.float64, device=DEV)
    for h, A, x, xh, y in zip(hs, mats, xs, xs_h, ys):
        h.spmv(x, y1[:A.rows])
        torch.cuda.synchronize()
        assert torch.equal(y, y1[:A.rows]), A.name
        check_spmv(A, xh, y.cpu().numpy(), TOL_F64)
    for h in hs:
        h.destroy()


def test_batch_tuner_results_and_cache():
    """The batch autotuner changes layouts only; every matrix still equals
    its single call bitwise and the oracle within tolerance, and handles
    created afterwards start from the tuned plan of their class."""
    try:
        _batch_tuner_checks()
    finally:
        L.lilac_tune_clear()   # later tests expect the default plans
    # after clearing, a fresh handle starts from the default plan again
    A = gen.stencil(30, 27)
    h = L.Csr.from_gen(A)
    assert h.info().layout == L.LAYOUT_BAND
    h.destroy()


def _batch_tuner_checks():
    mats = _batch(60, 17, n_hi=60000)
    hs = [L.Csr.from_gen(A) for A in mats]
    xs_h = [gen.vector(max(A.cols, 1), 300 + i) for i, A in enumerate(mats)]
    xs = [_dev(x) for x in xs_h]
    ys = [torch.empty(max(A.rows, 1), dtype=torch.float64, device=DEV) for A in mats]
    ms = L.lilac_spmv_batched_tune(hs, xs, ys)
    assert ms > 0
    lay = [h.info().layout for h in hs]
    L.lilac_spmv_batched(hs, xs, ys)
    torch.cuda.synchronize()
    for i, (h, A, x, y) in enumerate(zip(hs, mats, xs, ys)):
        y1 = torch.empty_like(y)
        h.spmv(x, y1)
        torch.cuda.synchronize()
        assert torch.equal(y, y1)
        if A.rows:
            check_spmv(A, xs_h[i], y.cpu().numpy()[:A.rows], TOL_F64)
    # a fresh handle of each matrix gets its class's tuned plan
    for A, h, l0 in zip(mats, hs, lay):
        h2 = L.Csr.from_gen(A)
        assert h2.tune_class() == h.tune_class()
        assert h2.info().layout == l0, (A.name, h.tune_class())
        h2.destroy()
    for h in hs:
        h.destroy()

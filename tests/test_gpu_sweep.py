"""A seeded sweep of small matrices of assorted shapes through every storage
layout of the product, against the oracle: row lengths from empty to a few
thousand, scattered and local columns, sorted and unsorted, duplicates,
float64 and float32, x aligned and 8 bytes off a 16-byte boundary, and the
product with the fused dot (float64)."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2001_07938_amd as L
from tests.helpers import TOL_F32, TOL_F64, check_spmv

pytestmark = pytest.mark.gpu

DEV = "cuda"
LAYOUTS = (L.LAYOUT_ROWS, L.LAYOUT_PANELS, L.LAYOUT_BAND, L.LAYOUT_HOT, -1)


def _case(i):
    """Matrix i of the sweep (seeded by i)."""
    rng = np.random.default_rng(gen.BASE_SEED + 500 + i)
    kind = i % 4
    rows = int(rng.integers(1, 30000))
    if kind == 0:    # ragged lengths, scattered columns
        cols = int(rng.integers(1, 200000))
        return gen.ragged(rows, cols, seed=1000 + i, max_len=int(rng.integers(1, 400)),
                          long_rows=int(rng.integers(0, 3)),
                          long_len=int(rng.integers(1000, 20000)),
                          empty_frac=float(rng.uniform(0, 0.5)),
                          dup=bool(rng.integers(0, 2)),
                          sort_cols=bool(rng.integers(0, 2)))
    if kind == 1:    # uniform random rows
        cols = int(rng.integers(64, 120000))
        lo = int(rng.integers(1, 40))
        return gen.random_rows(rows, lo, lo + int(rng.integers(0, 80)), seed=1000 + i,
                               cols=cols)
    if kind == 2:    # consecutive columns at scattered or banded offsets
        cols = int(rng.integers(600, 300000))
        k = int(rng.integers(1, min(600, cols)))
        A = gen.strided_rows(rows, k, cols, seed=1000 + i, dtype=np.float64,
                             window=bool(rng.integers(0, 2)))
        return gen.Csr(A.rows, A.cols, A.row_ptr.astype(np.int32), A.col_idx,
                       A.vals, f"strided{i}")
    n = int(rng.integers(4, 26))  # stencils
    return gen.stencil(n, 7 if rng.integers(0, 2) else 27)


@pytest.mark.parametrize("i", range(96))
def test_sweep_all_layouts(i):
    A = _case(i)
    rng = np.random.default_rng(gen.BASE_SEED + 900 + i)
    for dt, tol in ((np.float64, TOL_F64), (np.float32, TOL_F32)):
        B = A.astype(dt)
        x = gen.vector(B.cols, 2000 + i, dtype=dt)
        h = L.Csr.from_gen(B, cols=B.cols)
        tdt = torch.float64 if dt == np.float64 else torch.float32
        # x at an aligned address, or 8 bytes past one (float64: odd element)
        off = int(rng.integers(0, 2)) * (2 if dt == np.float32 else 1)
        buf = torch.empty(B.cols + off, dtype=tdt, device=DEV)
        buf[off:] = torch.from_numpy(x).to(DEV)
        xd = buf[off:]
        w = gen.vector(B.rows, 5000 + i)
        wd = torch.from_numpy(w).to(DEV)
        for lay in LAYOUTS:
            h.set_layout(lay)
            yd = torch.full((B.rows,), float("nan"), dtype=tdt, device=DEV)
            h.spmv(xd, yd)
            torch.cuda.synchronize()
            y = yd.cpu().numpy()
            check_spmv(B, x, y, tol)
            if dt == np.float64:
                # the product with the fused dot: the same y, and w . y
                y2 = torch.empty_like(yd)
                out = torch.empty(1, dtype=torch.float64, device=DEV)
                h.spmv_dot(xd, y2, wd, out)
                torch.cuda.synchronize()
                assert np.array_equal(y2.cpu().numpy(), y), (i, lay)
                assert abs(out.item() - oracle.dot(w, y)) <= TOL_F64 * oracle.dot_abs(w, y)
        h.destroy()
    # integer data: every layout exact
    A.vals = gen.int_vector(A.nnz, 3000 + i)
    xi = gen.int_vector(A.cols, 4000 + i)
    ref = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, xi)
    h = L.Csr.from_gen(A, cols=A.cols)
    xd = torch.from_numpy(xi).to(DEV)
    for lay in LAYOUTS:
        h.set_layout(lay)
        yd = torch.empty(A.rows, dtype=torch.float64, device=DEV)
        h.spmv(xd, yd)
        torch.cuda.synchronize()
        assert np.array_equal(yd.cpu().numpy(), ref), (i, lay)
    h.destroy()

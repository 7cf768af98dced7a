"""IEEE special values through every storage layout of the product: NaN and
infinities in x and in the matrix values must reach exactly the rows whose
entries touch them, whatever the summation order (a NaN term, an infinity
times zero, or infinities of both signs give NaN; infinities of one sign
give that infinity), and must not leak into other rows through padding,
shared scans or staged copies.  Rows that touch no special value stay
within the stated tolerance of the oracle."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2001_07938_amd as L
from tests.helpers import TOL_F32, TOL_F64, assert_rows_close

pytestmark = pytest.mark.gpu

DEV = "cuda"
LAYOUTS = (L.LAYOUT_ROWS, L.LAYOUT_PANELS, L.LAYOUT_BAND, L.LAYOUT_HOT, -1)


def _plant(A, x, seed):
    """NaN and infinities at chosen places: x[0] (the column that padding
    entries name), a few other x entries, and a few matrix values; one zero
    value against an infinite x entry."""
    rng = np.random.default_rng(seed)
    x = x.copy()
    vals = A.vals.copy()
    x[0] = np.nan
    cols = rng.choice(A.cols, size=min(A.cols, 8), replace=False)
    x[cols[1:3]] = np.inf
    x[cols[3:5]] = -np.inf
    x[cols[5:6]] = np.nan
    ks = rng.choice(A.nnz, size=min(A.nnz, 9), replace=False)
    vals[ks[0:3]] = np.nan
    vals[ks[3:6]] = np.inf
    vals[ks[6:8]] = -np.inf
    # an exact zero value against an infinite x entry: 0 * inf = NaN
    hit = np.nonzero(np.isin(A.col_idx, cols[1:2]))[0]
    if hit.size:
        vals[hit[0]] = 0.0
    return gen.Csr(A.rows, A.cols, A.row_ptr, A.col_idx, vals, A.name + "_ieee"), x


def _expected(A, x):
    """Per row: NaN, +inf, -inf or finite, decided term by term (order-free)."""
    rows = np.repeat(np.arange(A.rows), np.diff(A.row_ptr))
    with np.errstate(invalid="ignore", over="ignore"):
        t = A.vals.astype(np.float64) * x[A.col_idx].astype(np.float64)
    nan = np.zeros(A.rows, bool)
    pos = np.zeros(A.rows, bool)
    neg = np.zeros(A.rows, bool)
    np.logical_or.at(nan, rows, np.isnan(t))
    np.logical_or.at(pos, rows, t == np.inf)
    np.logical_or.at(neg, rows, t == -np.inf)
    nan |= pos & neg
    pos &= ~nan
    neg &= ~nan
    return nan, pos, neg


CASES = {
    # long rows (split chunks), empty rows, columns < 65536 (band possible)
    "ragged_split": lambda: gen.ragged(6000, 30000, seed=31, max_len=300,
                                       long_rows=3, long_len=12000, empty_frac=0.2),
    "random5_60": lambda: gen.random_rows(40000, 5, 60, seed=32, cols=40000),
    "stencil27": lambda: gen.stencil(14, 27),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_nan_inf_reach_exactly_their_rows(name, dt):
    A0 = CASES[name]().astype(dt)
    x0 = gen.vector(A0.cols, 33, dtype=dt)
    A, x = _plant(A0, x0, 34)
    nan, pos, neg = _expected(A, x)
    assert nan.any() and pos.any() and neg.any(), "the case must hold every kind"
    fin = ~(nan | pos | neg)
    ref = oracle.spmv_csr(A.row_ptr, A.col_idx, A.vals, x)
    assert np.array_equal(np.isnan(ref), nan)
    with np.errstate(invalid="ignore"):
        mag = oracle.spmv_abs(A.row_ptr, A.col_idx, A.vals, x)
    tol = TOL_F64 if dt == np.float64 else TOL_F32
    tdt = torch.float64 if dt == np.float64 else torch.float32
    h = L.Csr.from_gen(A, cols=A.cols)
    xd = torch.from_numpy(x).to(DEV)
    seen = set()
    for lay in LAYOUTS:
        h.set_layout(lay)
        seen.add(h.info().layout)
        yd = torch.full((A.rows,), 12345.0, dtype=tdt, device=DEV)
        h.spmv(xd, yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy().astype(np.float64)
        assert np.array_equal(np.isnan(y), nan), (name, lay, "NaN rows differ")
        assert np.array_equal(y == np.inf, pos), (name, lay, "+inf rows differ")
        assert np.array_equal(y == -np.inf, neg), (name, lay, "-inf rows differ")
        assert_rows_close(y[fin], ref[fin], mag[fin], tol, f"{name} layout {lay}")
    h.destroy()
    assert L.LAYOUT_HOT in seen and L.LAYOUT_PANELS in seen

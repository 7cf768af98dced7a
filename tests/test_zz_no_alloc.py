"""The CG entry point that allocates nothing (solver state in the library's
fixed device array) against the allocating one, through the C ABI: two
calls in a row, the second on a smaller matrix, each bitwise equal to
lilac_cg without a graph and within the stated tolerance of the oracle's
CG; sizes past the fixed array and handles with pending updates are
refused."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2001_07938_amd as L

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _solve_both(A, iters, seed):
    b = gen.vector(A.rows, seed)
    bd = torch.from_numpy(b).to(DEV)
    h = L.Csr.from_gen(A)
    x_ref = torch.full((A.rows,), np.nan, dtype=torch.float64, device=DEV)
    h.cg(bd, x_ref, iters, graph=False)
    x_na = torch.full((A.rows,), np.nan, dtype=torch.float64, device=DEV)
    h.cg_noalloc(bd, x_na, iters)
    torch.cuda.synchronize()
    got, want = x_na.cpu().numpy(), x_ref.cpu().numpy()
    h.destroy()
    return b, got, want


def test_noalloc_cg_matches_allocating_cg_twice_smaller_second():
    cases = [(gen.spd_random(30000, 40, seed=81), 40),
             (gen.spd_random(4000, 12, seed=82), 25)]   # second call: smaller
    for A, iters in cases:
        b, got, want = _solve_both(A, iters, 83)
        assert np.array_equal(got, want), A.rows
        x_or, done, _ = oracle.cg(A.row_ptr, A.col_idx, A.vals, b, iters)
        assert done == iters
        assert np.max(np.abs(got - x_or)) <= 1e-10 * np.max(np.abs(x_or)), A.rows


def test_noalloc_cg_panel_layout_and_stencil():
    """A column-panel matrix and a band-layout stencil take their own
    product kernels inside the solve."""
    for A in (gen.spd_random(60000, 100, seed=84), gen.stencil(30, 27)):
        b, got, want = _solve_both(A, 30, 85)
        assert np.array_equal(got, want), A.name


def test_noalloc_cg_refuses_what_it_cannot_hold():
    n = (1 << 20) + 1
    big = L.Csr.from_gen(gen.identity(n))
    b = torch.ones(n, dtype=torch.float64, device=DEV)
    x = torch.empty_like(b)
    with pytest.raises(L.LilacError) as e:
        big.cg_noalloc(b, x, 3)
    assert e.value.code == -1 and "1048576" in str(e.value)
    big.destroy()
    A = gen.spd_random(2000, 8, seed=86)
    h = L.Csr.from_gen(A, flags=L.KEEP_HOST)
    vals2 = A.vals * 2.0
    h.update_values(vals2)       # uploads at once: the handle stays usable
    b = torch.from_numpy(gen.vector(A.rows, 87)).to(DEV)
    x = torch.empty_like(b)
    h.cg_noalloc(b, x, 3)
    torch.cuda.synchronize()
    h.invalidate()               # re-upload pending: refused
    with pytest.raises(L.LilacError) as e:
        h.cg_noalloc(b, x, 3)
    assert e.value.code == -6
    # a call that may allocate re-uploads the handle; then it runs
    y = torch.empty_like(b)
    h.spmv(b, y)
    h.cg_noalloc(b, x, 3)
    torch.cuda.synchronize()
    x_or, _, _ = oracle.cg(A.row_ptr, A.col_idx, vals2, b.cpu().numpy(), 3)
    assert np.max(np.abs(x.cpu().numpy() - x_or)) <= 1e-10 * np.max(np.abs(x_or))
    h.destroy()

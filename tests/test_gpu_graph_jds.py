"""The second format (JDS) and SpMV-based BFS on the GPU: both bit-exact
against the oracle."""
import json
import os

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2001_07938_amd as L

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _jds_dict(J):
    return dict(perm=J.perm, nzcnt=J.nzcnt, jd_ptr=J.jd_ptr, col_ind=J.jd_col,
                val=J.jd_val, max_len=J.max_len)


def test_jds_paper_example(golden_dir):
    with open(os.path.join(golden_dir, "jds_5x5.json")) as f:
        j = json.load(f)
    with open(os.path.join(golden_dir, "csr_5x5.json")) as f:
        c = json.load(f)
    y = np.zeros(5)
    L.lilac_spmv_jds(5, 3, np.array(j["perm"], np.int32), np.array(j["nzcnt"], np.int32),
                     np.array(j["jd_ptr"], np.int32), np.array(j["col_ind"], np.int32),
                     np.array(j["val"], np.float64), np.array(c["x_ramp"], np.float64), y)
    assert list(y) == c["y_ramp"]


@pytest.mark.parametrize("rows,cols,max_len", [(1000, 800, 40), (50000, 30000, 300),
                                                (7, 3, 2)])
def test_jds_bitwise_against_oracle(rows, cols, max_len):
    J = gen.random_jds(rows, cols, max_len, seed=rows)
    x = gen.vector(cols, rows + 1)
    ref = oracle.spmv_jds(_jds_dict(J), x)
    y = np.empty(rows)
    L.lilac_spmv_jds(rows, J.max_len, J.perm, J.nzcnt, J.jd_ptr, J.jd_col, J.jd_val, x, y)
    assert np.array_equal(y, ref)
    # device operands
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    yd = torch.empty(rows, dtype=torch.float64, device=DEV)
    L.lilac_spmv_jds(rows, J.max_len, d(J.perm), d(J.nzcnt), d(J.jd_ptr), d(J.jd_col),
                     d(J.jd_val), d(x), yd)
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), ref)


@pytest.mark.parametrize("scale,edges", [(10, 6000), (16, 1 << 19), (20, 1 << 23)])
def test_bfs_levels_bit_exact(scale, edges):
    G = gen.rmat_pagerank(scale, edges, seed=scale)
    h = L.Csr.from_gen(G)
    lens = np.diff(G.row_ptr)
    for src in (int(np.argmax(lens)), 0):
        ref, nref = oracle.bfs_levels(G.row_ptr, G.col_idx, src)
        lvl = torch.empty(G.rows, dtype=torch.int32, device=DEV)
        n = h.bfs(src, lvl)
        torch.cuda.synchronize()
        assert np.array_equal(lvl.cpu().numpy(), ref)
        assert n == nref
    h.destroy()

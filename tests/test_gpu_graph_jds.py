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


def _host_jds(J):
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in J.items()}


def test_csr_to_jds_paper_example(golden_dir):
    """The device conversion of the paper's 5x5 CSR example gives the
    paper's JDS arrays exactly."""
    with open(os.path.join(golden_dir, "jds_5x5.json")) as f:
        j = json.load(f)
    with open(os.path.join(golden_dir, "csr_5x5.json")) as f:
        c = json.load(f)
    h = L.Csr(np.array(c["row_ptr"]), np.array(c["col_ind"]), np.array(c["val"], np.float64))
    J = _host_jds(h.to_jds())
    for key in ("perm", "nzcnt", "jd_ptr", "col_ind"):
        assert list(J[key]) == j[key], key
    assert list(J["val"]) == j["val"]
    assert J["max_len"] == 3
    h.destroy()


JDS_MATS = {
    # the single-product size: 4096 rows, ragged lengths, empty rows and ties
    "ragged4096": lambda: gen.ragged(4096, 4096, seed=61, max_len=40, empty_frac=0.1),
    "uniform4096x16": lambda: gen.uniform_rows(4096, 16),
    "ragged_long": lambda: gen.ragged(30000, 50000, seed=62, max_len=300, long_rows=3,
                                      long_len=20000, dup=True, sort_cols=False),
    "all_empty": lambda: gen.empty_matrix(1000, 10),
    "one_row": lambda: gen.ragged(1, 100, seed=63, max_len=50, empty_frac=0.0),
    "rmat20": lambda: gen.rmat_pagerank(20, 1 << 23, seed=64),
}


@pytest.mark.parametrize("name", sorted(JDS_MATS))
def test_csr_to_jds_bit_exact(name):
    """Every JDS array bit for bit against the oracle's conversion (float64
    and float32 values), then the product over the converted arrays
    bitwise against the oracle's JDS product."""
    A = JDS_MATS[name]()
    ref = oracle.csr_to_jds(A.row_ptr, A.col_idx, A.vals.astype(np.float64))
    for dt in (np.float64, np.float32):
        B = A.astype(dt)
        h = L.Csr.from_gen(B)
        J = _host_jds(h.to_jds())
        assert J["max_len"] == ref["max_len"]
        for key in ("perm", "nzcnt", "jd_ptr", "col_ind"):
            assert np.array_equal(J[key], ref[key]), (name, key)
        assert J["val"].dtype == dt
        assert np.array_equal(J["val"], ref["val"].astype(dt)), name
        h.destroy()
    # the converted arrays feed the JDS product
    h = L.Csr.from_gen(A.astype(np.float64))
    Jd = h.to_jds()
    x = gen.vector(max(A.cols, 1), 65)
    yd = torch.empty(max(A.rows, 1), dtype=torch.float64, device=DEV)
    if A.rows:
        L.lilac_spmv_jds(A.rows, Jd["max_len"], Jd["perm"], Jd["nzcnt"], Jd["jd_ptr"],
                         Jd["col_ind"] if A.nnz else None, Jd["val"] if A.nnz else None,
                         torch.from_numpy(x).to(DEV), yd)
        torch.cuda.synchronize()
        assert np.array_equal(yd.cpu().numpy()[:A.rows], oracle.spmv_jds(ref, x))
    h.destroy()


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

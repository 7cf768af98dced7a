"""The request server on the GPU: results are the same alone and in the mix
(bitwise), agree with the oracle, and admission, eviction, failure and the
trace replay behave."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2001_07938_amd as L
from tests.helpers import TOL_F64, check_spmv

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _workload():
    # layouts: column panels (spd 40000), band (spd 6000, stencils, random
    # rows), row-class tiles (ragged with long rows, the small stencil).  CG
    # requests run on every SPD one: the panel and band products write the
    # r.w partials themselves, the tiles take the separate r.w pass
    spd = [gen.spd_random(6000, 30, seed=1), gen.stencil(16, 7), gen.stencil(10, 27),
           gen.spd_random(40000, 60, seed=4), gen.stencil(8, 7)]
    other = [gen.random_rows(9000, 5, 60, seed=2),
             gen.ragged(2500, 30000, seed=3, long_rows=2, long_len=20000)]
    return spd, other


def _requests(spd, other, ids_spd, ids_other, iters=30):
    reqs = []
    for A, mid in zip(spd + other, ids_spd + ids_other):
        x = gen.vector(A.cols, 100 + mid)
        reqs.append((L.REQ_SPMV, mid, A, x))
    for A, mid in zip(spd, ids_spd):
        b = gen.vector(A.rows, 200 + mid)
        reqs.append((L.REQ_CG, mid, A, b))
    return reqs


def _run(S, reqs, iters, together):
    outs, tickets = [], []
    ins = [_dev(v) for (_, _, _, v) in reqs]
    for (kind, mid, A, v), vin in zip(reqs, ins):
        out = torch.full((A.rows,), np.nan, dtype=torch.float64, device=DEV)
        torch.cuda.synchronize()
        t = S.submit(kind, mid, vin, out, iters=iters)
        if not together:
            S.wait(t)
        outs.append(out)
        tickets.append(t)
    for t in tickets:
        S.wait(t)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def test_server_layouts_cover_all_grouped_paths():
    spd, other = _workload()
    hs = [L.Csr.from_gen(A) for A in spd + other]
    lays = {h.info().layout for h in hs}
    for h in hs:
        h.destroy()
    assert {L.LAYOUT_PANELS, L.LAYOUT_BAND, L.LAYOUT_ROWS} <= lays, lays
    hs = [L.Csr.from_gen(A) for A in spd]
    spd_lays = {h.info().layout for h in hs}
    for h in hs:
        h.destroy()
    assert {L.LAYOUT_PANELS, L.LAYOUT_BAND, L.LAYOUT_ROWS} <= spd_lays, spd_lays


def test_alone_equals_mix_and_oracle():
    spd, other = _workload()
    S = L.Server()
    ids_spd = [S.add_matrix(A) for A in spd]
    ids_other = [S.add_matrix(A) for A in other]
    iters = 30
    reqs = _requests(spd, other, ids_spd, ids_other, iters)
    alone = _run(S, reqs, iters, together=False)
    mix = _run(S, reqs, iters, together=True)
    mix2 = _run(S, reqs[::-1], iters, together=True)[::-1]
    for a, m, m2 in zip(alone, mix, mix2):
        assert np.array_equal(a, m) and np.array_equal(a, m2)
    for (kind, mid, A, v), y in zip(reqs, alone):
        if kind == L.REQ_SPMV:
            check_spmv(A, v, y, TOL_F64)
        else:
            x_or, _, _ = oracle.cg(A.row_ptr, A.col_idx, A.vals, v, iters)
            assert np.max(np.abs(y - x_or)) <= 1e-10 * np.max(np.abs(x_or))
    st = S.stats()
    assert st["completed"] == 3 * len(reqs) and st["failed"] == 0
    assert st["p99_us"] >= st["p50_us"] > 0
    S.destroy()


def test_eviction_keeps_results():
    spd, other = _workload()
    S = L.Server(pool_capacity=2)
    ids = [S.add_matrix(A) for A in spd + other]
    reqs = [(L.REQ_SPMV, mid, A, gen.vector(A.cols, 300 + mid))
            for A, mid in zip(spd + other, ids)] * 2
    ys = _run(S, reqs, 1, together=True)
    for (kind, mid, A, v), y in zip(reqs, ys):
        check_spmv(A, v, y, TOL_F64)
    assert S.stats()["evictions"] > 0
    S.destroy()


def test_budget_too_small_fails_cleanly():
    A = gen.spd_random(20000, 40, seed=5)
    S = L.Server(hbm_budget=1 << 20)
    mid = S.add_matrix(A)
    x = _dev(gen.vector(A.cols, 6))
    y = torch.empty(A.rows, dtype=torch.float64, device=DEV)
    t = S.submit(L.REQ_SPMV, mid, x, y)
    with pytest.raises(L.LilacError):
        S.wait(t)
    assert S.poll(t) == -1
    S.destroy()


def test_fifo_mode_matches_oracle():
    spd, other = _workload()
    S = L.Server(fifo=True)
    ids_spd = [S.add_matrix(A) for A in spd]
    ids_other = [S.add_matrix(A) for A in other]
    iters = 20
    reqs = _requests(spd, other, ids_spd, ids_other, iters)
    ys = _run(S, reqs, iters, together=True)
    for (kind, mid, A, v), y in zip(reqs, ys):
        if kind == L.REQ_SPMV:
            check_spmv(A, v, y, TOL_F64)
        else:
            x_or, _, _ = oracle.cg(A.row_ptr, A.col_idx, A.vals, v, iters)
            assert np.max(np.abs(y - x_or)) <= 1e-10 * np.max(np.abs(x_or))
    S.destroy()


def test_trace_replay_small():
    spd, other = _workload()
    S = L.Server()
    ids = [S.add_matrix(A) for A in spd + other]
    tr = gen.poisson_trace(2000.0, 400, pool_size=len(ids), seed=9)
    mats = np.array(ids)[tr.matrix % len(ids)]
    kind = np.where(np.isin(mats, ids[:len(spd)]), tr.kind, 0)  # CG only on SPD ones
    st = S.run_trace(tr.arrival_ns, kind, mats, 10)
    assert st["completed"] == 400 and st["failed"] == 0
    assert st["cg_done"] == int(kind.sum())
    assert st["p99_us"] >= st["p50_us"] > 0 and st["req_per_s"] > 0
    S.destroy()


def test_budget_pressure_peak_within_budget():
    """A pool whose resident copies need more than a 1 GiB budget: uploads
    wait for idle matrices to be evicted, the server's real device bytes
    (its allocator account: matrices, slots, tables) never pass the budget,
    and every result equals the same request run alone and the oracle."""
    budget = 1 << 30
    mats = [gen.spd_random(60000, 100, seed=11 + i) for i in range(4)]
    mats += [gen.stencil(40, 27), gen.stencil(36, 7),
             gen.random_rows(200000, 5, 60, seed=15), gen.random_rows(120000, 5, 60, seed=16)]
    spd = [True] * 6 + [False] * 2
    S = L.Server(hbm_budget=budget)
    ids = [S.add_matrix(A) for A in mats]
    iters = 15
    reqs = []
    for A, mid, s in zip(mats, ids, spd):
        reqs.append((L.REQ_SPMV, mid, A, gen.vector(A.cols, 400 + mid)))
        if s:
            reqs.append((L.REQ_CG, mid, A, gen.vector(A.rows, 500 + mid)))
    alone = _run(S, reqs, iters, together=False)
    order = list(range(len(reqs)))
    np.random.default_rng(7).shuffle(order)
    mixed = _run(S, [reqs[i] for i in order], iters, together=True)
    st = S.stats()
    assert st["failed"] == 0 and st["completed"] == 2 * len(reqs)
    assert st["evictions"] > 0
    assert 0 < st["peak_device_bytes"] <= budget, st
    assert st["planned_peak_bytes"] <= budget, st
    for k, i in enumerate(order):
        assert np.array_equal(mixed[k], alone[i]), i
    for (kind, mid, A, v), y in zip(reqs, alone):
        if kind == L.REQ_SPMV:
            check_spmv(A, v, y, TOL_F64)
        else:
            x_or, _, _ = oracle.cg(A.row_ptr, A.col_idx, A.vals, v, iters)
            assert np.max(np.abs(y - x_or)) <= 1e-10 * np.max(np.abs(x_or))
    S.destroy()


def test_trace_mode_cg_outputs_do_not_share():
    """Trace-mode requests (no caller vectors) write into their own slot's
    vector: two CG requests on one matrix in flight together both run
    (regression: they once shared one output vector)."""
    A = gen.spd_random(20000, 30, seed=21)
    S = L.Server()
    mid = S.add_matrix(A)
    st = S.run_trace(np.array([0, 1000, 2000, 3000]), np.array([1, 1, 1, 0]),
                     np.array([mid] * 4), 40)
    assert st["completed"] == 4 and st["failed"] == 0 and st["cg_done"] == 3
    assert st["peak_device_bytes"] > 0
    S.destroy()

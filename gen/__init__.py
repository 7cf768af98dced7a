"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This module only builds matrices and vectors (structure and values).  It holds
none of the arithmetic of the method itself (no products, no sums over rows, no
reductions): that lives, independently, in ``oracle/`` and in the HIP library.

CSR layout follows the paper's statement of the format (section "Sparse Matrix
Variations in LiLAC-What", paragraph on CSR, and the worked 5x5 example in the
CSR figure): ``vals`` and ``col_idx`` are flat arrays of the non-zeros in row
order and ``row_ptr[i]`` is the offset of row ``i``; ``rows = len(row_ptr)-1``
and the column count is not part of the format.  Indices are 0-based int32.

Workload recipes (sizes, distributions, seeds) are the synthetic stand-ins for
the paper's evaluation programs: a CG solve (NPB-CG), PageRank over a
power-law graph (the University of Florida graphs), many small stencil and
random matrices, and a stream of requests over resident matrices.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BASE_SEED = 20010793


@dataclasses.dataclass
class Csr:
    rows: int
    cols: int
    row_ptr: np.ndarray  # int32 [rows+1]
    col_idx: np.ndarray  # int32 [nnz]
    vals: np.ndarray     # float64 or float32 [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.rows > 0 else 0

    def astype(self, dtype) -> "Csr":
        return dataclasses.replace(self, vals=self.vals.astype(dtype))


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _from_sorted_keys(rows: int, cols: int, r: np.ndarray, c: np.ndarray,
                      v: np.ndarray, name: str) -> Csr:
    """Build CSR from (row, col, val) triples already sorted by (row, col)."""
    counts = np.bincount(r, minlength=rows).astype(np.int64)
    row_ptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    return Csr(rows, cols, row_ptr.astype(np.int32), c.astype(np.int32),
               np.ascontiguousarray(v), name)


def vector(n: int, seed: int, dtype=np.float64, lo=-1.0, hi=1.0) -> np.ndarray:
    """Dense vector with entries uniform in [lo, hi)."""
    return _rng(seed).uniform(lo, hi, n).astype(dtype)


def int_vector(n: int, seed: int, dtype=np.float64, lo=-4, hi=4) -> np.ndarray:
    """Dense vector of small integers (every partial sum is exact in FP)."""
    return _rng(seed).integers(lo, hi + 1, n).astype(dtype)


# --------------------------------------------------------------------------
# Single-matrix workloads
# --------------------------------------------------------------------------

def uniform_rows(n: int = 4096, per_row: int = 16, seed: int = BASE_SEED + 1,
                 dtype=np.float64) -> Csr:
    """Square n x n, exactly ``per_row`` distinct uniformly random columns per
    row (sorted), values uniform[-1,1)."""
    rng = _rng(seed)
    cols = np.empty((n, per_row), dtype=np.int64)
    for i in range(n):
        cols[i] = np.sort(rng.choice(n, size=per_row, replace=False))
    vals = rng.uniform(-1.0, 1.0, n * per_row).astype(dtype)
    row_ptr = (np.arange(n + 1, dtype=np.int64) * per_row).astype(np.int32)
    return Csr(n, n, row_ptr, cols.reshape(-1).astype(np.int32), vals,
               f"uniform{n}x{per_row}")


def spd_random(n: int = 150_000, half_per_row: int = 120,
               seed: int = BASE_SEED + 2) -> Csr:
    """Symmetric, strictly diagonally dominant (hence SPD) random matrix.

    Row i draws ``half_per_row`` partners j != i uniformly; each distinct
    unordered pair {i, j} receives one value v ~ U[-1,1) stored at (i, j) and
    (j, i).  The diagonal is sum_j |a_ij| + 1.  About 2*half_per_row+1
    entries per row; the exact count is whatever the draw gives.
    """
    rng = _rng(seed)
    i = np.repeat(np.arange(n, dtype=np.int64), half_per_row)
    j = (i + 1 + rng.integers(0, n - 1, i.size)) % n
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key % n
    v = rng.uniform(-1.0, 1.0, key.size)
    diag = np.bincount(lo, weights=np.abs(v), minlength=n) + \
        np.bincount(hi, weights=np.abs(v), minlength=n) + 1.0
    r = np.concatenate([lo, hi, np.arange(n, dtype=np.int64)])
    c = np.concatenate([hi, lo, np.arange(n, dtype=np.int64)])
    vv = np.concatenate([v, v, diag])
    order = np.argsort(r * n + c, kind="stable")
    return _from_sorted_keys(n, n, r[order], c[order], vv[order],
                             f"spd{n}")


def rmat_edges(scale: int, n_edges: int, a=0.57, b=0.19, c=0.19,
               seed: int = BASE_SEED + 3):
    """R-MAT edge sampler (Chakrabarti, Zhan, Faloutsos 2004): each edge picks
    one of four quadrants per level with probabilities (a, b, c, d).  Returns
    (src, dst) int64 arrays, duplicates included."""
    rng = _rng(seed)
    src = np.zeros(n_edges, dtype=np.int64)
    dst = np.zeros(n_edges, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for _ in range(scale):
        u = rng.random(n_edges, dtype=np.float32)
        down = u >= ab                       # quadrants c, d: source bit 1
        right = ((u >= a) & (u < ab)) | (u >= abc)   # quadrants b, d
        src = (src << 1) | down
        dst = (dst << 1) | right
    return src, dst


def rmat_pagerank(scale: int = 22, n_edges: int = 1 << 26,
                  seed: int = BASE_SEED + 3) -> Csr:
    """Pull-direction CSR of an R-MAT graph for PageRank.

    Vertices are relabelled with a seeded random permutation (so hubs are
    spread out), duplicate edges are removed, self loops kept, and the matrix
    is A[v, u] = 1/outdeg(u) for every edge u -> v, stored float32, columns
    sorted within each row.  Rows are destinations, columns are sources.
    """
    nv = 1 << scale
    src, dst = rmat_edges(scale, n_edges, seed=seed)
    perm = _rng(seed + 1000).permutation(nv).astype(np.int64)
    key = (perm[dst] << scale) | perm[src]
    del src, dst
    key = np.unique(key)            # sorted by (destination, source), deduped
    dst = key >> scale
    src = key & (nv - 1)
    del key
    outdeg = np.bincount(src, minlength=nv)
    w = (1.0 / outdeg[src]).astype(np.float32)
    return _from_sorted_keys(nv, nv, dst, src, w, f"rmat{scale}")


def relabel_by_degree(A: Csr) -> Csr:
    """The same graph with vertices renumbered by decreasing number of
    stored entries per column (most referenced column first, ties in index
    order), rows and columns renumbered alike; values move with their
    entries.  A structural relabelling only: no value is computed."""
    n = A.rows
    assert A.cols == n
    deg = np.bincount(A.col_idx, minlength=n)
    order = np.argsort(-deg, kind="stable")
    newid = np.empty(n, dtype=np.int64)
    newid[order] = np.arange(n, dtype=np.int64)
    r = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.row_ptr))
    key = (newid[r] << 32) | newid[A.col_idx]
    o = np.argsort(key, kind="stable")
    return _from_sorted_keys(n, n, newid[r][o], newid[A.col_idx][o], A.vals[o],
                             A.name + "_bydeg")


def stencil(k: int, points: int = 7) -> Csr:
    """3D Laplacian-style stencil on a k^3 grid with Dirichlet truncation.
    7-point: diagonal 6, neighbours -1.  27-point: diagonal 26, neighbours -1.
    Columns sorted within rows."""
    assert points in (7, 27)
    n = k ** 3
    if points == 7:
        offs = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0),
                (0, 0, 1), (0, 1, 0), (1, 0, 0)]
    else:
        offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1)
                for dx in (-1, 0, 1)]
    offs.sort(key=lambda o: o[0] * k * k + o[1] * k + o[2])
    idx = np.arange(n, dtype=np.int64)
    z, y, x = idx // (k * k), (idx // k) % k, idx % k
    colm = np.full((n, len(offs)), -1, dtype=np.int64)
    valm = np.zeros((n, len(offs)), dtype=np.float64)
    for t, (dz, dy, dx) in enumerate(offs):
        ok = ((z + dz >= 0) & (z + dz < k) & (y + dy >= 0) & (y + dy < k) &
              (x + dx >= 0) & (x + dx < k))
        colm[ok, t] = idx[ok] + dz * k * k + dy * k + dx
        valm[ok, t] = float(points - 1) if (dz, dy, dx) == (0, 0, 0) else -1.0
    mask = colm >= 0
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Csr(n, n, row_ptr.astype(np.int32), colm[mask].astype(np.int32),
               valm[mask], f"stencil{points}_{k}")


def random_rows(n: int, lo: int = 5, hi: int = 60, seed: int = BASE_SEED + 4,
                cols: Optional[int] = None, dtype=np.float64) -> Csr:
    """n rows, each with a uniform integer count in [lo, hi] of distinct
    uniformly random columns (sorted), values U[-1,1).  Not symmetric."""
    rng = _rng(seed)
    cols = n if cols is None else cols
    cnt = rng.integers(lo, hi + 1, n).astype(np.int64)
    r = np.repeat(np.arange(n, dtype=np.int64), cnt)
    c = rng.integers(0, cols, r.size).astype(np.int64)
    key = np.unique(r * cols + c)
    r = key // cols
    c = key % cols
    v = rng.uniform(-1.0, 1.0, key.size).astype(dtype)
    return _from_sorted_keys(n, cols, r, c, v, f"random{n}")


# --------------------------------------------------------------------------
# Test-shaped matrices (ragged rows, empty rows, long rows, duplicates)
# --------------------------------------------------------------------------

def ragged(rows: int, cols: int, seed: int, max_len: int = 200,
           long_rows: int = 0, long_len: int = 20000, empty_frac: float = 0.1,
           dup: bool = False, sort_cols: bool = True, dtype=np.float64,
           integer_vals: bool = False) -> Csr:
    """Rows with a wide spread of lengths: a fraction empty, a geometric-ish
    spread up to ``max_len`` and ``long_rows`` rows of about ``long_len``.
    With ``dup`` a column may repeat inside a row; with ``sort_cols=False``
    columns are left in draw order."""
    rng = _rng(seed)
    lens = np.minimum(max_len, np.floor(rng.pareto(1.2, rows) * 8).astype(np.int64))
    lens[rng.random(rows) < empty_frac] = 0
    if long_rows:
        which = rng.choice(rows, size=min(long_rows, rows), replace=False)
        lens[which] = long_len + rng.integers(0, long_len // 4 + 1, which.size)
    if not dup:
        lens = np.minimum(lens, cols)
    row_ptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col_idx = np.empty(nnz, dtype=np.int64)
    for i in np.nonzero(lens)[0]:
        a, b = row_ptr[i], row_ptr[i + 1]
        if dup:
            cc = rng.integers(0, cols, b - a)
        else:
            cc = rng.choice(cols, size=b - a, replace=False) if b - a < cols // 4 \
                else rng.permutation(cols)[: b - a]
        col_idx[a:b] = np.sort(cc) if sort_cols else cc
    if integer_vals:
        vals = rng.integers(-3, 4, nnz).astype(dtype)
    else:
        vals = rng.uniform(-1.0, 1.0, nnz).astype(dtype)
    return Csr(rows, cols, row_ptr.astype(np.int32), col_idx.astype(np.int32),
               vals, f"ragged{rows}x{cols}")


def strided_rows(rows: int, k: int, cols: int, seed: int,
                 dtype=np.float32, chunk_rows: int = 1 << 17,
                 window: bool = False) -> Csr:
    """Exactly k distinct columns per row, {(a_i + j*s) mod cols : j < k}
    with s = cols // k and a seeded random offset a_i, stored in ascending
    order; with ``window`` instead the k consecutive columns a_i ... a_i +
    k - 1 (a_i <= cols - k).  Integer values in [-8, 8] (exact in float32
    and float64).  The row offsets are int64, so rows * k may reach past
    2^31 (the matrices of the 64-bit-offset handles); built in chunks of
    rows."""
    if k < 1 or cols < k:
        raise ValueError("need 1 <= k <= cols")
    rng = _rng(seed)
    s = 1 if window else cols // k
    nnz = rows * k
    row_ptr = np.arange(rows + 1, dtype=np.int64) * k
    col_idx = np.empty(nnz, dtype=np.int32)
    vals = np.empty(nnz, dtype=dtype)
    a_all = rng.integers(0, cols - k + 1 if window else cols, rows, dtype=np.int64)
    j = np.arange(k, dtype=np.int64)
    for r0 in range(0, rows, chunk_rows):
        r1 = min(rows, r0 + chunk_rows)
        a = a_all[r0:r1, None]
        if window:
            c = a.astype(np.int32) + j.astype(np.int32)[None, :]
        elif k * s == cols:
            # the steps cover cols exactly: the row is a % s, a % s + s, ...
            c = ((a % s).astype(np.int32) + (j * s).astype(np.int32)[None, :])
        else:
            # entries j >= j0 wrap past cols; listing them first keeps the
            # row sorted
            j0 = np.minimum(k, -((a - cols) // s))
            m = (j[None, :] + j0) % k
            c = a + m * s
            c -= cols * (c >= cols)
        col_idx[r0 * k:r1 * k] = c.reshape(-1)
        vals[r0 * k:r1 * k] = rng.integers(-8, 9, (r1 - r0) * k, dtype=np.int8)
    return Csr(rows, cols, row_ptr, col_idx, vals, f"strided{rows}x{k}")


def identity(n: int) -> Csr:
    return Csr(n, n, np.arange(n + 1, dtype=np.int32),
               np.arange(n, dtype=np.int32), np.ones(n), f"eye{n}")


def permutation(n: int, seed: int) -> Csr:
    """Row i holds a single 1 at column pi[i]."""
    pi = _rng(seed).permutation(n).astype(np.int32)
    return Csr(n, n, np.arange(n + 1, dtype=np.int32), pi, np.ones(n),
               f"perm{n}")


def empty_matrix(rows: int, cols: int) -> Csr:
    return Csr(rows, cols, np.zeros(rows + 1, dtype=np.int32),
               np.zeros(0, dtype=np.int32), np.zeros(0), "empty")


def diag_distinct(n: int, k: int, seed: int) -> Csr:
    """Diagonal SPD matrix with exactly k distinct eigenvalues (CG converges
    in k steps in exact arithmetic)."""
    rng = _rng(seed)
    ev = np.sort(rng.uniform(1.0, 10.0, k))
    d = ev[rng.integers(0, k, n)]
    d[:k] = ev  # every value present
    return Csr(n, n, np.arange(n + 1, dtype=np.int32),
               np.arange(n, dtype=np.int32), d, f"diag{n}k{k}")


def cycle_graph(n: int) -> Csr:
    """Pull CSR of the directed cycle u -> u+1 (mod n); each out-degree 1."""
    src = (np.arange(n) - 1) % n
    return Csr(n, n, np.arange(n + 1, dtype=np.int32), src.astype(np.int32),
               np.ones(n, dtype=np.float32), f"cycle{n}")


def star_graph(n: int) -> Csr:
    """Pull CSR of a star: leaves 1..n-1 each point to the hub 0 and the hub
    points back to every leaf.  Row 0 has n-1 entries (weight 1 each, leaves
    have out-degree 1); each leaf row holds the hub with weight 1/(n-1)."""
    row_ptr = np.concatenate([[0], np.arange(n - 1, 2 * n - 1)]).astype(np.int32)
    cols = np.concatenate([np.arange(1, n), np.zeros(n - 1, dtype=np.int64)])
    vals = np.concatenate([np.ones(n - 1), np.full(n - 1, 1.0 / (n - 1))])
    return Csr(n, n, row_ptr, cols.astype(np.int32), vals.astype(np.float32),
               f"star{n}")


# --------------------------------------------------------------------------
# Batched and serving workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass
class MatrixSpec:
    kind: str     # "st7", "st27", "rand"
    n: int        # requested size (stencils round to k^3)
    seed: int

    def build(self) -> Csr:
        if self.kind == "st7":
            return stencil(max(2, round(self.n ** (1.0 / 3.0))), 7)
        if self.kind == "st27":
            return stencil(max(2, round(self.n ** (1.0 / 3.0))), 27)
        return random_rows(self.n, 5, 60, seed=self.seed)


@dataclasses.dataclass
class SpdSpec:
    n: int = 150_000
    half_per_row: int = 120
    seed: int = BASE_SEED + 2

    def build(self) -> Csr:
        return spd_random(self.n, self.half_per_row, self.seed)


def batch_specs(count: int = 512, n_lo: int = 1000, n_hi: int = 200_000,
                seed: int = BASE_SEED + 4) -> List[MatrixSpec]:
    """Sizes log-uniform in [n_lo, n_hi]; kinds cycle through 7-point,
    27-point and random 5-60/row in equal thirds (assigned by a seeded
    shuffle)."""
    rng = _rng(seed)
    ns = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count))
    kinds = np.array(["st7", "st27", "rand"])[np.arange(count) % 3]
    rng.shuffle(kinds)
    return [MatrixSpec(str(kinds[t]), int(round(ns[t])), seed * 7 + t)
            for t in range(count)]


@dataclasses.dataclass
class Trace:
    arrival_ns: np.ndarray   # int64, ascending
    kind: np.ndarray         # int32: 0 = SpMV, 1 = CG solve
    matrix: np.ndarray       # int32: slot in the pool (>= pool_size: new upload)
    iters: int


def poisson_trace(lam: float, n_req: int, pool_size: int = 64,
                  n_spd: int = 4, reuse: float = 0.9, cg_frac: float = 0.2,
                  cg_iters: int = 50, seed: int = BASE_SEED + 5) -> Trace:
    """Open-loop Poisson arrivals at rate ``lam`` per second.  Each request
    names a pool matrix (reuse) or a new one to upload (1-reuse).  CG requests
    only target SPD matrices (the first ``n_spd`` pool slots and stencils);
    the caller decides which pool slots are SPD."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / lam, n_req)
    t = np.cumsum(gaps)
    arrival = np.round(t * 1e9).astype(np.int64)
    kind = (rng.random(n_req) < cg_frac).astype(np.int32)
    new = rng.random(n_req) >= reuse
    mat = rng.integers(0, pool_size, n_req).astype(np.int32)
    mat[new] = pool_size + np.arange(int(new.sum()), dtype=np.int32)
    return Trace(arrival, kind, mat, cg_iters)


@dataclasses.dataclass
class Jds:
    rows: int
    cols: int
    max_len: int
    perm: np.ndarray     # int32 [rows]: position of original row i
    nzcnt: np.ndarray    # int32 [rows]: entries of the row at position p
    jd_ptr: np.ndarray   # int32 [max_len+1]
    jd_col: np.ndarray   # int32 [nnz]
    jd_val: np.ndarray   # float64 [nnz]


def random_jds(rows: int, cols: int, max_len: int, seed: int,
               empty_frac: float = 0.1) -> Jds:
    """A random matrix drawn directly in Jagged Diagonal Storage: row
    lengths (a tenth empty by default) sorted in decreasing order, a random
    row permutation, and diagonal j listing the j-th entry of every row with
    more than j entries (random columns, values U[-1,1))."""
    rng = _rng(seed)
    lens = rng.integers(0, max_len + 1, rows)
    lens[rng.random(rows) < empty_frac] = 0
    nzcnt = np.sort(lens)[::-1].astype(np.int32)
    perm = rng.permutation(rows).astype(np.int32)
    ml = int(nzcnt.max()) if rows else 0
    per_diag = np.array([int(np.sum(nzcnt > j)) for j in range(ml)], dtype=np.int64)
    jd_ptr = np.zeros(ml + 1, dtype=np.int64)
    np.cumsum(per_diag, out=jd_ptr[1:])
    nnz = int(jd_ptr[-1])
    return Jds(rows, cols, ml, perm, nzcnt, jd_ptr.astype(np.int32),
               rng.integers(0, cols, nnz).astype(np.int32),
               rng.uniform(-1.0, 1.0, nnz))

"""Python access to the plain C oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports, links or
calls anything here, and this module imports nothing from the product.

Every function takes and returns numpy arrays; the arithmetic happens in the
C file, built with ``gcc -O2 -ffp-contract=off`` (see ``build``).

Parity status of each function (what pins it, see ``tests/test_oracle_*.py``):
  spmv_csr / spmv_csr_f32 / spmv_abs : pinned (paper's 5x5 example, dense
      matvec, exact rational arithmetic, identity/permutation, scipy CSR;
      the float32 |A||x| scale against scipy on the widened arrays)
  spmv_csr_par                       : pinned (bitwise equal to spmv_csr)
  dot / dot_abs                      : pinned (closed forms, fsum, Fraction)
  cg                                 : pinned (direct solve, k-eigenvalue
      finite termination, zero right-hand side, A-norm monotonicity)
  pagerank_step / pagerank           : pinned (mass identity, cycle fixed
      point, star closed form, several steps on a cycle from a non-uniform
      start against x_k = d^k P^k x0 + (1 - d^k)/N)
  bins / split_chunks / cols / validate : pinned (library sort/search special
      cases, invariants, crafted bad inputs)
  csr_to_jds / spmv_jds              : pinned (paper's JDS example)
  bfs_levels                         : pinned (scipy breadth-first distances)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC",
          "-shared", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)


def _declare(L):
    I32, I64, F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.c_void_p
    L.oracle_csr_validate.argtypes = [I32, P, P, I32]
    L.oracle_csr_validate.restype = ctypes.c_int
    L.oracle_csr_cols.argtypes = [I64, P]
    L.oracle_csr_cols.restype = I32
    for nm in ("oracle_spmv_csr_f64", "oracle_spmv_csr_f32",
               "oracle_spmv_abs_f64", "oracle_spmv_abs_f32", "oracle_spmv_csr_f64_par"):
        getattr(L, nm).argtypes = [I32, P, P, P, P, P]
        getattr(L, nm).restype = None
    L.oracle_threads.argtypes = []
    L.oracle_threads.restype = ctypes.c_int
    L.oracle_dot.argtypes = [I64, P, P]
    L.oracle_dot.restype = F64
    L.oracle_dot_abs.argtypes = [I64, P, P]
    L.oracle_dot_abs.restype = F64
    L.oracle_cg.argtypes = [I32, P, P, P, P, P, ctypes.c_int, P]
    L.oracle_cg.restype = ctypes.c_int
    L.oracle_pagerank_step_f32.argtypes = [I32, P, P, P, P, F64, P]
    L.oracle_pagerank_step_f32.restype = None
    L.oracle_pagerank_f64.argtypes = [I32, P, P, P, F64, ctypes.c_int, P]
    L.oracle_pagerank_f64.restype = None
    L.oracle_bins.argtypes = [I32, P, I32, P, P, P, P]
    L.oracle_bins.restype = None
    L.oracle_split_chunks.argtypes = [I32, P, I32, I32, P, P, P]
    L.oracle_split_chunks.restype = I64
    L.oracle_csr_to_jds.argtypes = [I32, P, P, P, P, P, P, P, P]
    L.oracle_csr_to_jds.restype = I32
    L.oracle_spmv_jds_f64.argtypes = [I32, I32, P, P, P, P, P, P, P]
    L.oracle_spmv_jds_f64.restype = None
    L.oracle_bfs_levels.argtypes = [I32, P, P, I32, P]
    L.oracle_bfs_levels.restype = I32


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- structure

def validate(row_ptr, col_idx, cols: int = -1) -> int:
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    rows = rp.size - 1
    if rows >= 0 and rp.size > 0 and rp[0] == 0 and np.all(np.diff(rp) >= 0):
        if ci.size < rp[-1]:
            raise ValueError("col_idx shorter than row_ptr[rows]")
    return lib().oracle_csr_validate(rows, _p(rp), _p(ci), int(cols))


def cols(col_idx) -> int:
    ci = _c(col_idx, np.int32)
    return lib().oracle_csr_cols(ci.size, _p(ci))


# ---------------------------------------------------------------- SpMV / dot

def spmv_csr_par(row_ptr, col_idx, vals, x) -> np.ndarray:
    """spmv_csr for float64 data with the rows shared among host threads
    (identical result); for timing the host baseline on all its cores."""
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    rows = rp.size - 1
    y = np.empty(rows, dtype=np.float64)
    lib().oracle_spmv_csr_f64_par(rows, _p(rp), _p(ci), _p(_c(vals, np.float64)),
                                  _p(_c(x, np.float64)), _p(y))
    return y


def threads() -> int:
    """Host threads the parallel oracle product uses (OMP_NUM_THREADS)."""
    return int(lib().oracle_threads())


def spmv_csr(row_ptr, col_idx, vals, x) -> np.ndarray:
    """y = A x in binary64 (float32 inputs are widened first)."""
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    rows = rp.size - 1
    y = np.empty(rows, dtype=np.float64)
    if np.asarray(vals).dtype == np.float32:
        v = _c(vals, np.float32)
        xx = _c(x, np.float32)
        lib().oracle_spmv_csr_f32(rows, _p(rp), _p(ci), _p(v), _p(xx), _p(y))
    else:
        v = _c(vals, np.float64)
        xx = _c(x, np.float64)
        lib().oracle_spmv_csr_f64(rows, _p(rp), _p(ci), _p(v), _p(xx), _p(y))
    return y


def spmv_abs(row_ptr, col_idx, vals, x) -> np.ndarray:
    """Per-row sum |a_ik| |x_k|."""
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    rows = rp.size - 1
    y = np.empty(rows, dtype=np.float64)
    if np.asarray(vals).dtype == np.float32:
        lib().oracle_spmv_abs_f32(rows, _p(rp), _p(ci), _p(_c(vals, np.float32)),
                                  _p(_c(x, np.float32)), _p(y))
    else:
        lib().oracle_spmv_abs_f64(rows, _p(rp), _p(ci), _p(_c(vals, np.float64)),
                                  _p(_c(x, np.float64)), _p(y))
    return y


def dot(a, b) -> float:
    a = _c(a, np.float64)
    b = _c(b, np.float64)
    assert a.size == b.size
    return lib().oracle_dot(a.size, _p(a), _p(b))


def dot_abs(a, b) -> float:
    a = _c(a, np.float64)
    b = _c(b, np.float64)
    return lib().oracle_dot_abs(a.size, _p(a), _p(b))


# ---------------------------------------------------------------- solvers

def cg(row_ptr, col_idx, vals, b, iters: int):
    """Returns (x, completed_iterations, rho_history)."""
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    v = _c(vals, np.float64)
    bb = _c(b, np.float64)
    n = rp.size - 1
    x = np.zeros(n, dtype=np.float64)
    hist = np.empty(iters + 1, dtype=np.float64)
    done = lib().oracle_cg(n, _p(rp), _p(ci), _p(v), _p(bb), _p(x), iters,
                           _p(hist))
    return x, done, hist


def pagerank_step(row_ptr, col_idx, vals_f32, x_f32, d: float) -> np.ndarray:
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    y = np.empty(rp.size - 1, dtype=np.float64)
    lib().oracle_pagerank_step_f32(rp.size - 1, _p(rp), _p(ci),
                                   _p(_c(vals_f32, np.float32)),
                                   _p(_c(x_f32, np.float32)), float(d), _p(y))
    return y


def pagerank(row_ptr, col_idx, vals_f32, x0, d: float, iters: int) -> np.ndarray:
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    x = np.array(x0, dtype=np.float64, copy=True)
    lib().oracle_pagerank_f64(rp.size - 1, _p(rp), _p(ci),
                              _p(_c(vals_f32, np.float32)), float(d), iters,
                              _p(x))
    return x


# ---------------------------------------------------------------- analysis

def bins(row_ptr, upper):
    """Returns (bin_of_row, bin_off, bin_rows)."""
    rp = _c(row_ptr, np.int32)
    up = _c(upper, np.int32)
    rows = rp.size - 1
    bor = np.empty(rows, dtype=np.int32)
    off = np.empty(up.size + 1, dtype=np.int32)
    br = np.empty(rows, dtype=np.int32)
    lib().oracle_bins(rows, _p(rp), up.size, _p(up), _p(bor), _p(off), _p(br))
    return bor, off, br


def split_chunks(row_ptr, t_split: int, chunk: int):
    """Returns (c_row, c_k0, c_k1)."""
    rp = _c(row_ptr, np.int32)
    rows = rp.size - 1
    m = lib().oracle_split_chunks(rows, _p(rp), t_split, chunk, None, None, None)
    cr = np.empty(m, dtype=np.int32)
    c0 = np.empty(m, dtype=np.int32)
    c1 = np.empty(m, dtype=np.int32)
    lib().oracle_split_chunks(rows, _p(rp), t_split, chunk, _p(cr), _p(c0), _p(c1))
    return cr, c0, c1


def csr_to_jds(row_ptr, col_idx, vals):
    """Returns dict(perm, nzcnt, jd_ptr, col_ind, val, max_len)."""
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    v = _c(vals, np.float64)
    rows = rp.size - 1
    nnz = int(rp[-1]) if rows > 0 else 0
    max_len = int(np.max(np.diff(rp))) if rows > 0 else 0
    perm = np.empty(rows, dtype=np.int32)
    nzcnt = np.empty(rows, dtype=np.int32)
    jd_ptr = np.empty(max_len + 1, dtype=np.int32)
    jc = np.empty(max(nnz, 1), dtype=np.int32)
    jv = np.empty(max(nnz, 1), dtype=np.float64)
    ml = lib().oracle_csr_to_jds(rows, _p(rp), _p(ci), _p(v), _p(perm),
                                 _p(nzcnt), _p(jd_ptr), _p(jc), _p(jv))
    return dict(perm=perm, nzcnt=nzcnt, jd_ptr=jd_ptr, col_ind=jc[:nnz],
                val=jv[:nnz], max_len=ml)


def spmv_jds(jds, x) -> np.ndarray:
    rows = jds["perm"].size
    y = np.empty(rows, dtype=np.float64)
    jc = _c(jds["col_ind"], np.int32)
    jv = _c(jds["val"], np.float64)
    lib().oracle_spmv_jds_f64(rows, jds["max_len"], _p(jds["perm"]),
                              _p(jds["nzcnt"]), _p(jds["jd_ptr"]), _p(jc),
                              _p(jv), _p(_c(x, np.float64)), _p(y))
    return y


def bfs_levels(row_ptr, col_idx, source: int):
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    lvl = np.empty(rp.size - 1, dtype=np.int32)
    n = lib().oracle_bfs_levels(rp.size - 1, _p(rp), _p(ci), int(source), _p(lvl))
    return lvl, n

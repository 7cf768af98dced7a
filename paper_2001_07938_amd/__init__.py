"""Python binding of liblilac.so (CSR SpMV + dot for AMD Instinct MI355X).

Argument marshalling only: every computation runs in the library's HIP
kernels.  The names follow the C ABI in ``include/lilac.h``.  PyTorch is
imported first so that the library shares torch's HIP runtime; torch tensors
(host or device) and numpy arrays are accepted wherever the C ABI takes a
pointer.  The library is loaded on first use; if it has not been built that
first call raises ImportError (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (shares its HIP runtime with the library)

__all__ = [
    "LilacError", "lib", "lilac_spmv_csr", "lilac_spmv_csr_f32", "lilac_dot",
    "lilac_invalidate", "lilac_release_all", "lilac_init", "lilac_finalize",
    "lilac_dot_dev", "lilac_spmv_batched", "lilac_spmv_batched_tune", "lilac_hbm_stream", "Csr", "Csr64", "F64", "F32",
    "KEEP_HOST", "CG_GRAPH", "NCLASS", "HEADER_FUNCTIONS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblilac.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lilac.h")

F64, F32 = 0, 1
LAYOUT_AUTO, LAYOUT_ROWS, LAYOUT_PANELS, LAYOUT_HOT, LAYOUT_BAND = -1, 0, 1, 2, 3
KEEP_HOST = 1
CG_GRAPH = 1
NCLASS = 9

ERRORS = {-1: "LILAC_ERR_ARG", -2: "LILAC_ERR_CSR", -3: "LILAC_ERR_OOM",
          -4: "LILAC_ERR_BUDGET", -5: "LILAC_ERR_DEVICE", -6: "LILAC_ERR_STATE",
          -7: "LILAC_ERR_UNSUPPORTED"}


class LilacError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class CsrInfo(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int), ("cols", ctypes.c_int),
                ("nnz", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("dtype", ctypes.c_int), ("nbins", ctypes.c_int),
                ("bin_upper", ctypes.c_int * 16), ("bin_count", ctypes.c_int * 16),
                ("chunk", ctypes.c_int), ("nchunks", ctypes.c_int64),
                ("ntiles", ctypes.c_int), ("layout", ctypes.c_int),
                ("npanels", ctypes.c_int)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_SIGS = {
    "lilac_init": ([_I], _I),
    "lilac_finalize": ([], _I),
    "lilac_last_error": ([], ctypes.c_char_p),
    "lilac_version": ([], _I),
    "lilac_spmv_csr": ([_I, _P, _P, _P, _P, _P], _I),
    "lilac_spmv_csr_f32": ([_I, _P, _P, _P, _P, _P], _I),
    "lilac_dot": ([_I64, _P, _P], ctypes.c_double),
    "lilac_dot_f32": ([_I64, _P, _P], ctypes.c_float),
    "lilac_invalidate": ([_P], _I),
    "lilac_release_all": ([], _I),
    "lilac_csr_create": ([ctypes.POINTER(_P), _I, _I, _I64, _P, _P, _P, _I,
                          ctypes.c_uint], _I),
    "lilac_csr_update_values": ([_P, _P], _I),
    "lilac_csr_invalidate": ([_P], _I),
    "lilac_csr_destroy": ([_P], _I),
    "lilac_csr_info": ([_P, ctypes.POINTER(CsrInfo)], _I),
    "lilac_csr_analysis": ([_P, _P, _P, _P, _P, _P], _I),
    "lilac_csr_set_plan": ([_P, _P, _P, _I], _I),
    "lilac_csr_set_layout": ([_P, _I], _I),
    "lilac_spmv": ([_P, _P, _P, _P], _I),
    "lilac_spmv_dot": ([_P, _P, _P, _P, _P, _P], _I),
    "lilac_dot_dev": ([_I64, _P, _P, _P, _I, _P], _I),
    "lilac_cg": ([_P, _P, _P, _I, ctypes.c_uint, _P, _P, _P], _I),
    "lilac_pagerank": ([_P, ctypes.c_float, _I, _P, _P], _I),
    "lilac_spmv_batched": ([_I, _P, _P, _P, _P], _I),
    "lilac_csr64_create": ([ctypes.POINTER(_P), _I, _I, _I64, _P, _P, _P, _I], _I),
    "lilac_csr64_spmv": ([_P, _P, _P, _P], _I),
    "lilac_csr64_info": ([_P, _P, _P, _P, _P], _I),
    "lilac_csr64_destroy": ([_P], _I),
    "lilac_csr_tune": ([_P, _P], _I),
    "lilac_csr_tune_class": ([_P, ctypes.c_char_p, _I], _I),
    "lilac_tune_clear": ([], _I),
    "lilac_hbm_stream": ([_P, _P, _I64, _I, _P], _I),
    "lilac_spmv_batched_tune": ([_I, _P, _P, _P, _P], _I),
    "lilac_bfs": ([_P, _I, _P, _P, _P], _I),
    "lilac_spmv_jds": ([_I, _I, _P, _P, _P, _P, _P, _P, _P], _I),
    "lilac_csr_to_jds": ([_P, _P, _P, _P, _I, _P, _P, _P, _P], _I),
    "lilac_cg_noalloc": ([_P, _P, _P, _I, _P], _I),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load liblilac.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2001_07938_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib




def header_functions() -> list:
    """Names of the functions declared in include/lilac.h."""
    import re
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lilac_[a-z0-9_]+)\s*\(", txt)))


HEADER_FUNCTIONS = header_functions()


def _check(st: int):
    if st != 0:
        raise LilacError(st, lib().lilac_last_error().decode())


def _ptr(a) -> Optional[int]:
    """Address of a numpy array / torch tensor / raw int (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr()
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data
    if isinstance(a, int):
        return a
    raise TypeError(f"unsupported argument type {type(a)}")


def _stream(stream) -> Optional[int]:
    """hipStream_t for an async call: torch's current stream by default, so
    the work is ordered after the torch operations that produced its
    inputs."""
    if stream is None:
        return torch.cuda.current_stream().cuda_stream or None
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream or None
    return int(stream) or None


def _elem_size(a) -> int:
    if isinstance(a, torch.Tensor):
        return a.element_size()
    if isinstance(a, np.ndarray):
        return a.itemsize
    raise TypeError("pass dtype= with a raw pointer")


def _as_i32(a):
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.int32:
            raise TypeError("index arrays must be int32")
        return a
    return np.ascontiguousarray(a, dtype=np.int32)


# ------------------------------------------------------------ paper-shaped

def lilac_init(device: int = -1):
    _check(lib().lilac_init(device))


def lilac_finalize():
    _check(lib().lilac_finalize())


def lilac_spmv_csr(rows: int, row_ptr, col_idx, vals, x, y):
    """y = A x (float64).  Arguments: numpy arrays or torch tensors, host or
    device; y is written in place."""
    _check(lib().lilac_spmv_csr(rows, _ptr(row_ptr), _ptr(col_idx), _ptr(vals),
                                _ptr(x), _ptr(y)))
    return y


def lilac_spmv_csr_f32(rows: int, row_ptr, col_idx, vals, x, y):
    _check(lib().lilac_spmv_csr_f32(rows, _ptr(row_ptr), _ptr(col_idx),
                                    _ptr(vals), _ptr(x), _ptr(y)))
    return y


def lilac_dot(n: int, a, b) -> float:
    r = lib().lilac_dot(n, _ptr(a), _ptr(b))
    if np.isnan(r):
        err = lib().lilac_last_error().decode()
        if err:
            raise LilacError(-1, err)
    return r


def lilac_dot_f32(n: int, a, b) -> float:
    r = lib().lilac_dot_f32(n, _ptr(a), _ptr(b))
    if np.isnan(r):
        err = lib().lilac_last_error().decode()
        if err:
            raise LilacError(-1, err)
    return r


def lilac_dot_dev(n: int, a, b, out, dtype: int = None, stream=None):
    """out = a . b on the device; dtype defaults to out's element type."""
    if dtype is None:
        dtype = F32 if _elem_size(out) == 4 else F64
    _check(lib().lilac_dot_dev(n, _ptr(a), _ptr(b), _ptr(out), dtype, _stream(stream)))


def lilac_hbm_stream(src, nbytes: int, dst=None, groups_per_cu: int = 8, stream=None):
    """Streams nbytes of device memory (read, or copy into dst)."""
    _check(lib().lilac_hbm_stream(_ptr(src), _ptr(dst), nbytes, groups_per_cu,
                                  _stream(stream)))


def lilac_invalidate(ptr):
    _check(lib().lilac_invalidate(_ptr(ptr)))


def lilac_release_all():
    _check(lib().lilac_release_all())


def lilac_spmv_jds(rows: int, max_len: int, perm, nzcnt, jd_ptr, jd_col,
                   jd_val, x, y):
    """y = A x with A in Jagged Diagonal Storage (see include/lilac.h)."""
    _check(lib().lilac_spmv_jds(rows, max_len, _ptr(perm), _ptr(nzcnt),
                                _ptr(jd_ptr), _ptr(jd_col), _ptr(jd_val),
                                _ptr(x), _ptr(y)))
    return y


def lilac_spmv_batched(handles: Sequence["Csr"], xs, ys, stream=None):
    n = len(handles)
    H = (ctypes.c_void_p * n)(*[h.handle for h in handles])
    X = (ctypes.c_void_p * n)(*[_ptr(x) for x in xs])
    Y = (ctypes.c_void_p * n)(*[_ptr(y) for y in ys])
    _check(lib().lilac_spmv_batched(n, ctypes.cast(H, _P), ctypes.cast(X, _P),
                                    ctypes.cast(Y, _P), _stream(stream)))


def lilac_tune_clear() -> None:
    """Forgets the tuned plans held in memory; new handles start from the
    default plan."""
    _check(lib().lilac_tune_clear())


def lilac_spmv_batched_tune(handles: Sequence["Csr"], xs, ys) -> float:
    """Tunes the batch's layouts class by class on the batched call itself;
    returns the time (ms) of one batched call with the chosen plans."""
    n = len(handles)
    H = (ctypes.c_void_p * n)(*[h.handle for h in handles])
    X = (ctypes.c_void_p * n)(*[_ptr(x) for x in xs])
    Y = (ctypes.c_void_p * n)(*[_ptr(y) for y in ys])
    ms = ctypes.c_double(0.0)
    _check(lib().lilac_spmv_batched_tune(n, ctypes.cast(H, _P), ctypes.cast(X, _P),
                                         ctypes.cast(Y, _P), ctypes.addressof(ms)))
    return ms.value


# ------------------------------------------------------------ handle

class Csr:
    """Device-resident CSR matrix (lilac_csr_create ... lilac_csr_destroy)."""

    def __init__(self, row_ptr, col_idx, vals, cols: int = -1,
                 flags: int = 0):
        self._keep = None
        rp = _as_i32(row_ptr)
        ci = _as_i32(col_idx)
        if isinstance(vals, torch.Tensor):
            dt = F32 if vals.dtype == torch.float32 else F64
            if vals.dtype not in (torch.float32, torch.float64):
                raise TypeError("vals must be float32 or float64")
        else:
            vals = np.ascontiguousarray(vals)
            if vals.dtype not in (np.float32, np.float64):
                vals = vals.astype(np.float64)
            dt = F32 if vals.dtype == np.float32 else F64
        rows = (rp.numel() if isinstance(rp, torch.Tensor) else rp.size) - 1
        nnz = ci.numel() if isinstance(ci, torch.Tensor) else ci.size
        h = ctypes.c_void_p()
        if flags & KEEP_HOST:
            self._keep = (rp, ci, vals)
        _check(lib().lilac_csr_create(ctypes.byref(h), rows, cols, nnz, _ptr(rp),
                                      _ptr(ci), _ptr(vals), dt, flags))
        self.handle = h.value
        self.dtype = dt
        self.np_dtype = np.float32 if dt == F32 else np.float64
        self.torch_dtype = torch.float32 if dt == F32 else torch.float64
        inf = self.info()
        self.rows, self.cols, self.nnz = inf.rows, inf.cols, inf.nnz

    @classmethod
    def from_gen(cls, A, **kw):
        return cls(A.row_ptr, A.col_idx, A.vals, **kw)

    def info(self) -> CsrInfo:
        out = CsrInfo()
        _check(lib().lilac_csr_info(self.handle, ctypes.byref(out)))
        return out

    def analysis(self):
        """(bin_off, bin_rows, c_row, c_k0, c_k1) as numpy int32 arrays."""
        inf = self.info()
        off = np.empty(NCLASS + 1, dtype=np.int32)
        br = np.empty(max(inf.rows, 1), dtype=np.int32)
        m = max(inf.nchunks, 1)
        cr = np.empty(m, dtype=np.int32)
        c0 = np.empty(m, dtype=np.int32)
        c1 = np.empty(m, dtype=np.int32)
        _check(lib().lilac_csr_analysis(self.handle, _ptr(off), _ptr(br), _ptr(cr),
                                        _ptr(c0), _ptr(c1)))
        k = inf.nchunks
        return off, br[:inf.rows], cr[:k], c0[:k], c1[:k]

    def upper(self) -> np.ndarray:
        inf = self.info()
        return np.array(inf.bin_upper[:NCLASS], dtype=np.int32)

    def set_plan(self, upper=None, rows_per_group=None, chunk: int = 0):
        up = None if upper is None else np.ascontiguousarray(upper, dtype=np.int32)
        rg = None if rows_per_group is None else \
            np.ascontiguousarray(rows_per_group, dtype=np.int32)
        _check(lib().lilac_csr_set_plan(self.handle, _ptr(up), _ptr(rg), chunk))

    def set_layout(self, layout: int):
        """LAYOUT_AUTO (-1), LAYOUT_ROWS (0), LAYOUT_PANELS (1), LAYOUT_HOT (2) or
        LAYOUT_BAND (3)."""
        _check(lib().lilac_csr_set_layout(self.handle, layout))

    def spmv(self, x, y, stream=None):
        _check(lib().lilac_spmv(self.handle, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def spmv_dot(self, x, y, w, out, stream=None):
        _check(lib().lilac_spmv_dot(self.handle, _ptr(x), _ptr(y), _ptr(w),
                                    _ptr(out), _stream(stream)))

    def update_values(self, vals):
        _check(lib().lilac_csr_update_values(self.handle, _ptr(vals)))
        if self._keep is not None:
            self._keep = (self._keep[0], self._keep[1], vals)

    def invalidate(self):
        _check(lib().lilac_csr_invalidate(self.handle))

    def cg(self, b, x, iters: int, graph: bool = True, stream=None,
           want_result: bool = False):
        rho = ctypes.c_double(0.0)
        it = ctypes.c_int(0)
        _check(lib().lilac_cg(self.handle, _ptr(b), _ptr(x), iters,
                              CG_GRAPH if graph else 0, _stream(stream),
                              ctypes.addressof(rho) if want_result else None,
                              ctypes.addressof(it) if want_result else None))
        return (rho.value, it.value) if want_result else None

    def cg_noalloc(self, b, x, iters: int, stream=None):
        """CG with the solver state in the library's fixed device array (no
        allocation); async."""
        _check(lib().lilac_cg_noalloc(self.handle, _ptr(b), _ptr(x), iters,
                                      _stream(stream)))

    def pagerank(self, damping: float, iters: int, x, stream=None):
        _check(lib().lilac_pagerank(self.handle, float(damping), iters, _ptr(x),
                                    _stream(stream)))
        return x

    def bfs(self, source: int, level, stream=None) -> int:
        """Fills the device int32 tensor `level`; returns the level count."""
        n = ctypes.c_int(0)
        _check(lib().lilac_bfs(self.handle, source, _ptr(level),
                               ctypes.addressof(n), _stream(stream)))
        return n.value

    def to_jds(self, stream=None) -> dict:
        """JDS arrays of the matrix as device tensors: perm, nzcnt, jd_ptr,
        col_ind (int32) and val (the handle's dtype), plus max_len."""
        ml = ctypes.c_int(0)
        _check(lib().lilac_csr_to_jds(self.handle, None, None, None, 0, None, None,
                                      ctypes.addressof(ml), _stream(stream)))
        i32 = dict(dtype=torch.int32, device="cuda")
        out = dict(perm=torch.empty(max(self.rows, 1), **i32),
                   nzcnt=torch.empty(max(self.rows, 1), **i32),
                   jd_ptr=torch.empty(ml.value + 1, **i32),
                   col_ind=torch.empty(max(self.nnz, 1), **i32),
                   val=torch.empty(max(self.nnz, 1), dtype=self.torch_dtype,
                                   device="cuda"))
        _check(lib().lilac_csr_to_jds(self.handle, _ptr(out["perm"]), _ptr(out["nzcnt"]),
                                      _ptr(out["jd_ptr"]), ml.value + 1,
                                      _ptr(out["col_ind"]), _ptr(out["val"]),
                                      ctypes.addressof(ml), _stream(stream)))
        for k in ("perm", "nzcnt"):
            out[k] = out[k][:self.rows]
        for k in ("col_ind", "val"):
            out[k] = out[k][:self.nnz]
        out["max_len"] = ml.value
        return out

    def tune_class(self) -> str:
        buf = ctypes.create_string_buffer(96)
        _check(lib().lilac_csr_tune_class(self.handle, buf, 96))
        return buf.value.decode()

    def tune(self) -> float:
        us = ctypes.c_double(0.0)
        _check(lib().lilac_csr_tune(self.handle, ctypes.addressof(us)))
        return us.value

    def destroy(self):
        if getattr(self, "handle", None):
            _check(lib().lilac_csr_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.lilac_csr_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


class Csr64:
    """CSR matrix with int64 row offsets (lilac_csr64_create ...
    lilac_csr64_destroy): consecutive row parts, each an ordinary handle."""

    def __init__(self, row_ptr, col_idx, vals, cols: int = -1):
        if isinstance(row_ptr, torch.Tensor):
            if row_ptr.dtype != torch.int64:
                raise TypeError("row_ptr must be int64")
            rp = row_ptr
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = _as_i32(col_idx)
        if isinstance(vals, torch.Tensor):
            if vals.dtype not in (torch.float32, torch.float64):
                raise TypeError("vals must be float32 or float64")
            dt = F32 if vals.dtype == torch.float32 else F64
        else:
            vals = np.ascontiguousarray(vals)
            if vals.dtype not in (np.float32, np.float64):
                vals = vals.astype(np.float64)
            dt = F32 if vals.dtype == np.float32 else F64
        rows = (rp.numel() if isinstance(rp, torch.Tensor) else rp.size) - 1
        nnz = ci.numel() if isinstance(ci, torch.Tensor) else ci.size
        h = ctypes.c_void_p()
        _check(lib().lilac_csr64_create(ctypes.byref(h), rows, cols, nnz, _ptr(rp),
                                        _ptr(ci), _ptr(vals), dt))
        self.handle = h.value
        self.dtype = dt
        self.rows, self.cols, self.nnz, self.nparts = self.info()

    @classmethod
    def from_gen(cls, A, **kw):
        return cls(A.row_ptr, A.col_idx, A.vals, **kw)

    def info(self):
        """(rows, cols, nnz, nparts)."""
        r, c, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        z = ctypes.c_int64()
        _check(lib().lilac_csr64_info(self.handle, ctypes.byref(r), ctypes.byref(c),
                                      ctypes.byref(z), ctypes.byref(p)))
        return r.value, c.value, z.value, p.value

    def spmv(self, x, y, stream=None):
        _check(lib().lilac_csr64_spmv(self.handle, _ptr(x), _ptr(y), _stream(stream)))

    def destroy(self):
        if getattr(self, "handle", None):
            _check(lib().lilac_csr64_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.lilac_csr64_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


# ------------------------------------------------------------ request server

class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("max_active", ctypes.c_int),
                ("pool_capacity", ctypes.c_int), ("fifo", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("matrix", ctypes.c_int),
                ("iters", ctypes.c_int), ("in_", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("arrival_ns", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("spmv_done", ctypes.c_int64),
                ("cg_done", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("req_per_s", ctypes.c_double),
                ("solves_per_s", ctypes.c_double),
                ("gbytes_per_s", ctypes.c_double), ("uploads", ctypes.c_int64),
                ("evictions", ctypes.c_int64), ("ticks", ctypes.c_int64),
                ("peak_device_bytes", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("planned_peak_bytes", ctypes.c_int64),
                ("mean_wait_us", ctypes.c_double), ("mean_run_us", ctypes.c_double),
                ("waited_upload", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


REQ_SPMV, REQ_CG = 0, 1

_SIGS.update({
    "lilac_server_create": ([_P, ctypes.POINTER(ServerConfig)], _I),
    "lilac_server_add_matrix": ([_P, _I, _I, _I64, _P, _P, _P, ctypes.POINTER(_I)], _I),
    "lilac_server_submit": ([_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], _I),
    "lilac_server_poll": ([_P, ctypes.c_uint64, ctypes.POINTER(_I)], _I),
    "lilac_server_wait": ([_P, ctypes.c_uint64], _I),
    "lilac_server_now": ([_P, ctypes.POINTER(_I64)], _I),
    "lilac_server_stats_get": ([_P, ctypes.POINTER(ServerStats)], _I),
    "lilac_server_reset_stats": ([_P], _I),
    "lilac_server_run_trace": ([_P, _I, _P, _P, _P, _I, ctypes.POINTER(ServerStats)], _I),
    "lilac_server_destroy": ([_P], _I),
})


class Server:
    """lilac_server_* wrapper.  Host matrices passed to add_matrix are kept
    alive by this object."""

    def __init__(self, hbm_budget: int = 0, max_active: int = 0,
                 pool_capacity: int = 0, fifo: bool = False):
        cfg = ServerConfig(hbm_budget, max_active, pool_capacity, int(fifo))
        h = ctypes.c_void_p()
        _check(lib().lilac_server_create(ctypes.byref(h), ctypes.byref(cfg)))
        self.handle = h.value
        self._keep = []

    def add_matrix(self, A) -> int:
        rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
        v = np.ascontiguousarray(A.vals, dtype=np.float64)
        self._keep.append((rp, ci, v))
        mid = ctypes.c_int(-1)
        _check(lib().lilac_server_add_matrix(self.handle, rp.size - 1, A.cols,
                                             ci.size, _ptr(rp), _ptr(ci), _ptr(v),
                                             ctypes.byref(mid)))
        return mid.value

    def submit(self, kind: int, matrix: int, inp, out, iters: int = 0,
               arrival_ns: int = 0) -> int:
        r = Request(kind, matrix, iters, _ptr(inp), _ptr(out), arrival_ns)
        t = ctypes.c_uint64(0)
        _check(lib().lilac_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> int:
        d = ctypes.c_int(0)
        _check(lib().lilac_server_poll(self.handle, ticket, ctypes.byref(d)))
        return d.value

    def wait(self, ticket: int):
        _check(lib().lilac_server_wait(self.handle, ticket))

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().lilac_server_stats_get(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def reset_stats(self):
        _check(lib().lilac_server_reset_stats(self.handle))

    def run_trace(self, arrival_ns, kind, matrix, cg_iters: int) -> dict:
        a = np.ascontiguousarray(arrival_ns, dtype=np.int64)
        k = np.ascontiguousarray(kind, dtype=np.int32)
        m = np.ascontiguousarray(matrix, dtype=np.int32)
        s = ServerStats()
        _check(lib().lilac_server_run_trace(self.handle, a.size, _ptr(a), _ptr(k),
                                            _ptr(m), cg_iters, ctypes.byref(s)))
        return s.as_dict()

    def destroy(self):
        if getattr(self, "handle", None):
            _check(lib().lilac_server_destroy(self.handle))
            self.handle = None


HEADER_FUNCTIONS = header_functions()

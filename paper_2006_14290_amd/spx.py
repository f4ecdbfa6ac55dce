"""Python binding of libspx.so (include/spx.h): argument marshalling only.

Device memory and streams come from PyTorch; every computation runs in the
library's HIP kernels. Importing this module loads libspx.so and raises if it
is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SPX_LIBRARY") or os.path.join(_HERE, "libspx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2006_14290_amd/build.py (or __graft_entry__.build())")
_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------------ enums
OK, ERR_ARG, ERR_FORMAT, ERR_UNSORTED, ERR_DUPLICATE, ERR_RANGE, ERR_NOMEM, ERR_BUDGET, ERR_HIP, \
    ERR_ZERO_DIAG, ERR_NOT_CONVERGED, ERR_BREAKDOWN, ERR_NONFINITE, PENDING, CANCELLED = range(15)
F64, F32, F16 = 0, 1, 2
CSR, COO, ELL, HYB, SELLP = 0, 1, 2, 3, 4

_VAL_DTYPE = {F64: torch.float64, F32: torch.float32, F16: torch.float16}
_VEC_DTYPE = {F64: torch.float64, F32: torch.float32, F16: torch.float32}
DTYPE_NAMES = {"f64": F64, "f32": F32, "f16": F16}


class SpxError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        name = _lib.spx_status_string(status).decode()
        detail = _lib.spx_last_error().decode()
        super().__init__(f"{where}: {name}: {detail}")


class MatrixDesc(ctypes.Structure):
    _fields_ = [
        ("fmt", ctypes.c_int32), ("val_type", ctypes.c_int32), ("nrows", ctypes.c_int32),
        ("ncols", ctypes.c_int32), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
        ("rowidx", ctypes.c_void_p), ("colidx", ctypes.c_void_p), ("vals", ctypes.c_void_p),
        ("coo_nnz", ctypes.c_int64), ("ell_width", ctypes.c_int32), ("max_row_len", ctypes.c_int32),
        ("ell_ld", ctypes.c_int64), ("ell_col", ctypes.c_void_p), ("ell_val", ctypes.c_void_p),
        ("csr_part", ctypes.c_void_p), ("slice_size", ctypes.c_int32), ("stride_factor", ctypes.c_int32),
        ("slice_sets", ctypes.c_void_p), ("slice_cols", ctypes.c_int64),
        ("csr_cb", ctypes.c_void_p), ("csr_cb_tiles", ctypes.c_int32), ("csr_cb_live", ctypes.c_int32),
    ]


_vp, _i32, _i64, _f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_MP = ctypes.POINTER(MatrixDesc)


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("spx_status_string", [ctypes.c_int], ctypes.c_char_p)
_sig("spx_last_error", [], ctypes.c_char_p)
_sig("spx_version", [], ctypes.c_int32)
_sig("spx_validate", [_MP, _vp])
_sig("spx_validate_csr_host", [_i32, _i32, _i64, _vp, _vp])
_sig("spx_spmv", [_MP, _vp, _vp, _f64, _f64, _vp])
_sig("spx_csr_spmv", [_MP, _vp, _vp, _f64, _f64, _vp])
_sig("spx_csr_analysis_bytes", [_MP], ctypes.c_int64)
_sig("spx_csr_analyse", [_MP, _vp, ctypes.c_size_t, _vp])
_sig("spx_csr_colblock_bytes", [_MP], ctypes.c_int64)
_sig("spx_csr_colblock", [_MP, _vp, ctypes.c_size_t, _vp])
_sig("spx_convert_plan", [_MP, _i32, _i32, _i64, _MP, ctypes.POINTER(ctypes.c_size_t), _vp])
_sig("spx_convert", [_MP, _MP, _vp, ctypes.c_size_t, _vp])
_sig("spx_cast_values", [_MP, _MP, _vp])
_sig("spx_csr_transpose_workspace", [_MP, ctypes.POINTER(ctypes.c_size_t)])
_sig("spx_csr_transpose", [_MP, _MP, _vp, ctypes.c_size_t, _vp])
class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("x0_zero", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("spmv_count", ctypes.c_int32),
                ("outer_iters", ctypes.c_int32), ("relres_recursive", ctypes.c_double),
                ("relres_true", ctypes.c_double), ("device_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class IrOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("inner_maxit", ctypes.c_int32), ("check_every", ctypes.c_int32), ("reserved", ctypes.c_int32)]


SOLVER_CG, SOLVER_BICGSTAB, SOLVER_GMRES, SOLVER_BICG, SOLVER_PIPECG = 0, 1, 2, 3, 4
_SOP = ctypes.POINTER(SolveOpts)
_SIP = ctypes.POINTER(SolveInfo)
_sig("spx_solve_workspace", [_i32, _MP, _SOP, ctypes.POINTER(ctypes.c_size_t)])
for _nm in ("spx_cg_solve", "spx_bicgstab_solve", "spx_gmres_solve", "spx_bicg_solve", "spx_pipecg_solve"):
    _sig(_nm, [_MP, _vp, _vp, _SOP, _vp, ctypes.c_size_t, _SIP, _vp])
_sig("spx_ir_workspace", [_MP, _MP, ctypes.POINTER(ctypes.c_size_t)])
_sig("spx_ir_solve", [_MP, _MP, _vp, _vp, ctypes.POINTER(IrOpts), _vp, ctypes.c_size_t, _SIP, _vp])
class BatchSystem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("path", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colidx", ctypes.c_void_p), ("vals", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("x", ctypes.c_void_p), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int32), ("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("spmv_count", ctypes.c_int32), ("relres_true", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_slots", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_size_t),
                ("iters_per_tick", ctypes.c_int32), ("tick_us", ctypes.c_int32), ("wide_min_rows", ctypes.c_int32),
                ("debug_fail_tick", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("inflight_bytes", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("solver", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colidx", ctypes.c_void_p), ("vals", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("x_out", ctypes.c_void_p), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("active", ctypes.c_int64), ("rejected", ctypes.c_int64), ("ticks", ctypes.c_int64),
                ("pool_bytes_total", ctypes.c_size_t), ("pool_bytes_in_use", ctypes.c_size_t),
                ("pool_bytes_peak", ctypes.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_sig("spx_cg_batch_workspace", [ctypes.POINTER(BatchSystem), _i32, ctypes.POINTER(ctypes.c_size_t)])
_sig("spx_cg_batch", [ctypes.POINTER(BatchSystem), _i32, _vp, ctypes.c_size_t, _vp])
_sig("spx_cg_batch_noalloc", [ctypes.POINTER(BatchSystem), _i32, _vp])
_sig("spx_server_create", [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)])
_sig("spx_serve_submit", [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)])
_sig("spx_serve_poll", [_vp, ctypes.c_uint64, _SIP])
_sig("spx_serve_wait", [_vp, ctypes.c_uint64, ctypes.c_double, _SIP])
_sig("spx_serve_cancel", [_vp, ctypes.c_uint64])
_sig("spx_server_get_stats", [_vp, ctypes.POINTER(ServerStats)])
_sig("spx_server_destroy", [_vp])
_sig("spx_subwarp_sum", [_vp, _vp, _i64, _i32, _i32, _vp])
_sig("spx_subwarp_vote", [_vp, _vp, _vp, _vp, _i64, _i32, _vp])
_sig("spx_wave_segscan", [_vp, _vp, _vp, _i64, _vp])
_sig("spx_stream_copy", [_vp, _vp, _i64, _vp])
_sig("spx_stream_read", [_vp, _i64, _vp, _vp])


def check(status: int, where: str):
    if status != OK:
        raise SpxError(status, where)


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("spx works on device tensors")
    if not t.is_contiguous():
        raise ValueError("spx needs contiguous tensors")
    return t.data_ptr() if t.numel() > 0 else None


# ------------------------------------------------------------------ matrices
@dataclass
class Matrix:
    """A device sparse matrix: torch tensors plus the C descriptor."""

    fmt: int
    dtype: int
    nrows: int
    ncols: int
    nnz: int
    rowptr: Optional[torch.Tensor] = None
    rowidx: Optional[torch.Tensor] = None
    colidx: Optional[torch.Tensor] = None
    vals: Optional[torch.Tensor] = None
    coo_nnz: int = 0
    ell_width: int = 0
    ell_ld: int = 0
    ell_col: Optional[torch.Tensor] = None
    ell_val: Optional[torch.Tensor] = None
    max_row_len: int = 0
    csr_part: Optional[torch.Tensor] = None
    slice_size: int = 0
    stride_factor: int = 0
    slice_sets: Optional[torch.Tensor] = None
    slice_cols: int = 0
    csr_cb: Optional[torch.Tensor] = None
    csr_cb_tiles: int = 0
    csr_cb_live: int = 0
    _desc: MatrixDesc = field(default=None, repr=False)

    def desc(self) -> MatrixDesc:
        d = MatrixDesc()
        d.fmt, d.val_type, d.nrows, d.ncols, d.nnz = self.fmt, self.dtype, self.nrows, self.ncols, self.nnz
        d.rowptr, d.rowidx, d.colidx, d.vals = (_ptr(self.rowptr), _ptr(self.rowidx), _ptr(self.colidx),
                                                _ptr(self.vals))
        d.coo_nnz, d.ell_width, d.max_row_len, d.ell_ld = self.coo_nnz, self.ell_width, self.max_row_len, self.ell_ld
        d.ell_col, d.ell_val = _ptr(self.ell_col), _ptr(self.ell_val)
        d.csr_part = _ptr(self.csr_part)
        d.slice_size, d.stride_factor, d.slice_cols = self.slice_size, self.stride_factor, self.slice_cols
        d.slice_sets = _ptr(self.slice_sets)
        d.csr_cb, d.csr_cb_tiles, d.csr_cb_live = _ptr(self.csr_cb), self.csr_cb_tiles, self.csr_cb_live
        self._desc = d
        return d

    @property
    def vec_dtype(self):
        return _VEC_DTYPE[self.dtype]

    def nbytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in
                   (self.rowptr, self.rowidx, self.colidx, self.vals, self.ell_col, self.ell_val, self.slice_sets)
                   if t is not None)


def _dev_vals(vals: np.ndarray, dtype: int, device) -> torch.Tensor:
    """Host float64 values stored as dtype on the device: uploaded in float64
    and rounded (nearest even) on the device by spx_cast_values."""
    v = torch.from_numpy(np.ascontiguousarray(vals, dtype=np.float64)).to(device)
    if dtype == F64 or v.numel() == 0:
        return v if dtype == F64 else v.to(_VAL_DTYPE[dtype])
    out = torch.empty(v.numel(), dtype=_VAL_DTYPE[dtype], device=v.device)
    # a one-row CSR descriptor over the value array: the cast reads only the
    # values (the column-index pointer is a placeholder it never follows)
    rp = torch.tensor([0, v.numel()], dtype=torch.int32, device=v.device)
    src = Matrix(CSR, F64, 1, 1, v.numel(), rowptr=rp, colidx=rp, vals=v)
    dst = Matrix(CSR, dtype, 1, 1, v.numel(), rowptr=rp, colidx=rp, vals=out)
    st = _lib.spx_cast_values(ctypes.byref(src.desc()), ctypes.byref(dst.desc()), _stream(None))
    if st not in (OK, ERR_RANGE):  # ERR_RANGE: finite values beyond binary16, written as infinities
        check(st, "spx_cast_values")
    return out


def csr_from_host(A, dtype: int = F64, device="cuda") -> Matrix:
    """Upload a host CSR (rowptr/col/val numpy arrays) as a device Matrix."""
    lens = np.diff(A.rowptr.astype(np.int64))
    return Matrix(CSR, dtype, int(A.n), int(A.n), int(A.rowptr[-1]),
                  rowptr=torch.from_numpy(np.ascontiguousarray(A.rowptr, np.int32)).to(device),
                  colidx=torch.from_numpy(np.ascontiguousarray(A.col, np.int32)).to(device),
                  vals=_dev_vals(A.val, dtype, device),
                  max_row_len=int(lens.max()) if lens.size else 0)


def coo_from_host(n, row, col, val, dtype: int = F64, device="cuda") -> Matrix:
    return Matrix(COO, dtype, int(n), int(n), int(len(row)),
                  rowidx=torch.from_numpy(np.ascontiguousarray(row, np.int32)).to(device),
                  colidx=torch.from_numpy(np.ascontiguousarray(col, np.int32)).to(device),
                  vals=_dev_vals(val, dtype, device))


def ell_from_host(n, K, ld, ecol, eval_, dtype: int = F64, device="cuda") -> Matrix:
    ecol = np.ascontiguousarray(ecol, np.int32)
    return Matrix(ELL, dtype, int(n), int(n), int((ecol != -1).sum()), ell_width=int(K), ell_ld=int(ld),
                  ell_col=torch.from_numpy(ecol).to(device), ell_val=_dev_vals(eval_, dtype, device))


def sellp_from_host(n, C, T, slice_sets, scol, sval, dtype: int = F64, device="cuda") -> Matrix:
    """Upload a host SELL-P matrix (slice size C, stride factor T)."""
    scol = np.ascontiguousarray(scol, np.int32)
    sets = np.ascontiguousarray(slice_sets, np.int32)
    return Matrix(SELLP, dtype, int(n), int(n), int((scol != -1).sum()), slice_size=int(C), stride_factor=int(T),
                  slice_sets=torch.from_numpy(sets).to(device), slice_cols=int(sets[-1]),
                  ell_col=torch.from_numpy(scol).to(device), ell_val=_dev_vals(sval, dtype, device))


def hyb_from_host(n, K, ld, ecol, eval_, row, col, val, dtype: int = F64, device="cuda") -> Matrix:
    ecol = np.ascontiguousarray(ecol, np.int32)
    return Matrix(HYB, dtype, int(n), int(n), int((ecol != -1).sum()) + int(len(row)), ell_width=int(K),
                  ell_ld=int(ld), ell_col=torch.from_numpy(ecol).to(device), ell_val=_dev_vals(eval_, dtype, device),
                  coo_nnz=int(len(row)),
                  rowidx=torch.from_numpy(np.ascontiguousarray(row, np.int32)).to(device),
                  colidx=torch.from_numpy(np.ascontiguousarray(col, np.int32)).to(device),
                  vals=_dev_vals(val, dtype, device))


def csr_analyse(A: Matrix, stream=None) -> Matrix:
    """Compute the CSR partition once (stored in A.csr_part, reused by every
    later product on A)."""
    d = A.desc()
    nbytes = _lib.spx_csr_analysis_bytes(ctypes.byref(d))
    buf = torch.empty(max(1, nbytes // 4), dtype=torch.int32, device=A.rowptr.device)
    check(_lib.spx_csr_analyse(ctypes.byref(d), _ptr(buf), nbytes, _stream(stream)), "spx_csr_analyse")
    A.csr_part = buf
    return A


def csr_colblock(A: Matrix, stream=None) -> Matrix:
    """Build A's column-blocked copy (8 column ranges, one per XCD; blocking).
    Later products on A through spmv/csr_spmv use it."""
    d = A.desc()
    nbytes = int(_lib.spx_csr_colblock_bytes(ctypes.byref(d)))
    device = A.rowptr.device if A.rowptr is not None else torch.device("cuda", torch.cuda.current_device())
    buf = torch.empty(max(256, nbytes), dtype=torch.uint8, device=device)
    check(_lib.spx_csr_colblock(ctypes.byref(d), _ptr(buf), buf.numel(), _stream(stream)), "spx_csr_colblock")
    A.csr_cb, A.csr_cb_tiles, A.csr_cb_live = buf, d.csr_cb_tiles, d.csr_cb_live
    return A


# ------------------------------------------------------------------ conversion
def convert(A: Matrix, fmt: int, ell_width: int = -1, ell_ld: int = 0, slice_size: int = 0,
            stride_factor: int = 0, stream=None) -> Matrix:
    """Convert A to `fmt` on the device (plan: blocking size query; then an
    asynchronous conversion into freshly allocated tensors). slice_size and
    stride_factor apply to SELLP (0 = 64 and 1)."""
    src = A.desc()
    shape = MatrixDesc()
    shape.slice_size, shape.stride_factor = slice_size, stride_factor
    ws = ctypes.c_size_t(0)
    check(_lib.spx_convert_plan(ctypes.byref(src), fmt, ell_width, ell_ld, ctypes.byref(shape), ctypes.byref(ws),
                                _stream(stream)), "spx_convert_plan")
    dev = next(t for t in (A.rowptr, A.ell_col, A.colidx, A.slice_sets) if t is not None).device
    vt = _VAL_DTYPE[A.dtype]
    i32 = dict(dtype=torch.int32, device=dev)
    out = Matrix(fmt, A.dtype, shape.nrows, shape.ncols, shape.nnz, coo_nnz=shape.coo_nnz,
                 ell_width=shape.ell_width, ell_ld=shape.ell_ld, slice_size=shape.slice_size,
                 stride_factor=shape.stride_factor, slice_cols=shape.slice_cols)
    if fmt == CSR:
        out.rowptr = torch.empty(shape.nrows + 1, **i32)
        out.colidx = torch.empty(shape.nnz, **i32)
        out.vals = torch.empty(shape.nnz, dtype=vt, device=dev)
    elif fmt == COO:
        out.rowidx = torch.empty(shape.nnz, **i32)
        out.colidx = torch.empty(shape.nnz, **i32)
        out.vals = torch.empty(shape.nnz, dtype=vt, device=dev)
    elif fmt == SELLP:
        ns = -(-shape.nrows // shape.slice_size)
        out.slice_sets = torch.empty(ns + 1, **i32)
        out.ell_col = torch.empty(shape.slice_cols * shape.slice_size, **i32)
        out.ell_val = torch.empty(shape.slice_cols * shape.slice_size, dtype=vt, device=dev)
    else:
        out.ell_col = torch.empty(shape.ell_width * shape.ell_ld, **i32)
        out.ell_val = torch.empty(shape.ell_width * shape.ell_ld, dtype=vt, device=dev)
        if fmt == HYB:
            out.rowidx = torch.empty(shape.coo_nnz, **i32)
            out.colidx = torch.empty(shape.coo_nnz, **i32)
            out.vals = torch.empty(shape.coo_nnz, dtype=vt, device=dev)
    wst = torch.empty(max(1, ws.value), dtype=torch.uint8, device=dev)
    check(_lib.spx_convert(ctypes.byref(A.desc()), ctypes.byref(out.desc()), _ptr(wst), ws.value, _stream(stream)),
          "spx_convert")
    out._ws = wst  # keep the workspace alive until the stream has consumed it
    return out


def cast_values(A: Matrix, dtype: int, stream=None) -> Matrix:
    """Copy of A (sharing its index arrays) with values rounded to dtype."""
    out = Matrix(A.fmt, dtype, A.nrows, A.ncols, A.nnz, rowptr=A.rowptr, rowidx=A.rowidx, colidx=A.colidx,
                 coo_nnz=A.coo_nnz, ell_width=A.ell_width, ell_ld=A.ell_ld, ell_col=A.ell_col,
                 max_row_len=A.max_row_len, csr_part=A.csr_part, slice_size=A.slice_size,
                 stride_factor=A.stride_factor, slice_sets=A.slice_sets, slice_cols=A.slice_cols)
    vt = _VAL_DTYPE[dtype]
    if A.vals is not None:
        out.vals = torch.empty(A.vals.numel(), dtype=vt, device=A.vals.device)
    if A.ell_val is not None:
        out.ell_val = torch.empty(A.ell_val.numel(), dtype=vt, device=A.ell_val.device)
    check(_lib.spx_cast_values(ctypes.byref(A.desc()), ctypes.byref(out.desc()), _stream(stream)), "spx_cast_values")
    return out


# ------------------------------------------------------------------ validation
def validate(A: Matrix, stream=None) -> int:
    """Canonical-form check of A's index arrays on the device (blocking).
    Returns the status code (OK, ERR_FORMAT, ERR_RANGE, ERR_UNSORTED or
    ERR_DUPLICATE); raises SpxError for argument and HIP errors."""
    st = _lib.spx_validate(ctypes.byref(A.desc()), _stream(stream))
    if st not in (OK, ERR_FORMAT, ERR_RANGE, ERR_UNSORTED, ERR_DUPLICATE):
        raise SpxError(st, "spx_validate")
    return st


def validate_csr_host(nrows: int, ncols: int, rowptr: np.ndarray, col: np.ndarray, nnz: Optional[int] = None) -> int:
    """The CSR checks of validate() on host arrays (no device involved);
    nnz defaults to len(col)."""
    rp = np.ascontiguousarray(rowptr, np.int32)
    c = np.ascontiguousarray(col, np.int32)
    if rp.size != nrows + 1:
        raise ValueError("rowptr must have nrows + 1 entries")
    nnz = c.size if nnz is None else int(nnz)
    if nnz > c.size:
        raise ValueError("nnz exceeds the column array")
    return _lib.spx_validate_csr_host(int(nrows), int(ncols), nnz, rp.ctypes.data, c.ctypes.data if c.size else None)


def last_error() -> str:
    return _lib.spx_last_error().decode()


# ------------------------------------------------------------------ SpMV
def spmv(A: Matrix, x: torch.Tensor, y: Optional[torch.Tensor] = None, alpha: float = 1.0, beta: float = 0.0,
         stream=None, csr_only: bool = False) -> torch.Tensor:
    """y = alpha*A*x + beta*y on the device (asynchronous on the stream)."""
    if y is None:
        y = torch.empty(A.nrows, dtype=A.vec_dtype, device=x.device)
    for v, nm in ((x, "x"), (y, "y")):
        if v.dtype != A.vec_dtype:
            raise TypeError(f"{nm} must be {A.vec_dtype}")
    fn = _lib.spx_csr_spmv if csr_only else _lib.spx_spmv
    check(fn(ctypes.byref(A.desc()), _ptr(x), _ptr(y), float(alpha), float(beta), _stream(stream)),
          "spx_csr_spmv" if csr_only else "spx_spmv")
    return y


# ------------------------------------------------------------------ solvers
_SOLVER_FN = {SOLVER_CG: "spx_cg_solve", SOLVER_BICGSTAB: "spx_bicgstab_solve", SOLVER_GMRES: "spx_gmres_solve",
              SOLVER_BICG: "spx_bicg_solve", SOLVER_PIPECG: "spx_pipecg_solve"}
_ws_cache = {}


def _workspace(nbytes: int, device) -> torch.Tensor:
    """A reusable device workspace of at least nbytes (grown on demand)."""
    key = str(device)
    t = _ws_cache.get(key)
    if t is None or t.numel() < nbytes:
        t = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = t
    return t


def solve(solver: int, A: Matrix, b: torch.Tensor, x: Optional[torch.Tensor] = None, tol: float = 1e-10,
          maxit: int = 10000, precond: int = 0, restart: int = 30, check_every: int = 0, stream=None):
    """Solve A x = b on the device (blocking). Returns (x, info dict); raises
    SpxError on failure unless the failure is NOT_CONVERGED/BREAKDOWN, which
    are reported in info['status'] with x holding the last iterate."""
    opts = SolveOpts(tol, maxit, restart, precond, 1 if x is None else 0, check_every, 0)
    if x is None:
        x = torch.empty_like(b)
    d = A.desc()
    nbytes = ctypes.c_size_t(0)
    check(_lib.spx_solve_workspace(solver, ctypes.byref(d), ctypes.byref(opts), ctypes.byref(nbytes)),
          "spx_solve_workspace")
    ws = _workspace(nbytes.value, b.device)
    info = SolveInfo()
    st = getattr(_lib, _SOLVER_FN[solver])(ctypes.byref(d), _ptr(b), _ptr(x), ctypes.byref(opts), _ptr(ws),
                                             ws.numel(), ctypes.byref(info), _stream(stream))
    if st not in (OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN, ERR_NONFINITE):
        check(st, _SOLVER_FN[solver])
    out = info.as_dict()
    out["status"] = st
    out["error"] = _lib.spx_last_error().decode() if st != OK else ""
    return x, out


def cg_solve(A, b, x=None, **kw):
    return solve(SOLVER_CG, A, b, x, **kw)


def bicgstab_solve(A, b, x=None, **kw):
    return solve(SOLVER_BICGSTAB, A, b, x, **kw)


def gmres_solve(A, b, x=None, **kw):
    return solve(SOLVER_GMRES, A, b, x, **kw)


def bicg_solve(A, b, x=None, **kw):
    return solve(SOLVER_BICG, A, b, x, **kw)


def pipecg_solve(A, b, x=None, **kw):
    return solve(SOLVER_PIPECG, A, b, x, **kw)


def csr_transpose(A: Matrix, stream=None) -> Matrix:
    """A^T of a CSR matrix as a new device CSR matrix (asynchronous on stream)."""
    if A.fmt != CSR:
        raise SpxError(ERR_ARG, "csr_transpose: the matrix must be CSR")
    dev = A.rowptr.device
    At = Matrix(CSR, A.dtype, A.ncols, A.nrows, A.nnz,
                rowptr=torch.empty(A.ncols + 1, dtype=torch.int32, device=dev),
                colidx=torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev),
                vals=torch.empty(max(A.nnz, 1), dtype=A.vals.dtype, device=dev))
    d, dt = A.desc(), At.desc()
    nbytes = ctypes.c_size_t(0)
    check(_lib.spx_csr_transpose_workspace(ctypes.byref(d), ctypes.byref(nbytes)), "spx_csr_transpose_workspace")
    ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=dev)
    check(_lib.spx_csr_transpose(ctypes.byref(d), ctypes.byref(dt), _ptr(ws), ws.numel(), _stream(stream)),
          "spx_csr_transpose")
    At._ws = ws  # keep the workspace alive until the stream has used it
    return At


def ir_solve(A64: Matrix, Alow: Matrix, b: torch.Tensor, tol: float = 1e-10, inner_tol: float = 1e-3,
             max_outer: int = 50, inner_maxit: int = 20000, check_every: int = 0, stream=None):
    """Mixed-precision iterative refinement (blocking). Returns (x, info)."""
    x = torch.empty_like(b)
    opts = IrOpts(tol, inner_tol, max_outer, inner_maxit, check_every, 0)
    d64, dlo = A64.desc(), Alow.desc()
    nbytes = ctypes.c_size_t(0)
    check(_lib.spx_ir_workspace(ctypes.byref(d64), ctypes.byref(dlo), ctypes.byref(nbytes)), "spx_ir_workspace")
    ws = _workspace(nbytes.value, b.device)
    info = SolveInfo()
    st = _lib.spx_ir_solve(ctypes.byref(d64), ctypes.byref(dlo), _ptr(b), _ptr(x), ctypes.byref(opts), _ptr(ws),
                           ws.numel(), ctypes.byref(info), _stream(stream))
    if st not in (OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN, ERR_NONFINITE):
        check(st, "spx_ir_solve")
    out = info.as_dict()
    out["status"] = st
    out["error"] = _lib.spx_last_error().decode() if st != OK else ""
    return x, out


# ------------------------------------------------------------------ batched CG and serving
BATCH_AUTO, BATCH_ONE_GROUP, BATCH_WIDE = 0, 1, 2


def cg_batch(mats, bs, tol=1e-8, maxit=100000, path=BATCH_AUTO, stream=None, noalloc=False):
    """Solve independent CSR systems (device Matrix objects, float64) together:
    one work-group per small system, the wide path for large ones (`path`
    forces one). noalloc=True calls spx_cg_batch_noalloc (the library's own
    fixed device scratch instead of a workspace). Returns (xs, infos)."""
    count = len(mats)
    arr = (BatchSystem * count)()
    xs = []
    for i, (A, b) in enumerate(zip(mats, bs)):
        x = torch.empty_like(b)
        xs.append(x)
        arr[i] = BatchSystem(A.nrows, path, A.nnz, _ptr(A.rowptr), _ptr(A.colidx), _ptr(A.vals), _ptr(b), _ptr(x),
                             tol, maxit, 0, 0, 0, 0.0)
    if noalloc:
        st = _lib.spx_cg_batch_noalloc(arr, count, _stream(stream))
    else:
        nbytes = ctypes.c_size_t(0)
        check(_lib.spx_cg_batch_workspace(arr, count, ctypes.byref(nbytes)), "spx_cg_batch_workspace")
        ws = _workspace(nbytes.value, bs[0].device)
        st = _lib.spx_cg_batch(arr, count, _ptr(ws), ws.numel(), _stream(stream))
    if st not in (OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN, ERR_NONFINITE):
        check(st, "spx_cg_batch_noalloc" if noalloc else "spx_cg_batch")
    infos = [{"status": arr[i].status, "iters": arr[i].iters, "spmv_count": arr[i].spmv_count,
              "relres_true": arr[i].relres_true} for i in range(count)]
    return xs, infos


class Server:
    """Continuous-batching CG / BiCGSTAB server (host requests, results copied
    back). inflight_bytes > 0: bound on the summed per-iteration bytes of the
    resident systems (strict FIFO past it); <= 0: no bound."""

    def __init__(self, device: int = 0, max_slots: int = 1024, hbm_budget_bytes: int = 32 << 30,
                 iters_per_tick: int = 0, tick_us: int = 0, wide_min_rows: int = 0, debug_fail_tick: int = 0,
                 inflight_bytes: int = 0):
        cfg = ServerConfig(device, max_slots, hbm_budget_bytes, iters_per_tick, tick_us, wide_min_rows,
                           debug_fail_tick, 0, inflight_bytes)
        h = ctypes.c_void_p()
        check(_lib.spx_server_create(ctypes.byref(cfg), ctypes.byref(h)), "spx_server_create")
        self._h = h
        self._keep = {}  # ticket -> host arrays kept alive until completion

    def submit(self, A, b: np.ndarray, tol: float = 1e-8, maxit: int = 0, x_out: Optional[np.ndarray] = None,
               solver: int = SOLVER_CG):
        """A: host CSR (rowptr/col/val numpy); solver SOLVER_CG (SPD) or
        SOLVER_BICGSTAB (nonsymmetric); returns the ticket."""
        rp = np.ascontiguousarray(A.rowptr, np.int32)
        ci = np.ascontiguousarray(A.col, np.int32)
        va = np.ascontiguousarray(A.val, np.float64)
        bb = np.ascontiguousarray(b, np.float64)
        x = np.empty(A.n, np.float64) if x_out is None else x_out
        req = Request(int(A.n), int(solver), int(rp[-1]), rp.ctypes.data, ci.ctypes.data, va.ctypes.data,
                      bb.ctypes.data, x.ctypes.data, tol, maxit, 0)
        t = ctypes.c_uint64(0)
        check(_lib.spx_serve_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "spx_serve_submit")
        self._keep[t.value] = (rp, ci, va, bb, x)
        return t.value

    def _result(self, ticket, st, info):
        out = info.as_dict()
        out["status"] = st
        x = self._keep.pop(ticket)[4] if st != PENDING else None
        return x, out

    def poll(self, ticket):
        info = SolveInfo()
        st = _lib.spx_serve_poll(self._h, ticket, ctypes.byref(info))
        if st == ERR_ARG:
            check(st, "spx_serve_poll")
        return self._result(ticket, st, info)

    def wait(self, ticket, timeout_s: float = -1.0):
        info = SolveInfo()
        st = _lib.spx_serve_wait(self._h, ticket, timeout_s, ctypes.byref(info))
        if st == ERR_ARG:
            check(st, "spx_serve_wait")
        return self._result(ticket, st, info)

    def cancel(self, ticket):
        check(_lib.spx_serve_cancel(self._h, ticket), "spx_serve_cancel")

    def stats(self):
        s = ServerStats()
        check(_lib.spx_server_get_stats(self._h, ctypes.byref(s)), "spx_server_get_stats")
        return s.as_dict()

    def close(self):
        if self._h:
            _lib.spx_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ primitives
def subwarp_sum(x: torch.Tensor, size: int, inner_loops: int = 1, out=None, stream=None) -> torch.Tensor:
    out = torch.empty_like(x) if out is None else out
    check(_lib.spx_subwarp_sum(_ptr(x), _ptr(out), x.numel(), size, inner_loops, _stream(stream)), "spx_subwarp_sum")
    return out


def subwarp_vote(pred: torch.Tensor, size: int, stream=None):
    n = pred.numel()
    ballot = torch.empty(n, dtype=torch.int64, device=pred.device)
    anyv = torch.empty(n, dtype=torch.int32, device=pred.device)
    allv = torch.empty(n, dtype=torch.int32, device=pred.device)
    check(_lib.spx_subwarp_vote(_ptr(pred), _ptr(ballot), _ptr(anyv), _ptr(allv), n, size, _stream(stream)),
          "spx_subwarp_vote")
    return ballot, anyv, allv


def wave_segscan(x: torch.Tensor, head: torch.Tensor, stream=None) -> torch.Tensor:
    out = torch.empty_like(x)
    check(_lib.spx_wave_segscan(_ptr(x), _ptr(head), _ptr(out), x.numel(), _stream(stream)), "spx_wave_segscan")
    return out


def stream_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    check(_lib.spx_stream_copy(_ptr(src), _ptr(dst), src.numel(), _stream(stream)), "spx_stream_copy")


def stream_read(src: torch.Tensor, sink: torch.Tensor, stream=None):
    check(_lib.spx_stream_read(_ptr(src), src.numel(), _ptr(sink), _stream(stream)), "spx_stream_read")


def version() -> int:
    return _lib.spx_version()

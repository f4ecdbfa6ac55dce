"""CPU oracle (TEST INFRASTRUCTURE ONLY).

Plain, sequential float64 reference implementations of what the library's GPU
path computes: sparse matrix-vector products in CSR/COO/ELL, format
conversions and the CSR transpose, value casts, scalar and block Jacobi
preconditioners, CG, pipelined CG, BiCG, BiCGSTAB, restarted GMRES and
mixed-precision iterative refinement. The arithmetic lives
in ``spx_oracle.c`` (plain C, compiled with gcc); this module only marshals
numpy arrays to it.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. It shares no code with the GPU library, and the GPU
library never calls it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spx_oracle.c")
_SRC_OMP = os.path.join(_HERE, "spx_oracle_omp.c")
_LIB = os.path.join(_HERE, "_spx_oracle.so")
# A differently built copy of the same sources (the sanitizer test builds one
# with AddressSanitizer/UBSan) may be loaded instead.
_LIB_OVERRIDE = os.environ.get("SPX_ORACLE_LIB")

# Status codes of the oracle's solvers.
OK, NOT_CONVERGED, BREAKDOWN, NONFINITE, ZERO_DIAG = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc. -ffp-contract=off keeps every float
    operation as written (the Dot2 error-free transformations rely on it)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
               "-fno-fast-math", "-Wall", "-Wno-unused-function", "-o", _LIB + ".tmp", _SRC, _SRC_OMP, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not _LIB_OVERRIDE and not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB_OVERRIDE or _LIB)
        _declare(_lib)
    return _lib


_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_i32, _i64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("spmv_count", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("relres_recursive", ctypes.c_double), ("relres_true", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _declare(L):
    L.orc_csr_spmv.argtypes = [_i32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64, _f64]
    L.orc_csr_spmv.restype = None
    L.orc_csr_spmv_dot2.argtypes = [_i32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64, _f64, ctypes.c_void_p]
    L.orc_csr_spmv_dot2.restype = None
    L.orc_coo_spmv.argtypes = [_i32, _i64, _i32p, _i32p, _f64p, _f64p, _f64p, _f64, _f64]
    L.orc_coo_spmv.restype = None
    L.orc_ell_spmv.argtypes = [_i32, _i32, _i64, _i32p, _f64p, _f64p, _f64p, _f64, _f64]
    L.orc_ell_spmv.restype = None
    L.orc_csr_check.argtypes = [_i32, _i32, _i32p, _i32p]
    L.orc_csr_to_coo.argtypes = [_i32, _i32p, _i32p]
    L.orc_csr_to_coo.restype = None
    L.orc_coo_to_csr.argtypes = [_i32, _i64, _i32p, _i32p]
    L.orc_max_row_length.argtypes = [_i32, _i32p]
    L.orc_csr_to_ell.argtypes = [_i32, _i32p, _i32p, _f64p, _i32, _i64, _i32p, _f64p]
    L.orc_ell_count.argtypes = [_i32, _i32, _i64, _i32p]
    L.orc_ell_count.restype = _i64
    L.orc_ell_to_csr.argtypes = [_i32, _i32, _i64, _i32p, _f64p, _i32p, _i32p, _f64p]
    L.orc_hyb_coo_count.argtypes = [_i32, _i32p, _i32]
    L.orc_hyb_coo_count.restype = _i64
    L.orc_csr_to_hyb.argtypes = [_i32, _i32p, _i32p, _f64p, _i32, _i64, _i32p, _f64p, _i32p, _i32p, _f64p]
    L.orc_hyb_to_csr.argtypes = [_i32, _i32, _i64, _i32p, _f64p, _i64, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p]
    L.orc_hyb_auto_width.argtypes = [_i32, _i32p, _i32, _i32]
    L.orc_sellp_shape.argtypes = [_i32, _i32p, _i32, _i32, _i32p]
    L.orc_csr_to_sellp.argtypes = [_i32, _i32p, _i32p, _f64p, _i32, _i32p, _i32p, _f64p]
    L.orc_sellp_spmv.argtypes = [_i32, _i32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64, _f64]
    L.orc_sellp_spmv.restype = None
    L.orc_sellp_count.argtypes = [_i32, _i32, _i32p, _i32p]
    L.orc_sellp_count.restype = _i64
    L.orc_sellp_to_csr.argtypes = [_i32, _i32, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p]
    L.orc_cast_values.argtypes = [_i64, _f64p, _i32, ctypes.c_void_p]
    L.orc_cast_values.restype = _i64
    L.orc_f16_to_f64.argtypes = [ctypes.c_uint16]
    L.orc_f16_to_f64.restype = _f64
    L.orc_residual.argtypes = [_i32, _i32p, _i32p, _f64p, _f64p, _f64p, ctypes.c_void_p]
    L.orc_residual.restype = _f64
    L.orc_jacobi_setup.argtypes = [_i32, _i32p, _i32p, _f64p, _f64p]
    L.orc_block_jacobi_setup.argtypes = [_i32, _i32p, _i32p, _f64p, _i32, _f64p]
    L.orc_block_jacobi_apply.argtypes = [_i32, _i32, _f64p, _f64p, _f64p]
    L.orc_block_jacobi_apply.restype = None
    solver = [_i32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64, _i32]
    L.orc_cg.argtypes = solver + [_i32, _i32, ctypes.POINTER(Info)]
    L.orc_cg_omp.argtypes = solver + [_i32, ctypes.POINTER(Info)]
    L.orc_csr_spmv_omp.argtypes = [_i32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64, _f64]
    L.orc_csr_spmv_omp.restype = None
    L.orc_omp_threads.restype = ctypes.c_int
    L.orc_bicgstab.argtypes = solver + [_i32, _i32, ctypes.POINTER(Info)]
    L.orc_gmres.argtypes = solver + [_i32, _i32, _i32, ctypes.POINTER(Info)]
    L.orc_bicg.argtypes = solver + [_i32, _i32, ctypes.c_void_p, _i32, ctypes.POINTER(Info)]
    L.orc_pipecg.argtypes = solver + [_i32, _i32, ctypes.POINTER(Info)]
    L.orc_csr_transpose.argtypes = [_i32, _i32, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p]
    L.orc_arnoldi.argtypes = [_i32, _i32p, _i32p, _f64p, _f64p, _i32, _i32, _f64p, _f64p]
    L.orc_ir.argtypes = [_i32, _i32p, _i32p, _f64p, _f32p, _f64p, _f64p, _f64, _f64, _i32, _i32,
                         ctypes.POINTER(Info)]


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _csr(A):
    return _c(A.rowptr, np.int32), _c(A.col, np.int32), _c(A.val, np.float64)


# ---------------------------------------------------------------- SpMV
def csr_spmv(A, x, y=None, alpha=1.0, beta=0.0):
    """Plain float64 y = alpha*A*x + beta*y (sequential row sums)."""
    rp, c, v = _csr(A)
    out = np.zeros(A.n) if y is None else _c(y, np.float64).copy()
    lib().orc_csr_spmv(A.n, rp, c, v, _c(x, np.float64), out, alpha, beta)
    return out


def csr_spmv_dot2(A, x, y=None, alpha=1.0, beta=0.0):
    """Dot2-accurate y = alpha*A*x + beta*y; returns (y, |A||x|)."""
    rp, c, v = _csr(A)
    out = np.zeros(A.n) if y is None else _c(y, np.float64).copy()
    absax = np.zeros(A.n)
    lib().orc_csr_spmv_dot2(A.n, rp, c, v, _c(x, np.float64), out, alpha, beta,
                            absax.ctypes.data_as(ctypes.c_void_p))
    return out, absax


def coo_spmv(n, row, col, val, x, y=None, alpha=1.0, beta=0.0):
    out = np.zeros(n) if y is None else _c(y, np.float64).copy()
    lib().orc_coo_spmv(n, len(row), _c(row, np.int32), _c(col, np.int32), _c(val, np.float64),
                       _c(x, np.float64), out, alpha, beta)
    return out


def ell_spmv(n, K, ld, ecol, eval_, x, y=None, alpha=1.0, beta=0.0):
    out = np.zeros(n) if y is None else _c(y, np.float64).copy()
    lib().orc_ell_spmv(n, K, ld, _c(ecol, np.int32), _c(eval_, np.float64), _c(x, np.float64),
                       out, alpha, beta)
    return out


# ---------------------------------------------------------------- formats
def csr_check(A, ncols=None):
    return lib().orc_csr_check(A.n, A.n if ncols is None else ncols, _c(A.rowptr, np.int32),
                               _c(A.col, np.int32))


def csr_to_coo_rows(A):
    row = np.empty(A.nnz, np.int32)
    lib().orc_csr_to_coo(A.n, _c(A.rowptr, np.int32), row)
    return row


def coo_to_csr_rowptr(n, row):
    rp = np.empty(n + 1, np.int32)
    st = lib().orc_coo_to_csr(n, len(row), _c(row, np.int32), rp)
    if st != 0:
        raise ValueError(f"coo_to_csr failed: {st}")
    return rp


def max_row_length(A):
    return lib().orc_max_row_length(A.n, _c(A.rowptr, np.int32))


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray


@dataclass
class Ell:
    n: int
    K: int
    ld: int
    col: np.ndarray
    val: np.ndarray


@dataclass
class Hyb:
    ell: Ell
    row: np.ndarray
    col: np.ndarray
    val: np.ndarray


def csr_to_ell(A, K=None, ld=None):
    K = max_row_length(A) if K is None else int(K)
    ld = A.n if ld is None else int(ld)
    ecol = np.empty(K * ld, np.int32)
    ev = np.empty(K * ld, np.float64)
    if ld > A.n:  # rows past n are not part of the matrix; mark them padding
        ecol[:] = -1
        ev[:] = 0.0
    rp, c, v = _csr(A)
    st = lib().orc_csr_to_ell(A.n, rp, c, v, K, ld, ecol, ev)
    if st != 0:
        raise ValueError(f"csr_to_ell failed: {st}")
    return Ell(A.n, K, ld, ecol, ev)


def ell_to_csr(E):
    cnt = lib().orc_ell_count(E.n, E.K, E.ld, _c(E.col, np.int32))
    rp = np.empty(E.n + 1, np.int32)
    col = np.empty(cnt, np.int32)
    val = np.empty(cnt, np.float64)
    st = lib().orc_ell_to_csr(E.n, E.K, E.ld, _c(E.col, np.int32), _c(E.val, np.float64), rp, col, val)
    if st != 0:
        raise ValueError(f"ell_to_csr failed: {st}")
    return CSR(E.n, rp, col, val)


@dataclass
class Sellp:
    n: int
    C: int  # slice size (rows per slice)
    T: int  # stride factor (slice widths are multiples of it)
    slice_sets: np.ndarray  # int32 [nslices + 1], prefix sums of slice widths
    col: np.ndarray  # int32 [slice_sets[-1] * C]
    val: np.ndarray  # float64


def csr_to_sellp(A, C=64, T=1):
    nslices = (A.n + C - 1) // C
    sets = np.empty(nslices + 1, np.int32)
    rp, c, v = _csr(A)
    st = lib().orc_sellp_shape(A.n, rp, C, T, sets)
    if st != 0:
        raise ValueError(f"sellp_shape failed: {st}")
    total = int(sets[-1]) * C
    scol = np.empty(total, np.int32)
    sval = np.empty(total, np.float64)
    st = lib().orc_csr_to_sellp(A.n, rp, c, v, C, sets, scol, sval)
    if st != 0:
        raise ValueError(f"csr_to_sellp failed: {st}")
    return Sellp(A.n, C, T, sets, scol, sval)


def sellp_spmv(P, x, y=None, alpha=1.0, beta=0.0):
    out = np.zeros(P.n) if y is None else _c(y, np.float64).copy()
    lib().orc_sellp_spmv(P.n, P.C, _c(P.slice_sets, np.int32), _c(P.col, np.int32), _c(P.val, np.float64),
                         _c(x, np.float64), out, alpha, beta)
    return out


def sellp_to_csr(P):
    sets, scol = _c(P.slice_sets, np.int32), _c(P.col, np.int32)
    cnt = lib().orc_sellp_count(P.n, P.C, sets, scol)
    if cnt < 0:
        raise ValueError(f"sellp_count failed: {cnt}")
    rp = np.empty(P.n + 1, np.int32)
    col = np.empty(cnt, np.int32)
    val = np.empty(cnt, np.float64)
    lib().orc_sellp_to_csr(P.n, P.C, sets, scol, _c(P.val, np.float64), rp, col, val)
    return CSR(P.n, rp, col, val)


def hyb_auto_width(A, sv=8, si=4):
    return lib().orc_hyb_auto_width(A.n, _c(A.rowptr, np.int32), sv, si)


def csr_to_hyb(A, K=None, ld=None, sv=8):
    K = hyb_auto_width(A, sv) if K is None else int(K)
    ld = A.n if ld is None else int(ld)
    rp, c, v = _csr(A)
    cn = lib().orc_hyb_coo_count(A.n, rp, K)
    ecol = np.full(K * ld, -1, np.int32)
    ev = np.zeros(K * ld, np.float64)
    crow = np.empty(cn, np.int32)
    ccol = np.empty(cn, np.int32)
    cval = np.empty(cn, np.float64)
    st = lib().orc_csr_to_hyb(A.n, rp, c, v, K, ld, ecol, ev, crow, ccol, cval)
    if st != 0:
        raise ValueError(f"csr_to_hyb failed: {st}")
    return Hyb(Ell(A.n, K, ld, ecol, ev), crow, ccol, cval)


def hyb_to_csr(H):
    E = H.ell
    cnt = lib().orc_ell_count(E.n, E.K, E.ld, _c(E.col, np.int32)) + len(H.row)
    rp = np.empty(E.n + 1, np.int32)
    col = np.empty(cnt, np.int32)
    val = np.empty(cnt, np.float64)
    st = lib().orc_hyb_to_csr(E.n, E.K, E.ld, _c(E.col, np.int32), _c(E.val, np.float64), len(H.row),
                              _c(H.row, np.int32), _c(H.col, np.int32), _c(H.val, np.float64), rp, col, val)
    if st != 0:
        raise ValueError(f"hyb_to_csr failed: {st}")
    return CSR(E.n, rp, col, val)


def cast_values(val, dtype):
    """Round-to-nearest-even cast of float64 values; returns (array, n_overflow).
    dtype is 'f32' or 'f16'."""
    v = _c(val, np.float64)
    if dtype == "f32":
        out = np.empty(v.size, np.float32)
        ov = lib().orc_cast_values(v.size, v, 1, out.ctypes.data_as(ctypes.c_void_p))
    elif dtype == "f16":
        out = np.empty(v.size, np.float16)
        ov = lib().orc_cast_values(v.size, v, 2, out.ctypes.data_as(ctypes.c_void_p))
    else:
        raise ValueError(dtype)
    return out, int(ov)


def f16_to_f64(h: int) -> float:
    return lib().orc_f16_to_f64(int(h))


# ---------------------------------------------------------------- solvers
def residual(A, b, x):
    """(r, ||r||_2) with r = b - A x, each row sum by Dot2."""
    rp, c, v = _csr(A)
    r = np.empty(A.n)
    nr = lib().orc_residual(A.n, rp, c, v, _c(b, np.float64), _c(x, np.float64),
                            r.ctypes.data_as(ctypes.c_void_p))
    return r, nr


def jacobi_diag(A):
    rp, c, v = _csr(A)
    d = np.empty(A.n)
    st = lib().orc_jacobi_setup(A.n, rp, c, v, d)
    return st, d


def _solve(fn, A, b, x0, extra):
    rp, c, v = _csr(A)
    x = np.zeros(A.n) if x0 is None else _c(x0, np.float64).copy()
    info = Info()
    fn(A.n, rp, c, v, _c(b, np.float64), x, *extra, ctypes.byref(info))
    return x, info.as_dict()


def block_jacobi(A, bs):
    """Inverted diagonal blocks (nblocks, bs, bs) of A, or raises on a
    singular block."""
    nb = -(-A.n // bs)
    inv = np.empty(max(nb, 1) * bs * bs, np.float64)
    rp, c, v = _csr(A)
    st = lib().orc_block_jacobi_setup(A.n, rp, c, v, bs, inv)
    if st != 0:
        raise ValueError(f"block_jacobi_setup failed: {st}")
    return inv[: nb * bs * bs].reshape(nb, bs, bs)


def block_jacobi_apply(inv, r):
    nb, bs, _ = inv.shape
    z = np.empty(len(r), np.float64)
    lib().orc_block_jacobi_apply(len(r), bs, _c(inv.ravel(), np.float64), _c(r, np.float64), z)
    return z


def cg(A, b, tol=1e-10, maxit=10000, precond=0, x0=None):
    """precond: 0 none, 1 scalar Jacobi, bs >= 2 block Jacobi (bs x bs blocks)."""
    return _solve(lib().orc_cg, A, b, x0, [tol, maxit, precond, 1 if x0 is None else 0])


def omp_threads() -> int:
    """Threads the all-core variants use (OMP_NUM_THREADS or the host's cores)."""
    return int(lib().orc_omp_threads())


def csr_spmv_omp(A, x, y=None, alpha=1.0, beta=0.0):
    """csr_spmv with rows shared among OpenMP threads (bitwise the same y)."""
    rp, c, v = _csr(A)
    out = np.zeros(A.n) if y is None else _c(y, np.float64).copy()
    lib().orc_csr_spmv_omp(A.n, rp, c, v, _c(x, np.float64), out, alpha, beta)
    return out


def cg_omp(A, b, tol=1e-10, maxit=10000, precond=0):
    """cg from x0 = 0 with every loop shared among OpenMP threads (precond 0
    or 1); iterates agree with cg's to rounding."""
    return _solve(lib().orc_cg_omp, A, b, None, [tol, maxit, precond])


def bicgstab(A, b, tol=1e-10, maxit=10000, precond=0, x0=None):
    return _solve(lib().orc_bicgstab, A, b, x0, [tol, maxit, precond, 1 if x0 is None else 0])


def bicg(A, b, tol=1e-10, maxit=10000, precond=0, x0=None, nhist=0):
    """Preconditioned BiCG (precond 0 none, 1 scalar Jacobi). With nhist > 0
    also returns the residuals r_k and shadow residuals rt_k at the start of
    the first nhist iterations, as two (nhist, n) arrays."""
    hist = np.zeros((max(nhist, 1), 2, A.n))
    x, info = _solve(lib().orc_bicg, A, b, x0,
                     [tol, maxit, precond, 1 if x0 is None else 0,
                      hist.ctypes.data_as(ctypes.c_void_p) if nhist > 0 else None, nhist])
    if nhist > 0:
        return x, info, hist[:, 0, :].copy(), hist[:, 1, :].copy()
    return x, info


def pipecg(A, b, tol=1e-10, maxit=10000, precond=0, x0=None):
    """Pipelined preconditioned CG (precond 0 none, 1 scalar Jacobi)."""
    return _solve(lib().orc_pipecg, A, b, x0, [tol, maxit, precond, 1 if x0 is None else 0])


def csr_transpose(A, ncols=None):
    """Transpose of A (n rows, ncols columns, default square): returns
    (rowptr_t [ncols+1], col_t, val_t)."""
    nc = A.n if ncols is None else ncols
    rp, c, v = _csr(A)
    rpt = np.empty(nc + 1, np.int32)
    ct = np.empty(max(A.nnz, 1), np.int32)
    vt = np.empty(max(A.nnz, 1), np.float64)
    st = lib().orc_csr_transpose(A.n, nc, rp, c, v, rpt, ct, vt)
    if st != 0:
        raise ValueError(f"csr_transpose failed: {st}")
    return rpt, ct[: A.nnz].copy(), vt[: A.nnz].copy()


def gmres(A, b, tol=1e-10, maxit=10000, restart=30, precond=0, x0=None):
    return _solve(lib().orc_gmres, A, b, x0, [tol, maxit, restart, precond, 1 if x0 is None else 0])


def arnoldi(A, v0, m, precond=0):
    rp, c, v = _csr(A)
    V = np.zeros((m + 1, A.n))
    H = np.zeros((m, m + 1))
    steps = lib().orc_arnoldi(A.n, rp, c, v, _c(v0, np.float64), m, precond, V, H)
    return V.T.copy(), H.T.copy(), steps  # V: n x (m+1), H: (m+1) x m


def ir(A, val_low, b, tol=1e-10, inner_tol=1e-3, max_outer=50, inner_maxit=10000):
    """Mixed-precision iterative refinement; val_low are the low-precision
    matrix values widened to float32 (same pattern as A)."""
    rp, c, v = _csr(A)
    x = np.zeros(A.n)
    info = Info()
    lib().orc_ir(A.n, rp, c, v, _c(val_low, np.float32), _c(b, np.float64), x, tol, inner_tol,
                 max_outer, inner_maxit, ctypes.byref(info))
    return x, info.as_dict()


# ---------------------------------------------------------------- subwarp model
def _declare_subwarp(L):
    L.orc_subwarp_params.argtypes = [_i32, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                     ctypes.POINTER(ctypes.c_uint64)]
    L.orc_subwarp_params.restype = None
    L.orc_subwarp_vote.argtypes = [_i32p, _i32, _i32, _i32,
                                   np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS"), _i32p, _i32p]
    L.orc_subwarp_vote.restype = None
    L.orc_subwarp_reduce.argtypes = [_f64p, _f64p, _i32, _i32]
    L.orc_segmented_scan.argtypes = [_f64p, _i32p, _f64p, _i32, _i32]
    L.orc_segmented_scan.restype = None


def subwarp_params(tid, size, warpsize=64):
    L = lib()
    _declare_subwarp(L)
    r, o, m = _i32(), _i32(), ctypes.c_uint64()
    L.orc_subwarp_params(tid, size, warpsize, ctypes.byref(r), ctypes.byref(o), ctypes.byref(m))
    return r.value, o.value, m.value


def subwarp_vote(pred, size, warpsize=64):
    L = lib()
    _declare_subwarp(L)
    pred = _c(pred, np.int32)
    n = pred.size
    ballot = np.zeros(n, np.uint64)
    anyv = np.zeros(n, np.int32)
    allv = np.zeros(n, np.int32)
    L.orc_subwarp_vote(pred, n, size, warpsize, ballot, anyv, allv)
    return ballot, anyv, allv


def subwarp_reduce(data, size):
    L = lib()
    _declare_subwarp(L)
    d = _c(data, np.float64)
    out = np.empty_like(d)
    steps = L.orc_subwarp_reduce(d, out, d.size, size)
    return out, steps


def segmented_scan(data, head, width=64):
    L = lib()
    _declare_subwarp(L)
    d = _c(data, np.float64)
    out = np.empty_like(d)
    L.orc_segmented_scan(d, _c(head, np.int32), out, d.size, width)
    return out

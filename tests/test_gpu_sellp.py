"""SELL-P (the Sellp format the paper benchmarks, Section 4) on the GPU:
bit-exact conversion from and to CSR against the oracle, product parity
against the oracle's Dot2-accurate CSR product, run-to-run reproducibility,
and Jacobi-preconditioned CG on a SELL-P matrix, through the C ABI."""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_2006_14290_amd import synth as S

from gpu_util import assert_spmv_f64, assert_spmv_low, dev, host
from test_gpu_spmv import MATS, IDS, _round

pytestmark = pytest.mark.gpu

spx = pytest.importorskip("paper_2006_14290_amd.spx")

SHAPES = [(64, 1), (32, 4), (1, 1), (256, 2), (8, 1)]


def _bits(a):
    return np.ascontiguousarray(a).view({8: np.uint64, 4: np.uint32, 2: np.uint16}[a.dtype.itemsize])


@pytest.mark.parametrize("C,T", SHAPES)
@pytest.mark.parametrize("mi", range(len(MATS)), ids=IDS)
def test_sellp_convert_bit_exact(mi, C, T):
    name, make = MATS[mi]
    if name == "zipf_2e4" and C >= 256:
        pytest.skip("256-row slices of the Zipf rows pad to gigabytes; slice sizes <= 64 cover it")
    A = make()
    print(f"case {name} C={C} T={T}", flush=True)
    P = O.csr_to_sellp(A, C=C, T=T)
    Ad = spx.csr_from_host(A)
    Pd = spx.convert(Ad, spx.SELLP, slice_size=C, stride_factor=T)
    assert Pd.slice_cols == int(P.slice_sets[-1])
    np.testing.assert_array_equal(host(Pd.slice_sets), P.slice_sets)
    np.testing.assert_array_equal(host(Pd.ell_col), P.col)
    np.testing.assert_array_equal(_bits(host(Pd.ell_val)), _bits(P.val))
    B = spx.convert(Pd, spx.CSR)
    np.testing.assert_array_equal(host(B.rowptr), A.rowptr)
    np.testing.assert_array_equal(host(B.colidx), A.col)
    np.testing.assert_array_equal(_bits(host(B.vals)), _bits(np.asarray(A.val)))


@pytest.mark.parametrize("C,T", [(64, 1), (32, 4), (1, 1), (256, 1)])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
@pytest.mark.parametrize("mi", range(len(MATS)), ids=IDS)
def test_sellp_spmv_parity(mi, dtype, C, T):
    name, make = MATS[mi]
    if name == "zipf_2e4" and C >= 256:
        pytest.skip("256-row slices of the Zipf rows pad to gigabytes; slice sizes <= 64 cover it")
    A = make()
    print(f"case {name} {dtype} C={C} T={T}", flush=True)
    P = O.csr_to_sellp(A, C=C, T=T)
    Pd = spx.sellp_from_host(A.n, C, T, P.slice_sets, P.col, P.val, spx.DTYPE_NAMES[dtype])
    x = S.uniform_vector(A.n, seed=12)
    xr = _round(x, "f64" if dtype == "f64" else "f32")
    Ar = S.CSR(A.n, A.rowptr, A.col, _round(A.val, dtype))
    yref, absax = O.csr_spmv_dot2(Ar, xr)
    y = host(spx.spmv(Pd, dev(xr, Pd.vec_dtype)))
    if dtype == "f64":
        assert_spmv_f64(y, yref, absax)
        # alpha / beta
        y0 = S.uniform_vector(A.n, seed=13)
        yb = host(spx.spmv(Pd, dev(xr), dev(y0), alpha=-1.5, beta=0.25))
        assert_spmv_f64(yb, -1.5 * yref + 0.25 * y0, 1.5 * absax, beta_y=0.25 * y0)
    else:
        assert_spmv_low(y, yref, absax, np.diff(A.rowptr))


@pytest.mark.parametrize("T", [1, 2])
def test_sellp_zipf_256_row_slices(T):
    """The largest slice size (256 rows, the kernel's whole work-group) on
    Zipf(1.5) rows: a slice pads to its longest row (up to 10,000 entries),
    so a smaller matrix (n = 5,000; about 5e7 slots) stands in for the
    20,000-row case that the parametrised tests skip. Conversion bit-exact
    both ways, product per row against the oracle in f64 and f32."""
    A = S.zipf_matrix(5000, seed=9)
    print(f"case zipf_5e3 C=256 T={T}", flush=True)
    P = O.csr_to_sellp(A, C=256, T=T)
    Ad = spx.csr_from_host(A)
    Pd = spx.convert(Ad, spx.SELLP, slice_size=256, stride_factor=T)
    assert Pd.slice_cols == int(P.slice_sets[-1])
    np.testing.assert_array_equal(host(Pd.slice_sets), P.slice_sets)
    np.testing.assert_array_equal(host(Pd.ell_col), P.col)
    np.testing.assert_array_equal(_bits(host(Pd.ell_val)), _bits(P.val))
    B = spx.convert(Pd, spx.CSR)
    np.testing.assert_array_equal(host(B.rowptr), A.rowptr)
    np.testing.assert_array_equal(host(B.colidx), A.col)
    np.testing.assert_array_equal(_bits(host(B.vals)), _bits(np.asarray(A.val)))
    x = S.uniform_vector(A.n, seed=12)
    yref, absax = O.csr_spmv_dot2(A, x)
    assert_spmv_f64(host(spx.spmv(Pd, dev(x))), yref, absax)
    P32 = spx.sellp_from_host(A.n, 256, T, P.slice_sets, P.col, P.val, spx.F32)
    xr = _round(x, "f32")
    Ar = S.CSR(A.n, A.rowptr, A.col, _round(A.val, "f32"))
    yref32, absax32 = O.csr_spmv_dot2(Ar, xr)
    assert_spmv_low(host(spx.spmv(P32, dev(xr, P32.vec_dtype))), yref32, absax32, np.diff(A.rowptr))


def test_sellp_bitwise_reproducible_and_matches_convert():
    A = S.zipf_matrix(30000, seed=4)
    Ad = spx.csr_from_host(A)
    Pd = spx.convert(Ad, spx.SELLP)
    x = dev(S.uniform_vector(A.n, seed=1))
    y1 = host(spx.spmv(Pd, x))
    y2 = host(spx.spmv(Pd, x))
    np.testing.assert_array_equal(y1.view(np.uint64), y2.view(np.uint64))
    yref, absax = O.csr_spmv_dot2(A, host(x))
    assert_spmv_f64(y1, yref, absax)


def test_sellp_cast_and_cg_jacobi():
    A = S.poisson3d_7pt(40, 1, 1, 0.01)
    xs = S.uniform_vector(A.n, seed=0, purpose="xstar")
    b, _ = O.csr_spmv_dot2(A, xs)
    Pd = spx.convert(spx.csr_from_host(A), spx.SELLP)
    x, info = spx.cg_solve(Pd, dev(b), tol=1e-10, precond=1, maxit=5000)
    assert info["status"] == spx.OK, info
    r, rn = O.residual(A, b, host(x))
    assert rn / np.linalg.norm(b) <= 1e-10
    _, io = O.cg(A, b, tol=1e-10, precond=1)
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5
    P32 = spx.cast_values(Pd, spx.F32)
    np.testing.assert_array_equal(host(P32.ell_val), host(Pd.ell_val).astype(np.float32))


def test_sellp_bad_slice_size_rejected():
    A = S.poisson2d(8)
    Ad = spx.csr_from_host(A)
    with pytest.raises(spx.SpxError):
        spx.convert(Ad, spx.SELLP, slice_size=48)
    P = O.csr_to_sellp(A, C=64, T=1)
    Pd = spx.sellp_from_host(A.n, 64, 1, P.slice_sets, P.col, P.val)
    Pd.slice_size = 48
    x = dev(np.ones(A.n))
    y = dev(np.zeros(A.n))
    st = spx._lib.spx_spmv(ctypes.byref(Pd.desc()), spx._ptr(x), spx._ptr(y), 1.0, 0.0, spx._stream())
    assert st == spx.ERR_ARG


def test_sellp_bicgstab_gmres_convdiff():
    A = S.convdiff3d_upwind(20)
    xs = S.uniform_vector(A.n, seed=0, purpose="xstar")
    b, _ = O.csr_spmv_dot2(A, xs)
    Pd = spx.convert(spx.csr_from_host(A), spx.SELLP, slice_size=32, stride_factor=2)
    for fn in (spx.bicgstab_solve, spx.gmres_solve):
        x, info = fn(Pd, dev(b), tol=1e-10, precond=1, maxit=5000)
        assert info["status"] == spx.OK, info
        _, rn = O.residual(A, b, host(x))
        assert rn / np.linalg.norm(b) <= 1e-10

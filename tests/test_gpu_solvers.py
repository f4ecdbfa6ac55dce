"""GPU Krylov solvers (CG, BiCGSTAB, GMRES(m), mixed-precision IR) against the
oracle: the true relative residual is recomputed on the host with the
oracle's Dot2 residual, the solution error is bounded through the
condition number, iteration counts are compared with the oracle's, and the
status codes are forced by input."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2006_14290_amd import synth as S

from gpu_util import dev, host

pytestmark = pytest.mark.gpu

spx = pytest.importorskip("paper_2006_14290_amd.spx")


def _problem(A, seed=0):
    xs = S.uniform_vector(A.n, seed=seed, purpose="xstar")
    b, _ = O.csr_spmv_dot2(A, xs)
    return xs, b


def _true_relres(A, b, x):
    _, rn = O.residual(A, b, x)
    return rn / np.linalg.norm(b)


def _fmt(A, fmt):
    Ad = spx.csr_from_host(A)
    return Ad if fmt == "csr" else spx.convert(Ad, {"coo": spx.COO, "ell": spx.ELL, "hyb": spx.HYB}[fmt])


def _kappa_poisson(N, c):
    j = np.arange(1, N + 1)
    lam = 2 * (1 - np.cos(np.pi * j / (N + 1)))
    return sum(ci * lam.max() for ci in c) / sum(ci * lam.min() for ci in c)


# ------------------------------------------------------------------ CG
@pytest.mark.parametrize("fmt", ["csr", "coo", "ell", "hyb"])
@pytest.mark.parametrize("precond", [0, 1])
def test_cg_poisson64(fmt, precond):
    """2D 5-point 64x64 (n = 4096, nnz = 20,224), tol 1e-10."""
    A = S.poisson2d(64)
    xs, b = _problem(A)
    xo, io = O.cg(A, b, tol=1e-10, precond=precond)
    x, info = spx.cg_solve(_fmt(A, fmt), dev(b), tol=1e-10, precond=precond, check_every=8)
    x = host(x)
    assert info["status"] == spx.OK, info
    rr = _true_relres(A, b, x)
    assert rr <= 1e-10, rr
    assert abs(info["relres_true"] - rr) <= 1e-3 * rr + 1e-15
    # rounding-dependent count: within 10% (+5) of the oracle's
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5, (info["iters"], io["iters"])
    kappa = _kappa_poisson(64, (1, 1))
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-10


def test_cg_jacobi_nonconstant_diag_and_x0():
    A = S.spd_diag_dominant(20000, seed=2)
    xs, b = _problem(A, 3)
    x0 = S.uniform_vector(A.n, seed=9)
    x, info = spx.cg_solve(spx.csr_from_host(A), dev(b), x=dev(x0), tol=1e-10, precond=1)
    assert info["status"] == spx.OK
    assert _true_relres(A, b, host(x)) <= 1e-10
    xo, io = O.cg(A, b, tol=1e-10, precond=1, x0=x0)
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5


def test_cg_unaligned_solution_vector():
    """x that is not 32-byte aligned takes the element-wise update kernels;
    the solve must reach the same tolerance and (the same arithmetic in each
    element) the same iterate as an aligned x."""
    A = S.poisson2d(37)
    xs, b = _problem(A, seed=3)
    Ad = spx.csr_from_host(A)
    big = torch.zeros(A.n + 1, dtype=torch.float64, device="cuda")
    xu = big[1:]
    assert xu.data_ptr() % 32 != 0
    xu, info = spx.cg_solve(Ad, dev(b), xu, tol=1e-10, precond=1)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, host(xu)) <= 1e-10
    xa, ia = spx.cg_solve(Ad, dev(b), tol=1e-10, precond=1)
    assert ia["iters"] == info["iters"]
    np.testing.assert_array_equal(host(xa).view(np.uint64), host(xu).view(np.uint64))


@pytest.mark.parametrize("precond", [0, 1])
def test_cg_small_path_agrees_with_general(precond):
    """CSR systems of at most 4096 rows run the whole CG solve in one
    work-group; the same system in ELL takes the general multi-launch driver:
    both meet the tolerance with the same iteration count up to rounding."""
    A = S.poisson2d(64)  # n = 4096: the largest system of the one-group path
    xs, b = _problem(A, 4)
    Ad = spx.csr_from_host(A)
    xc, ic = spx.cg_solve(Ad, dev(b), tol=1e-10, precond=precond)
    xe, ie = spx.cg_solve(spx.convert(Ad, spx.ELL), dev(b), tol=1e-10, precond=precond)
    assert ic["status"] == ie["status"] == spx.OK
    assert abs(ic["iters"] - ie["iters"]) <= 2, (ic["iters"], ie["iters"])
    for x in (host(xc), host(xe)):
        assert _true_relres(A, b, x) <= 1e-10
    np.testing.assert_allclose(host(xc), host(xe), rtol=0, atol=1e-8 * np.abs(xs).max())
    xc2, _ = spx.cg_solve(Ad, dev(b), tol=1e-10, precond=precond)
    np.testing.assert_array_equal(host(xc).view(np.uint64), host(xc2).view(np.uint64))


@pytest.mark.parametrize("n", [1, 777, 4096, 4097])
def test_cg_small_path_x0_jacobi_vs_oracle(n):
    """Jacobi CG from a nonzero x0 on both sides of the one-group size limit."""
    A = S.spd_diag_dominant(n, kmin=1 if n < 5 else 5, seed=n)
    xs, b = _problem(A, n)
    x0 = S.uniform_vector(A.n, seed=n + 1)
    x, info = spx.cg_solve(spx.csr_from_host(A), dev(b), x=dev(x0), tol=1e-10, precond=1)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, host(x)) <= 1e-10
    _, io = O.cg(A, b, tol=1e-10, precond=1, x0=x0)
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5, (info["iters"], io["iters"])
    assert info["relres_true"] <= 1e-10


def test_cg_small_path_cached_matrix_x0():
    """Rows of at most 5 entries (5-point stencil, known from the row-length
    hint): the one-group solve keeps the matrix in registers."""
    A = S.poisson2d(45)
    assert np.diff(A.rowptr).max() <= 5
    xs, b = _problem(A, 6)
    x0 = S.uniform_vector(A.n, seed=7)
    Ad = spx.csr_from_host(A)
    assert 0 < Ad.max_row_len <= 5
    x, info = spx.cg_solve(Ad, dev(b), x=dev(x0), tol=1e-10, precond=1)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, host(x)) <= 1e-10
    _, io = O.cg(A, b, tol=1e-10, precond=1, x0=x0)
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5


def test_cg_small_path_row_hint_too_small():
    """A row-length hint below the true longest row must not change the
    result: the register-cached form hands the solve back to the streaming one."""
    A = S.spd_diag_dominant(3000, seed=8)
    xs, b = _problem(A, 8)
    good = spx.csr_from_host(A)
    bad = spx.csr_from_host(A)
    bad.max_row_len = 3
    xg, ig = spx.cg_solve(good, dev(b), tol=1e-10, precond=1)
    xb, ib = spx.cg_solve(bad, dev(b), tol=1e-10, precond=1)
    assert ig["status"] == ib["status"] == spx.OK
    assert ig["iters"] == ib["iters"]
    np.testing.assert_array_equal(host(xg).view(np.uint64), host(xb).view(np.uint64))
    assert _true_relres(A, b, host(xb)) <= 1e-10


def test_cg_bitwise_reproducible():
    A = S.poisson3d_7pt(20, 1, 1, 0.01)
    xs, b = _problem(A)
    Ad = spx.csr_from_host(A)
    x1, i1 = spx.cg_solve(Ad, dev(b), tol=1e-10, precond=1)
    x2, i2 = spx.cg_solve(Ad, dev(b), tol=1e-10, precond=1)
    assert i1["iters"] == i2["iters"]
    np.testing.assert_array_equal(host(x1).view(np.uint64), host(x2).view(np.uint64))


def test_cg_status_codes():
    # indefinite: p'Ap <= 0
    A = S.from_dense(np.diag([1.0, -1.0, 2.0]))
    x, info = spx.cg_solve(spx.csr_from_host(A), dev(np.array([1.0, 1.0, 0.0])), tol=1e-12)
    assert info["status"] == spx.ERR_BREAKDOWN
    P = S.poisson2d(16)
    xs, b = _problem(P)
    x, info = spx.cg_solve(spx.csr_from_host(P), dev(b), tol=1e-10, maxit=3)
    assert info["status"] == spx.ERR_NOT_CONVERGED and info["iters"] == 3
    bn = b.copy()
    bn[5] = np.nan
    x, info = spx.cg_solve(spx.csr_from_host(P), dev(bn), tol=1e-10)
    assert info["status"] == spx.ERR_NONFINITE
    Z = S.from_dense(np.diag([1.0, 0.0, 2.0]), keep_zeros=True)
    with pytest.raises(spx.SpxError, match="ZERO_DIAG"):
        spx.cg_solve(spx.csr_from_host(Z), dev(np.ones(3)), precond=1)
    x, info = spx.cg_solve(spx.csr_from_host(P), dev(np.zeros(P.n)), tol=1e-10)
    assert info["status"] == spx.OK and info["iters"] == 0 and np.all(host(x) == 0)
    I = S.from_dense(np.eye(50))
    bi = S.uniform_vector(50, seed=1)
    x, info = spx.cg_solve(spx.csr_from_host(I), dev(bi), tol=1e-12)
    assert info["status"] == spx.OK and info["iters"] == 1, info
    # alpha = r.r / p.q is 1 up to the rounding of two differently ordered sums
    np.testing.assert_allclose(host(x), bi, rtol=4e-16, atol=0)


@pytest.mark.timeout(600)
def test_cg_full_aniso_128():
    """Anisotropic 7-point 128^3 (coefficients 1/1/0.01, n = 2,097,152), CG +
    Jacobi to 1e-10; checked through the oracle's true residual and the
    condition-number bound on the error."""
    print("case cg aniso 128^3", flush=True)
    N = 128
    A = S.poisson3d_7pt(N, 1, 1, 0.01)
    assert A.n == 2097152 and A.nnz == 14581760
    xs, b = _problem(A)
    x, info = spx.cg_solve(spx.csr_from_host(A), dev(b), tol=1e-10, precond=1, maxit=5000)
    x = host(x)
    assert info["status"] == spx.OK, info
    rr = _true_relres(A, b, x)
    assert rr <= 1e-10
    kappa = _kappa_poisson(N, (1, 1, 0.01))
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-10
    bound = int(np.ceil(np.sqrt(kappa) / 2 * np.log(2 / 1e-10)))
    assert info["iters"] <= bound
    print("cg aniso 128^3:", info, flush=True)


# ------------------------------------------------------------------ BiCGSTAB
@pytest.mark.parametrize("fmt", ["csr", "coo", "hyb"])
@pytest.mark.parametrize("precond", [0, 1])
def test_bicgstab_convdiff(fmt, precond):
    A = S.convdiff3d_upwind(24)
    xs, b = _problem(A)
    x, info = spx.bicgstab_solve(_fmt(A, fmt), dev(b), tol=1e-10, precond=precond)
    x = host(x)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, x) <= 1e-10
    xo, io = O.bicgstab(A, b, tol=1e-10, precond=precond)
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5, (info["iters"], io["iters"])


def test_bicgstab_identity_and_status():
    I = S.from_dense(np.eye(40))
    bi = S.uniform_vector(40, seed=2)
    x, info = spx.bicgstab_solve(spx.csr_from_host(I), dev(bi), tol=1e-12)
    assert info["status"] == spx.OK and info["iters"] == 1 and info["spmv_count"] == 1
    np.testing.assert_array_equal(host(x), bi)
    A = S.convdiff3d_upwind(10)
    xs, b = _problem(A)
    x, info = spx.bicgstab_solve(spx.csr_from_host(A), dev(b), tol=1e-10, maxit=2)
    assert info["status"] == spx.ERR_NOT_CONVERGED


@pytest.mark.timeout(600)
def test_bicgstab_full_convdiff_128():
    print("case bicgstab convdiff 128^3", flush=True)
    A = S.convdiff3d_upwind(128)
    xs, b = _problem(A)
    x, info = spx.bicgstab_solve(spx.csr_from_host(A), dev(b), tol=1e-10, precond=1, maxit=5000)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, host(x)) <= 1e-10
    print("bicgstab convdiff 128^3:", info, flush=True)


# ------------------------------------------------------------------ GMRES
@pytest.mark.parametrize("fmt", ["csr", "ell"])
@pytest.mark.parametrize("precond", [0, 1])
@pytest.mark.parametrize("m", [30, 5])
def test_gmres_convdiff(fmt, precond, m):
    A = S.convdiff3d_upwind(16)
    xs, b = _problem(A)
    x, info = spx.gmres_solve(_fmt(A, fmt), dev(b), tol=1e-10, precond=precond, restart=m)
    x = host(x)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, x) <= 1e-10
    xo, io = O.gmres(A, b, tol=1e-10, precond=precond, restart=m)
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5, (info["iters"], io["iters"])


def test_gmres_full_space_and_identity():
    rng = np.random.default_rng(4)
    n = 20
    Ad = rng.standard_normal((n, n)) + 8 * np.eye(n)
    A = S.from_dense(Ad)
    b = rng.standard_normal(n)
    x, info = spx.gmres_solve(spx.csr_from_host(A), dev(b), tol=1e-12, restart=n)
    assert info["status"] == spx.OK and info["iters"] <= n
    xd = np.linalg.solve(Ad, b)
    assert np.linalg.norm(host(x) - xd) / np.linalg.norm(xd) <= np.linalg.cond(Ad) * 1e-12 * 4
    I = S.from_dense(np.eye(30))
    x, info = spx.gmres_solve(spx.csr_from_host(I), dev(b[:20].repeat(2)[:30]), tol=1e-12)
    assert info["status"] == spx.OK and info["iters"] == 1


@pytest.mark.timeout(600)
def test_gmres_full_convdiff_128():
    print("case gmres convdiff 128^3", flush=True)
    A = S.convdiff3d_upwind(128)
    xs, b = _problem(A)
    x, info = spx.gmres_solve(spx.csr_from_host(A), dev(b), tol=1e-10, precond=1, restart=30, maxit=5000)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, host(x)) <= 1e-10
    print("gmres convdiff 128^3:", info, flush=True)


# ------------------------------------------------------------------ IR
@pytest.mark.parametrize("low", ["f32", "f16"])
@pytest.mark.parametrize("fmt", ["csr", "ell"])
def test_ir_poisson(low, fmt):
    N = 24
    A = S.poisson3d_7pt(N)
    xs, b = _problem(A)
    A64 = _fmt(A, fmt)
    Alow = spx.cast_values(A64, spx.DTYPE_NAMES[low])
    x, info = spx.ir_solve(A64, Alow, dev(b), tol=1e-10, inner_tol=1e-3)
    x = host(x)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, x) <= 1e-10
    lv, _ = O.cast_values(A.val, low)
    xo, io = O.ir(A, lv.astype(np.float32), b, tol=1e-10, inner_tol=1e-3)
    kappa = _kappa_poisson(N, (1, 1, 1))
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 2 * kappa * 1e-10
    assert abs(info["outer_iters"] - io["outer_iters"]) <= 2


@pytest.mark.timeout(900)
def test_ir_full_192_vs_fp64_oracle():
    """7-point Poisson 192^3 (n = 7,077,888): FP32 and FP16-value IR reach a
    float64 true residual of 1e-10; their error is stated and bounded against
    the float64 oracle's CG solution (all-core variant, the same recurrences
    as the plain oracle) and against x*."""
    print("case ir 192^3", flush=True)
    N = 192
    A = S.poisson3d_7pt(N)
    xs, b = _problem(A)
    xo, io = O.cg_omp(A, b, tol=1e-10, maxit=5000)
    assert io["status"] == O.OK
    assert _true_relres(A, b, xo) <= 1e-10
    print("oracle cg 192^3:", io, flush=True)
    A64 = spx.csr_from_host(A)
    bd = dev(b)
    kappa = _kappa_poisson(N, (1, 1, 1))
    bound = 2 * kappa * 1e-10  # both sides solve to a relative residual of 1e-10
    x64, i64 = spx.cg_solve(A64, bd, tol=1e-10, maxit=5000)
    assert i64["status"] == spx.OK
    x64 = host(x64)
    assert _true_relres(A, b, x64) <= 1e-10
    e64 = np.linalg.norm(x64 - xo) / np.linalg.norm(xo)
    assert e64 <= bound
    print(f"gpu fp64 cg vs oracle: {e64:.3e}", flush=True)
    for low in (spx.F32, spx.F16):
        Alow = spx.cast_values(A64, low)
        x, info = spx.ir_solve(A64, Alow, bd, tol=1e-10, inner_tol=1e-3)
        x = host(x)
        assert info["status"] == spx.OK, info
        assert _true_relres(A, b, x) <= 1e-10
        err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        errs = np.linalg.norm(x - xs) / np.linalg.norm(xs)
        assert err <= bound and errs <= kappa * 1e-10
        print(f"ir 192^3 low={low}: error vs fp64 oracle {err:.3e}, vs x* {errs:.3e}", info, flush=True)


@pytest.mark.parametrize("low", ["f32", "f16"])
def test_ir_ell_inner(low):
    """IR with both matrices in ELL (fused product + dot epilogue of the ELL
    kernel in the inner CG)."""
    A = S.poisson3d_7pt(20)
    xs, b = _problem(A)
    E64 = spx.convert(spx.csr_from_host(A), spx.ELL)
    Elow = spx.cast_values(E64, spx.DTYPE_NAMES[low])
    x, info = spx.ir_solve(E64, Elow, dev(b), tol=1e-10, inner_tol=1e-5)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, host(x)) <= 1e-10
    xc, ic = spx.cg_solve(E64, dev(b), tol=1e-10, precond=1)
    assert ic["status"] == spx.OK
    assert _true_relres(A, b, host(xc)) <= 1e-10


# ---------------------------------------------------------------- block Jacobi
@pytest.mark.parametrize("bs", [2, 8, 32])
def test_cg_block_jacobi_matches_oracle(bs):
    A = S.poisson3d_7pt(23, 1.0, 0.01, 0.01)  # n = 12,167: the last block is partial
    xs, b = _problem(A, seed=4)
    x, info = spx.cg_solve(spx.csr_from_host(A), dev(b), tol=1e-10, precond=bs)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, host(x)) <= 1e-10
    _, io = O.cg(A, b, tol=1e-10, precond=bs)
    assert io["status"] == O.OK
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5


def test_cg_block_jacobi_block_diagonal_one_iteration():
    rng = np.random.default_rng(3)
    bs, n = 8, 8 * 200
    d = np.zeros((n, n))
    for i0 in range(0, n, bs):
        g = rng.uniform(-1, 1, (bs, bs))
        d[i0:i0 + bs, i0:i0 + bs] = g @ g.T + bs * np.eye(bs)
    A = S.from_dense(d)
    b = rng.uniform(-1, 1, n)
    x, info = spx.cg_solve(spx.csr_from_host(A), dev(b), tol=1e-12, precond=bs)
    assert info["status"] == spx.OK and info["iters"] == 1
    np.testing.assert_allclose(host(x), np.linalg.solve(d, b), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("bs", [2, 4, 8, 16, 32])
def test_cg_block_jacobi_exact_blocks_every_size(bs):
    """A block-diagonal SPD matrix whose blocks are the preconditioner's
    (the last one partial, bs - 1 rows): M = A, so one CG iteration solves it
    exactly; checks every block-size instantiation of the setup kernel."""
    rng = np.random.default_rng(10 + bs)
    sizes = [bs] * 40 + [bs - 1]
    n = sum(sizes)
    d = np.zeros((n, n))
    i0 = 0
    for m in sizes:
        g = rng.uniform(-1, 1, (m, m))
        d[i0:i0 + m, i0:i0 + m] = g @ g.T + m * np.eye(m)
        i0 += m
    A = S.from_dense(d)
    b = rng.uniform(-1, 1, n)
    x, info = spx.cg_solve(spx.csr_from_host(A), dev(b), tol=1e-12, precond=bs)
    assert info["status"] == spx.OK and info["iters"] == 1, info
    np.testing.assert_allclose(host(x), np.linalg.solve(d, b), rtol=1e-10, atol=1e-12)


def test_cg_block_jacobi_errors():
    d = np.eye(64)
    d[2:4, 2:4] = [[1.0, 2.0], [2.0, 4.0]]  # a singular 2 x 2 block
    with pytest.raises(spx.SpxError, match="ZERO_DIAG"):
        spx.cg_solve(spx.csr_from_host(S.from_dense(d)), dev(np.ones(64)), precond=2)
    A = S.poisson2d(12)
    Ad = spx.csr_from_host(A)
    b = dev(np.ones(A.n))
    for bad in (3, 64):
        with pytest.raises(spx.SpxError, match="ERR_ARG"):
            spx.cg_solve(Ad, b, precond=bad)
    with pytest.raises(spx.SpxError, match="ERR_ARG"):
        spx.bicgstab_solve(Ad, b, precond=4)
    with pytest.raises(spx.SpxError, match="ERR_ARG"):
        spx.cg_solve(spx.convert(Ad, spx.ELL), b, precond=4)


def _gj_swaps(B):
    """Row swaps Gauss-Jordan with partial pivoting (largest |pivot|, first
    row on ties) makes on B: the pivoting the block inverse must survive."""
    a = np.array(B, dtype=np.float64)
    m = a.shape[0]
    swaps = 0
    for j in range(m):
        piv = j + int(np.argmax(np.abs(a[j:, j])))
        if piv != j:
            a[[j, piv]] = a[[piv, j]]
            swaps += 1
        a[j] /= a[j, j]
        for r in range(m):
            if r != j:
                a[r] -= a[r, j] * a[j]
    return swaps


@pytest.mark.parametrize("bs", [2, 8, 32])
def test_cg_block_jacobi_inverse_with_row_swaps(bs):
    """SPD blocks B = L L^T + I with unit-diagonal L whose first columns are
    large, so every block's partial pivoting swaps rows; the matrix is its
    own block-Jacobi preconditioner, so one CG iteration gives A^-1 b."""
    rng = np.random.default_rng(40 + bs)
    blocks = []
    if bs == 2:
        blocks.append(np.array([[1.0, 2.0], [2.0, 5.0]]))
    while len(blocks) < 24:
        L = np.tril(rng.uniform(-1, 1, (bs, bs)), -1) * 0.3 + np.eye(bs)
        L[1:, 0] = rng.uniform(2.0, 3.0, bs - 1) * rng.choice([-1, 1], bs - 1)
        B = L @ L.T + np.eye(bs)
        if np.linalg.cond(B) < 1e5:
            blocks.append(B)
    assert all(_gj_swaps(B) >= 1 for B in blocks)
    n = bs * len(blocks)
    d = np.zeros((n, n))
    for k, B in enumerate(blocks):
        d[k * bs:(k + 1) * bs, k * bs:(k + 1) * bs] = B
    A = S.from_dense(d)
    b = rng.uniform(-1, 1, n)
    x, info = spx.cg_solve(spx.csr_from_host(A), dev(b), tol=1e-8, precond=bs)
    assert info["status"] == spx.OK and info["iters"] == 1, info
    xd = np.linalg.solve(d, b)
    cond = max(np.linalg.cond(B) for B in blocks)
    assert np.linalg.norm(host(x) - xd) / np.linalg.norm(xd) <= cond * 1e-13
    # the oracle's block inverse (pinned against numpy) agrees as well
    xo, io = O.cg(A, b, tol=1e-8, precond=bs)
    assert io["iters"] == 1
    assert np.linalg.norm(host(x) - xo) / np.linalg.norm(xo) <= cond * 1e-13


@pytest.mark.parametrize("precond", [0, 1])
def test_gmres_longest_restart(precond):
    """GMRES with the largest restart length (m = 62: the Hessenberg triangle
    fills its whole LDS copy) on a nonsymmetric system that needs several
    full cycles, against the oracle."""
    A = S.convdiff3d_upwind(30, peclet=1.0)  # n = 27,000; about 165 Arnoldi steps in 3 cycles
    xs, b = _problem(A, seed=6)
    x, info = spx.gmres_solve(spx.csr_from_host(A), dev(b), tol=1e-10, precond=precond, restart=62, maxit=3000)
    assert info["status"] == spx.OK, info
    assert _true_relres(A, b, host(x)) <= 1e-10
    xo, io = O.gmres(A, b, tol=1e-10, precond=precond, restart=62, maxit=3000)
    assert io["status"] == O.OK
    assert info["iters"] > 2 * 62 and io["iters"] > 2 * 62, (info, io)
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5, (info["iters"], io["iters"])
    with pytest.raises(spx.SpxError, match="ERR_ARG"):
        spx.gmres_solve(spx.csr_from_host(A), dev(b), restart=63)

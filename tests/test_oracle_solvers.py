"""Pins of the oracle's Krylov solvers against mathematics: special cases with
known iteration counts, Krylov optimality (monotone A-norm error / residual),
closed-form condition-number bounds, dense direct solves, the Arnoldi identity,
and an independent library (scipy) for iteration-count magnitudes."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from paper_2006_14290_amd import synth as S


def _problem(A, seed=0):
    xs = S.uniform_vector(A.n, seed=seed, purpose="xstar")
    b, _ = O.csr_spmv_dot2(A, xs)
    return xs, b


def _dense(A):
    return sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n)).toarray()


def _kappa_poisson(N, dims, c=None):
    c = c or [1.0] * dims
    j = np.arange(1, N + 1)
    lam = 2 * (1 - np.cos(np.pi * j / (N + 1)))
    return sum(ci * lam.max() for ci in c) / sum(ci * lam.min() for ci in c)


# ------------------------------------------------------------------ CG
def test_cg_identity_one_iteration():
    A = S.from_dense(np.eye(17))
    b = S.uniform_vector(17, seed=1)
    x, info = O.cg(A, b)
    assert info["status"] == O.OK and info["iters"] == 1
    np.testing.assert_array_equal(x, b)


@pytest.mark.parametrize("k", [1, 3, 7])
def test_cg_k_distinct_eigenvalues(k):
    n = 60
    eig = np.repeat(np.arange(1, k + 1, dtype=float) * 1.5, n // k + 1)[:n]
    A = S.from_dense(np.diag(eig))
    xs, b = _problem(A)
    x, info = O.cg(A, b, tol=1e-12)
    assert info["status"] == O.OK
    assert info["iters"] <= k + 2


def test_cg_a_norm_error_monotone():
    A = S.poisson2d(12)
    xs, b = _problem(A, 3)
    Ad = _dense(A)
    errs = []
    for m in range(1, 40):
        x, info = O.cg(A, b, tol=1e-14, maxit=m)
        e = x - xs
        errs.append(np.sqrt(e @ Ad @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))
    assert errs[-1] < 1e-6 * errs[0]


def test_cg_cfg_small_bounds_and_error():
    N = 64
    A = S.poisson2d(N)
    xs, b = _problem(A)
    x, info = O.cg(A, b, tol=1e-10)
    kappa = _kappa_poisson(N, 2)
    bound = int(np.ceil(np.sqrt(kappa) / 2 * np.log(2 / 1e-10)))
    assert bound == 491
    assert info["status"] == O.OK and info["iters"] <= bound
    assert info["relres_true"] <= 1e-10
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-10
    # independent library: iteration count of the same magnitude as scipy's CG
    m = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))
    its = []
    spla.cg(m, b, rtol=1e-10, maxiter=5000, callback=lambda xk: its.append(1))
    assert 0.8 * len(its) <= info["iters"] <= 1.2 * len(its) + 5


def test_cg_dense_direct_comparison():
    rng = np.random.default_rng(7)
    M = rng.standard_normal((30, 30))
    Ad = M @ M.T + 30 * np.eye(30)
    A = S.from_dense(Ad)
    b = rng.standard_normal(30)
    x, info = O.cg(A, b, tol=1e-13)
    xd = np.linalg.solve(Ad, b)
    kappa = np.linalg.cond(Ad)
    assert info["status"] == O.OK
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= kappa * 1e-13 * 2


def test_jacobi_constant_diagonal_invariant():
    # Constant diagonal: Jacobi is a uniform scaling, iterations unchanged.
    for A in (S.poisson3d_7pt(10, 1, 1, 0.01), S.poisson2d(20)):
        xs, b = _problem(A)
        _, i0 = O.cg(A, b, precond=0)
        _, i1 = O.cg(A, b, precond=1)
        assert abs(i0["iters"] - i1["iters"]) <= 1
    # Non-constant diagonal: Jacobi still converges to the same solution.
    A = S.spd_diag_dominant(500, seed=3)
    xs, b = _problem(A)
    x0, i0 = O.cg(A, b, precond=0)
    x1, i1 = O.cg(A, b, precond=1)
    assert i0["status"] == O.OK and i1["status"] == O.OK
    assert np.linalg.norm(x1 - xs) <= 1e-8 * np.linalg.norm(xs)


def test_cg_status_codes():
    A = S.from_dense(np.diag([1.0, -1.0]))
    _, info = O.cg(A, np.array([1.0, 1.0]))
    assert info["status"] == O.BREAKDOWN
    A = S.poisson2d(8)
    xs, b = _problem(A)
    _, info = O.cg(A, b, maxit=1)
    assert info["status"] == O.NOT_CONVERGED and info["iters"] == 1
    bn = b.copy()
    bn[3] = np.nan
    _, info = O.cg(A, bn)
    assert info["status"] == O.NONFINITE
    Z = S.from_dense(np.diag([1.0, 0.0, 2.0]), keep_zeros=True)
    _, info = O.cg(Z, np.ones(3), precond=1)
    assert info["status"] == O.ZERO_DIAG
    x, info = O.cg(A, np.zeros(A.n))
    assert info["status"] == O.OK and info["iters"] == 0 and np.all(x == 0)


# ------------------------------------------------------------------ BiCGSTAB
def test_bicgstab_identity_half_step():
    A = S.from_dense(np.eye(9))
    b = S.uniform_vector(9, seed=2)
    x, info = O.bicgstab(A, b)
    assert info["status"] == O.OK and info["iters"] == 1 and info["spmv_count"] == 1
    np.testing.assert_array_equal(x, b)


def test_bicgstab_nonsymmetric_dense_and_scipy():
    A = S.convdiff3d_upwind(10)
    xs, b = _problem(A)
    x, info = O.bicgstab(A, b, precond=1)
    assert info["status"] == O.OK and info["relres_true"] <= 1e-10
    Ad = _dense(A)
    xd = np.linalg.solve(Ad, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= np.linalg.cond(Ad) * 1e-10
    m = sp.csr_matrix(Ad)
    its = []
    Minv = spla.LinearOperator(m.shape, matvec=lambda v: v / Ad.diagonal())
    spla.bicgstab(m, b, rtol=1e-10, M=Minv, maxiter=5000, callback=lambda xk: its.append(1))
    assert 0.5 * len(its) <= info["iters"] <= 2 * len(its) + 5


def test_bicgstab_spd_and_status():
    A = S.spd_diag_dominant(400, seed=8)
    xs, b = _problem(A)
    x, info = O.bicgstab(A, b)
    assert info["status"] == O.OK and info["relres_true"] <= 1e-10
    _, info = O.bicgstab(A, b, maxit=1)
    assert info["status"] == O.NOT_CONVERGED


# ------------------------------------------------------------------ GMRES
def test_gmres_full_space_converges_in_n_steps():
    rng = np.random.default_rng(4)
    n = 20
    Ad = rng.standard_normal((n, n)) + 8 * np.eye(n)
    A = S.from_dense(Ad)
    b = rng.standard_normal(n)
    x, info = O.gmres(A, b, tol=1e-12, restart=n)
    assert info["status"] == O.OK and info["iters"] <= n
    xd = np.linalg.solve(Ad, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= np.linalg.cond(Ad) * 1e-12 * 4


def test_gmres_residual_non_increasing_across_restarts():
    A = S.convdiff3d_upwind(5)
    xs, b = _problem(A)
    res = []
    for m in range(1, 45):
        _, info = O.gmres(A, b, tol=1e-14, maxit=m, restart=8, precond=1)
        res.append(info["relres_true"])
    assert all(res[i + 1] <= res[i] * (1 + 1e-9) + 1e-15 for i in range(len(res) - 1))


def test_arnoldi_identity_and_orthonormality():
    A = S.convdiff3d_upwind(4)
    v0 = S.uniform_vector(A.n, seed=5)
    m = 12
    for precond in (0, 1):
        V, H, steps = O.arnoldi(A, v0, m, precond)
        assert steps == m
        Ad = _dense(A)
        Mi = np.diag(1 / Ad.diagonal()) if precond else np.eye(A.n)
        lhs = Ad @ Mi @ V[:, :m]
        rhs = V @ H
        assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.abs(Ad).sum(axis=1).max()
        # MGS loses orthogonality in proportion to the conditioning of the
        # Krylov basis (Bjorck 1967; Paige, Rozloznik, Strakos 2006): tight
        # for the first vectors, looser for the whole basis.
        G = V.T @ V - np.eye(m + 1)
        assert np.max(np.abs(G[:6, :6])) <= 1e-12
        assert np.max(np.abs(G)) <= 1e-6
        assert np.all(np.tril(H, -2) == 0)


def test_gmres_identity_and_scipy_magnitude():
    A = S.from_dense(np.eye(11))
    b = S.uniform_vector(11, seed=3)
    x, info = O.gmres(A, b)
    assert info["status"] == O.OK and info["iters"] == 1
    np.testing.assert_allclose(x, b, rtol=0, atol=1e-15)
    A = S.convdiff3d_upwind(10)
    xs, b = _problem(A)
    x, info = O.gmres(A, b, precond=1)
    assert info["status"] == O.OK and info["relres_true"] <= 1e-10
    Ad = _dense(A)
    its = []
    Minv = spla.LinearOperator(Ad.shape, matvec=lambda v: v / Ad.diagonal())
    spla.gmres(sp.csr_matrix(Ad), b, rtol=1e-10, restart=30, M=Minv, maxiter=200,
               callback=lambda pr: its.append(1), callback_type="pr_norm")
    assert 0.5 * len(its) <= info["iters"] <= 2 * len(its) + 5


# ------------------------------------------------------------------ IR
@pytest.mark.parametrize("low", ["f32", "f16"])
def test_ir_reaches_fp64_tolerance(low):
    A = S.poisson3d_7pt(16)
    xs, b = _problem(A)
    lv, ov = O.cast_values(A.val, low)
    assert ov == 0
    x, info = O.ir(A, lv.astype(np.float32), b, tol=1e-10, inner_tol=1e-3)
    assert info["status"] == O.OK
    _, rn = O.residual(A, b, x)
    assert rn / np.linalg.norm(b) <= 1e-10
    x64, i64 = O.cg(A, b)
    kappa = _kappa_poisson(16, 3)
    assert np.linalg.norm(x - x64) / np.linalg.norm(x64) <= 2 * kappa * 1e-10
    assert 2 <= info["outer_iters"] <= 8


def test_residual_dot2_exact_on_integers():
    A = S.poisson2d(9)
    x = np.arange(A.n, dtype=float)
    b = np.zeros(A.n)
    r, nr = O.residual(A, b, x)
    exp = -O.csr_spmv(A, x)  # integer data: both exact
    np.testing.assert_array_equal(r, exp)

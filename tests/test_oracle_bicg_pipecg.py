"""Pins of the oracle's CSR transpose, BiCG and pipelined CG.

Transpose: against the dense transpose and scipy's, involution, rectangular
and empty inputs. BiCG (Section 1 lists it among the library's solvers): on a
symmetric matrix with the shadow residual r~ = r it takes exactly CG's steps;
on nonsymmetric matrices the residual and shadow residual sequences are
bi-orthogonal (r~_j' M^-1 r_i = 0, i != j), which a product with A in place of
A^T or a wrong sign breaks; it reaches the dense solution and terminates in at
most n steps on small systems; the textbook breakdown case. Pipelined CG
(Ghysels & Vanroose 2014): its iterates agree with CG's step by step and it
reaches the dense solution."""
from types import SimpleNamespace

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2006_14290_amd import synth as S


def _dense(A, ncols=None):
    d = np.zeros((A.n, A.n if ncols is None else ncols))
    for i in range(A.n):
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            d[i, A.col[p]] = A.val[p]
    return d


def _rhs(A, seed=0):
    xs = S.uniform_vector(A.n, seed=seed, purpose="xstar")
    return O.csr_spmv(A, xs)


# ---------------------------------------------------------------- transpose
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_transpose_matches_dense_and_scipy(seed):
    A = S.random_small(97, 0.08, seed=seed, empty_rows=(0, 5, 96), long_rows=(3,))
    rpt, ct, vt = O.csr_transpose(A)
    T = S.CSR(A.n, rpt, ct, vt)
    np.testing.assert_array_equal(_dense(T), _dense(A).T)
    # rows of A^T sorted by column, and the arrays equal scipy's canonical form
    ref = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n)).T.tocsr()
    ref.sort_indices()
    np.testing.assert_array_equal(rpt, ref.indptr)
    np.testing.assert_array_equal(ct, ref.indices)
    np.testing.assert_array_equal(vt, ref.data)


def test_transpose_is_an_involution():
    A = S.convdiff3d_upwind(7)
    rpt, ct, vt = O.csr_transpose(A)
    r2, c2, v2 = O.csr_transpose(S.CSR(A.n, rpt, ct, vt))
    np.testing.assert_array_equal(r2, A.rowptr)
    np.testing.assert_array_equal(c2, A.col)
    np.testing.assert_array_equal(v2.view(np.uint64), A.val.view(np.uint64))


def test_transpose_rectangular_and_empty():
    rng = np.random.default_rng(3)
    d = rng.uniform(-1, 1, (13, 40)) * (rng.random((13, 40)) < 0.2)
    rows, cols = np.nonzero(d)
    rowptr = np.zeros(14, np.int32)
    np.add.at(rowptr, rows + 1, 1)
    A = SimpleNamespace(n=13, rowptr=np.cumsum(rowptr).astype(np.int32), col=cols.astype(np.int32),
                        val=d[rows, cols], nnz=len(rows))
    rpt, ct, vt = O.csr_transpose(A, ncols=40)
    assert len(rpt) == 41
    np.testing.assert_array_equal(_dense(S.CSR(40, rpt, ct, vt), ncols=13), d.T)
    E = S.CSR(5, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0))
    rpt, ct, vt = O.csr_transpose(E)
    assert not rpt.any() and len(ct) == 0
    bad = S.CSR(2, np.array([0, 1, 1], np.int32), np.array([2], np.int32), np.ones(1))
    with pytest.raises(ValueError):
        O.csr_transpose(bad)


# ---------------------------------------------------------------- BiCG
@pytest.mark.parametrize("precond", [0, 1])
def test_bicg_on_symmetric_matrix_is_cg(precond):
    A = S.spd_diag_dominant(300, seed=4)
    b = _rhs(A, 4)
    for k in (1, 3, 12):
        xb, ib = O.bicg(A, b, tol=1e-14, maxit=k, precond=precond)
        xc, ic = O.cg(A, b, tol=1e-14, maxit=k, precond=precond)
        assert ib["iters"] == ic["iters"] == k
        np.testing.assert_array_equal(xb.view(np.uint64), xc.view(np.uint64))
    xb, ib = O.bicg(A, b, tol=1e-10, precond=precond)
    xc, ic = O.cg(A, b, tol=1e-10, precond=precond)
    assert ib["status"] == O.OK and ib["iters"] == ic["iters"]
    assert ib["spmv_count"] == 2 * ib["iters"]


@pytest.mark.parametrize("precond", [0, 1])
def test_bicg_residuals_are_biorthogonal(precond):
    A = S.convdiff3d_upwind(6, peclet=20.0)
    d = _dense(A)
    assert np.abs(d - d.T).max() > 0.1
    b = _rhs(A, 5)
    k = 8
    _, _, R, RT = O.bicg(A, b, tol=1e-14, maxit=k, precond=precond, nhist=k)
    minv = 1.0 / np.diag(d) if precond else np.ones(A.n)
    Z = R * minv  # M^-1 r_i
    G = RT @ Z.T  # G[j, i] = r~_j' M^-1 r_i
    scale = np.outer(np.linalg.norm(RT, axis=1), np.linalg.norm(Z, axis=1))
    off = np.abs(G / scale)[~np.eye(k, dtype=bool)]
    assert off.max() < 1e-8, off.max()
    assert np.all(np.abs(np.diag(G) / np.diag(scale)) > 1e-6)


def test_bicg_reaches_dense_solution():
    A = S.convdiff3d_upwind(8, peclet=10.0)
    b = _rhs(A, 6)
    d = _dense(A)
    xd = np.linalg.solve(d, b)
    for precond in (0, 1):
        x, info = O.bicg(A, b, tol=1e-12, precond=precond)
        assert info["status"] == O.OK
        assert info["relres_true"] <= 1e-12
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < np.linalg.cond(d) * 1e-12


def test_bicg_finite_termination_small():
    rng = np.random.default_rng(7)
    n = 10
    d = rng.uniform(-1, 1, (n, n)) + np.diag(np.full(n, 6.0))
    A = S.from_dense(d)
    b = rng.uniform(-1, 1, n)
    x, info = O.bicg(A, b, tol=1e-11)
    assert info["status"] == O.OK and info["iters"] <= n
    np.testing.assert_allclose(x, np.linalg.solve(d, b), rtol=1e-9, atol=1e-12)


def test_bicg_breakdown_and_special_cases():
    # [[0,1],[1,0]], b = e0, no preconditioner: p = e0, q = A p = e1, p~'q = 0
    A = S.from_dense(np.array([[0.0, 1.0], [1.0, 0.0]]))
    _, info = O.bicg(A, np.array([1.0, 0.0]), tol=1e-10)
    assert info["status"] == O.BREAKDOWN
    # Jacobi needs the diagonal
    _, info = O.bicg(A, np.array([1.0, 0.0]), tol=1e-10, precond=1)
    assert info["status"] == O.ZERO_DIAG
    B = S.convdiff3d_upwind(4)
    x, info = O.bicg(B, np.zeros(B.n))
    assert info["status"] == O.OK and info["iters"] == 0 and not x.any()
    bn = np.ones(B.n)
    bn[3] = np.nan
    _, info = O.bicg(B, bn)
    assert info["status"] == O.NONFINITE
    # a diagonal system: one step
    D = S.from_dense(np.diag(np.arange(1.0, 9.0)))
    x, info = O.bicg(D, np.ones(8), precond=1)
    assert info["status"] == O.OK and info["iters"] == 1
    np.testing.assert_allclose(x, 1.0 / np.arange(1.0, 9.0), rtol=1e-15)


# ---------------------------------------------------------------- pipelined CG
@pytest.mark.parametrize("precond", [0, 1])
def test_pipecg_iterates_follow_cg(precond):
    A = S.spd_diag_dominant(400, seed=8)
    b = _rhs(A, 8)
    for k in (1, 2, 5, 15):
        xp, ip = O.pipecg(A, b, tol=1e-15, maxit=k, precond=precond)
        xc, ic = O.cg(A, b, tol=1e-15, maxit=k, precond=precond)
        assert ip["iters"] == ic["iters"] == k
        np.testing.assert_allclose(xp, xc, rtol=0, atol=1e-11 * np.abs(xc).max())


@pytest.mark.parametrize("precond", [0, 1])
def test_pipecg_reaches_dense_solution(precond):
    A = S.poisson3d_7pt(7, cx=1.0, cy=4.0, cz=0.5)
    b = _rhs(A, 9)
    d = _dense(A)
    xd = np.linalg.solve(d, b)
    x, info = O.pipecg(A, b, tol=1e-11, precond=precond)
    assert info["status"] == O.OK and info["relres_true"] <= 1e-11
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < np.linalg.cond(d) * 1e-11
    _, ic = O.cg(A, b, tol=1e-11, precond=precond)
    assert abs(info["iters"] - ic["iters"]) <= 2
    # one product per iteration plus the start's w = A u
    assert info["spmv_count"] >= info["iters"] + 1


def test_pipecg_special_cases():
    one = S.from_dense(np.array([[4.0]]))
    x, info = O.pipecg(one, np.array([2.0]))
    assert info["status"] == O.OK and info["iters"] == 1 and x[0] == 0.5
    n = 6
    ind = S.from_dense(np.diag([1.0, -1.0] * (n // 2)))
    _, info = O.pipecg(ind, np.ones(n))
    assert info["status"] == O.BREAKDOWN
    A = S.poisson2d(6)
    x, info = O.pipecg(A, np.zeros(A.n))
    assert info["status"] == O.OK and info["iters"] == 0 and not x.any()
    bn = np.ones(A.n)
    bn[0] = np.inf
    _, info = O.pipecg(A, bn)
    assert info["status"] == O.NONFINITE

"""Pins of the oracle's all-core variants against the plain (pinned) oracle:
the OpenMP product sums rows in the same order, so it is bitwise the plain
product; OpenMP CG takes the same steps with differently combined dot
products, so it must agree with plain CG to rounding and meet the same
closed-form checks."""
import numpy as np
import pytest

import oracle as O
from paper_2006_14290_amd import synth as S


def test_omp_product_bitwise_plain():
    for A in (S.stencil27_random(18, seed=2), S.zipf_matrix(20000, seed=4),
              S.random_small(500, 0.02, seed=3, empty_rows=(0, 1, 499), long_rows=(7,))):
        x = S.uniform_vector(A.n, seed=1)
        y0 = S.uniform_vector(A.n, seed=7)
        np.testing.assert_array_equal(O.csr_spmv_omp(A, x).view(np.uint64), O.csr_spmv(A, x).view(np.uint64))
        np.testing.assert_array_equal(O.csr_spmv_omp(A, x, y0, 0.5, -2.0).view(np.uint64),
                                      O.csr_spmv(A, x, y0, 0.5, -2.0).view(np.uint64))


@pytest.mark.parametrize("precond", [0, 1])
def test_omp_cg_agrees_with_plain_cg(precond):
    A = S.poisson3d_7pt(20, 1.0, 1.0, 0.01)
    xs = S.uniform_vector(A.n, seed=3, purpose="xstar")
    b, _ = O.csr_spmv_dot2(A, xs)
    xo, io = O.cg(A, b, tol=1e-10, precond=precond)
    xm, im = O.cg_omp(A, b, tol=1e-10, precond=precond)
    assert io["status"] == im["status"] == O.OK
    assert abs(io["iters"] - im["iters"]) <= 2
    _, rn = O.residual(A, b, xm)
    assert rn <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(xm - xo) / np.linalg.norm(xo) <= 1e-7


def test_omp_cg_closed_forms():
    # A = I: one iteration, x = b
    I = S.from_dense(np.eye(50))
    b = S.uniform_vector(50, seed=5)
    x, info = O.cg_omp(I, b)
    assert info["status"] == O.OK and info["iters"] == 1
    np.testing.assert_array_equal(x, b)
    # diagonal with 4 distinct eigenvalues: at most 4 (+2 for rounding) iterations
    d = np.repeat([1.0, 3.0, 7.0, 20.0], 25)
    x, info = O.cg_omp(S.from_dense(np.diag(d)), b.repeat(2), tol=1e-12)
    assert info["status"] == O.OK and info["iters"] <= 6
    np.testing.assert_allclose(x, b.repeat(2) / d, rtol=1e-11)
    # zero diagonal with Jacobi
    Z = S.from_dense(np.diag(np.r_[np.ones(9), 0.0]), keep_zeros=True)
    _, info = O.cg_omp(Z, np.ones(10), precond=1)
    assert info["status"] == O.ZERO_DIAG
    assert O.omp_threads() >= 1

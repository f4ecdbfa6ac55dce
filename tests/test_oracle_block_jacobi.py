"""Pins of the oracle's block-Jacobi preconditioner (Section 1 lists
block-Jacobi among the library's preconditioners; the scalar Jacobi is its
1x1 case): inverted blocks against numpy.linalg.inv, its application against
a dense block solve, exact one-step convergence of PCG on block-diagonal
systems, pivoting, partial last blocks and singular blocks."""
import numpy as np
import pytest

import oracle as O
from paper_2006_14290_amd import synth as S


def _dense_blocks(A, bs):
    d = np.zeros((A.n, A.n))
    for i in range(A.n):
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            d[i, A.col[p]] = A.val[p]
    out = []
    for i0 in range(0, A.n, bs):
        m = min(bs, A.n - i0)
        out.append(d[i0:i0 + m, i0:i0 + m])
    return out


@pytest.mark.parametrize("bs", [2, 4, 8, 32])
def test_block_inverses_match_numpy(bs):
    # nonsymmetric, diagonally dominant, n not a multiple of bs
    rng = np.random.default_rng(bs)
    n = 4 * bs + 3
    d = rng.uniform(-1, 1, (n, n)) * (rng.random((n, n)) < 0.4) + np.diag(rng.uniform(3, 5, n))
    A = S.from_dense(d)
    inv = O.block_jacobi(A, bs)
    for k, blk in enumerate(_dense_blocks(A, bs)):
        m = blk.shape[0]
        ref = np.linalg.inv(blk)
        np.testing.assert_allclose(inv[k, :m, :m], ref, rtol=1e-12, atol=1e-14)
        assert not inv[k, m:, :].any() and not inv[k, :, m:].any()
    r = rng.uniform(-1, 1, n)
    z = O.block_jacobi_apply(inv, r)
    zref = np.concatenate([np.linalg.solve(blk, r[i0:i0 + blk.shape[0]])
                           for i0, blk in zip(range(0, n, bs), _dense_blocks(A, bs))])
    np.testing.assert_allclose(z, zref, rtol=1e-12, atol=1e-14)


def test_pivoting_zero_diagonal_block():
    # the block [[0, 2], [3, 0]] is nonsingular but has zero diagonal entries
    d = np.array([[0.0, 2.0, 0, 0], [3.0, 0.0, 0, 0], [0, 0, 1.0, 0.5], [0, 0, 0.25, 2.0]])
    inv = O.block_jacobi(S.from_dense(d), 2)
    np.testing.assert_allclose(inv[0], np.linalg.inv(d[:2, :2]), rtol=1e-15)
    np.testing.assert_allclose(inv[1], np.linalg.inv(d[2:, 2:]), rtol=1e-15)


def test_singular_block_reported():
    d = np.eye(6)
    d[2:4, 2:4] = [[1.0, 2.0], [2.0, 4.0]]  # rank one
    with pytest.raises(ValueError):
        O.block_jacobi(S.from_dense(d), 2)
    A = S.from_dense(d)
    x, info = O.cg(A, np.ones(6), precond=2)
    assert info["status"] == O.ZERO_DIAG


@pytest.mark.parametrize("bs", [4, 8])
def test_pcg_block_diagonal_one_iteration(bs):
    """With M = A (A block diagonal with bs x bs SPD blocks), PCG is exact
    after one step."""
    rng = np.random.default_rng(7)
    n = 10 * bs
    d = np.zeros((n, n))
    for i0 in range(0, n, bs):
        g = rng.uniform(-1, 1, (bs, bs))
        d[i0:i0 + bs, i0:i0 + bs] = g @ g.T + bs * np.eye(bs)
    A = S.from_dense(d)
    b = rng.uniform(-1, 1, n)
    x, info = O.cg(A, b, tol=1e-12, precond=bs)
    assert info["status"] == O.OK and info["iters"] == 1
    np.testing.assert_allclose(x, np.linalg.solve(d, b), rtol=1e-12, atol=1e-13)


def test_one_block_is_exact_inverse():
    A = S.poisson2d(5)  # n = 25 -> one 32 x 32 block holding the whole matrix
    b = S.uniform_vector(A.n, seed=1)
    x, info = O.cg(A, b, tol=1e-12, precond=32)
    assert info["status"] == O.OK and info["iters"] == 1


def test_block_jacobi_pcg_converges_and_helps_on_lines():
    """Anisotropic Poisson with strong coupling along x: 8-row blocks hold
    pieces of x-lines, so block Jacobi needs fewer iterations than scalar
    Jacobi (and both reach the tolerance)."""
    A = S.poisson3d_7pt(16, 1.0, 0.01, 0.01)
    b = S.uniform_vector(A.n, seed=2)
    _, i1 = O.cg(A, b, tol=1e-10, precond=1)
    x8, i8 = O.cg(A, b, tol=1e-10, precond=8)
    assert i1["status"] == O.OK and i8["status"] == O.OK
    assert i8["relres_true"] <= 1e-10
    assert i8["iters"] < i1["iters"]

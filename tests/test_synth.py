"""The seeded input generators: shapes and structure the workloads state
(closed-form sizes, symmetry and diagonal dominance, Zipf row-length laws),
and the torch assembly path of the SPD generator giving the same matrix."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2006_14290_amd import synth as S


@pytest.mark.parametrize("n", [1000, 4321])
def test_spd_generator_symmetric_dominant_and_canonical(n):
    A = S.spd_diag_dominant(n, seed=n)
    M = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(n, n))
    assert (abs(M - M.T) > 0).nnz == 0
    d = M.diagonal()
    off = np.asarray(abs(M).sum(axis=1)).ravel() - np.abs(d)
    assert np.all(d > off + 0.999)
    lens = A.row_lengths()
    # (k-1)/2 partners drawn per row and mirrored: about k entries per row on average
    assert 15 < lens.mean() < 19 and lens.min() >= 1
    for i in range(0, n, 97):  # canonical rows
        c = A.col[A.rowptr[i]:A.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c


def test_spd_generator_torch_path_same_bits():
    for n in (1000, 20000):
        A = S.spd_diag_dominant(n, seed=7)
        B = S.spd_diag_dominant(n, seed=7, device="cpu")
        np.testing.assert_array_equal(A.rowptr, B.rowptr)
        np.testing.assert_array_equal(A.col, B.col)
        np.testing.assert_array_equal(A.val.view(np.uint64), B.val.view(np.uint64))


def test_zipf_rows_follow_the_clipped_law():
    Z = S.zipf_matrix(200000, seed=1)
    lens = Z.row_lengths()
    assert lens.min() >= 1 and lens.max() == 10000
    # P(len = 1) = 1/zeta(1.5) = 0.3828 for numpy's zipf(1.5)
    assert abs((lens == 1).mean() - 0.3828) < 0.005
    for i in range(0, Z.n, 9973):
        c = Z.col[Z.rowptr[i]:Z.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0) and c.min() >= 0 and c.max() < Z.n

"""spx_validate on the device: canonical matrices from the oracle pass, and
every declared class (FORMAT, RANGE, UNSORTED, DUPLICATE) is reported for a
planted defect in each format's index arrays. The validation kernels only
compare indices; structure is checked before any row pointer or slice
offset is followed, so planted defects never steer a load out of bounds."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2006_14290_amd import synth as S

pytestmark = pytest.mark.gpu

spx = pytest.importorskip("paper_2006_14290_amd.spx")


def _base():
    return S.random_small(300, 0.03, seed=11, empty_rows=tuple(range(40, 60)), long_rows=(7, 299))


def _row_with(A, minlen):
    lens = np.diff(A.rowptr)
    return [int(i) for i in np.flatnonzero(lens >= minlen)]


def _csr_dev(rowptr, col, val, n, nnz=None):
    return spx.Matrix(spx.CSR, spx.F64, n, n, int(rowptr[-1]) if nnz is None else nnz,
                      rowptr=torch.from_numpy(np.ascontiguousarray(rowptr, np.int32)).cuda(),
                      colidx=torch.from_numpy(np.ascontiguousarray(col, np.int32)).cuda(),
                      vals=torch.from_numpy(np.ascontiguousarray(val, np.float64)).cuda())


def test_csr_classes():
    A = _base()
    assert spx.validate(spx.csr_from_host(A)) == spx.OK
    rp = A.rowptr.copy()
    rp[0] = 1
    assert spx.validate(_csr_dev(rp, A.col, A.val, A.n, A.nnz)) == spx.ERR_FORMAT
    assert spx.validate(_csr_dev(A.rowptr, A.col, A.val, A.n, A.nnz + 1)) == spx.ERR_FORMAT
    rp = A.rowptr.copy()
    r = _row_with(A, 1)[3]  # three non-empty rows before it: rp[r] >= 3
    rp[r + 1] = rp[r] - 1
    assert spx.validate(_csr_dev(rp, A.col, A.val, A.n, A.nnz)) == spx.ERR_FORMAT
    i = _row_with(A, 3)[2]
    b = int(A.rowptr[i])
    for fix, code in (((b + 1, 300), spx.ERR_RANGE), ((b + 1, -5), spx.ERR_RANGE)):
        col = A.col.copy()
        col[fix[0]] = fix[1]
        assert spx.validate(_csr_dev(A.rowptr, col, A.val, A.n)) == code
        assert f"position {fix[0]}" in spx.last_error()
    col = A.col.copy()
    col[b], col[b + 1] = col[b + 1], col[b]
    assert spx.validate(_csr_dev(A.rowptr, col, A.val, A.n)) == spx.ERR_UNSORTED
    col = A.col.copy()
    col[b + 2] = col[b + 1]
    assert spx.validate(_csr_dev(A.rowptr, col, A.val, A.n)) == spx.ERR_DUPLICATE
    assert f"position {b + 1}" in spx.last_error()
    # a row may start below where the previous one ended
    B = S.CSR(3, np.array([0, 2, 4, 5], np.int32), np.array([1, 2, 0, 1, 2], np.int32), np.ones(5))
    assert spx.validate(spx.csr_from_host(B)) == spx.OK


def test_csr_host_and_device_agree():
    A = _base()
    rng = np.random.default_rng(5)
    for trial in range(12):
        col = A.col.copy()
        for _ in range(int(rng.integers(1, 4))):
            p = int(rng.integers(0, A.nnz))
            col[p] = int(rng.integers(-2, A.n + 2))
        hs = spx.validate_csr_host(A.n, A.n, A.rowptr, col)
        ds = spx.validate(_csr_dev(A.rowptr, col, A.val, A.n))
        assert hs == ds, (trial, hs, ds)


def test_coo_classes():
    A = _base()
    row = O.csr_to_coo_rows(A)
    ok = spx.coo_from_host(A.n, row, A.col, A.val)
    assert spx.validate(ok) == spx.OK
    p = int(A.rowptr[_row_with(A, 3)[1]])
    for mutate, code in (
        (lambda r, c: r.__setitem__(p, A.n), spx.ERR_RANGE),
        (lambda r, c: c.__setitem__(p, -1), spx.ERR_RANGE),
        (lambda r, c: (c.__setitem__(p, c[p + 1]), c.__setitem__(p + 1, A.col[p])), spx.ERR_UNSORTED),
        (lambda r, c: c.__setitem__(p + 1, c[p]), spx.ERR_DUPLICATE),
        (lambda r, c: r.__setitem__(p, r[p] + 1), spx.ERR_UNSORTED),  # rows out of order
    ):
        r, c = row.copy(), A.col.copy()
        mutate(r, c)
        assert spx.validate(spx.coo_from_host(A.n, r, c, A.val)) == code


def test_ell_classes():
    A = _base()
    E = O.csr_to_ell(A, ld=A.n + 3)
    assert spx.validate(spx.ell_from_host(E.n, E.K, E.ld, E.col, E.val)) == spx.OK
    lens = np.diff(A.rowptr)
    short = int(np.flatnonzero((lens >= 1) & (lens <= E.K - 2))[0])
    L = int(lens[short])
    # an entry after a padding slot
    col = E.col.copy()
    col[(L + 1) * E.ld + short] = A.n - 1
    M = spx.ell_from_host(E.n, E.K, E.ld, col, E.val)
    assert spx.validate(M) == spx.ERR_FORMAT
    i = _row_with(A, 3)[0]
    for k, v, code in ((1, A.n, spx.ERR_RANGE), (1, -2, spx.ERR_RANGE)):
        col = E.col.copy()
        col[k * E.ld + i] = v
        assert spx.validate(spx.ell_from_host(E.n, E.K, E.ld, col, E.val)) == code
    col = E.col.copy()
    col[i], col[E.ld + i] = col[E.ld + i], col[i]
    assert spx.validate(spx.ell_from_host(E.n, E.K, E.ld, col, E.val)) == spx.ERR_UNSORTED
    col = E.col.copy()
    col[E.ld + i] = col[i]
    assert spx.validate(spx.ell_from_host(E.n, E.K, E.ld, col, E.val)) == spx.ERR_DUPLICATE
    # nnz must count the stored entries
    M = spx.ell_from_host(E.n, E.K, E.ld, E.col, E.val)
    M.nnz += 1
    assert spx.validate(M) == spx.ERR_FORMAT


def test_hyb_classes():
    A = _base()
    H = O.csr_to_hyb(A, K=2)
    E = H.ell

    def mk(ecol=E.col, row=H.row, col=H.col):
        return spx.hyb_from_host(E.n, E.K, E.ld, ecol, E.val, row, col, H.val)

    assert len(H.row) > 0
    assert spx.validate(mk()) == spx.OK
    # a COO entry for a row whose ELL part is not full
    lens = np.diff(A.rowptr)
    i = int(np.flatnonzero(lens > 2)[0])
    ecol = E.col.copy()
    ecol[E.ld + i] = -1
    assert spx.validate(mk(ecol=ecol)) == spx.ERR_FORMAT
    # the row's first COO column at or below its last ELL column
    p = int(np.flatnonzero(H.row == i)[0])
    col = H.col.copy()
    col[p] = E.col[E.ld + i]
    assert spx.validate(mk(col=col)) == spx.ERR_DUPLICATE
    col[p] = E.col[i]
    assert spx.validate(mk(col=col)) == spx.ERR_UNSORTED
    row = H.row.copy()
    row[p] = A.n + 7
    assert spx.validate(mk(row=row)) == spx.ERR_RANGE


def test_sellp_classes():
    A = _base()
    P = O.csr_to_sellp(A, C=32, T=2)

    def mk(sets=P.slice_sets, col=P.col):
        return spx.sellp_from_host(P.n, P.C, P.T, sets, col, P.val)

    assert spx.validate(mk()) == spx.OK
    sets = P.slice_sets.copy()
    sets[1] += 1  # width no longer a multiple of the stride factor
    assert spx.validate(mk(sets=sets)) == spx.ERR_FORMAT
    # a stored entry in a padding row of the last slice (300 rows, slices of 32)
    col = P.col.copy()
    s = len(P.slice_sets) - 2
    last = P.n - s * P.C  # rows of the last slice that exist
    col[int(P.slice_sets[s]) * P.C + last] = 0
    assert spx.validate(mk(col=col)) == spx.ERR_FORMAT
    i = _row_with(A, 3)[0]
    s, l = divmod(i, P.C)
    col = P.col.copy()
    col[(int(P.slice_sets[s]) + 1) * P.C + l] = col[int(P.slice_sets[s]) * P.C + l]
    assert spx.validate(mk(col=col)) == spx.ERR_DUPLICATE


@pytest.mark.slow
@pytest.mark.parametrize("maker", ["27pt100", "zipf1e6"])
def test_full_size_matrices_are_canonical(maker):
    A = S.stencil27_random(100) if maker == "27pt100" else S.zipf_matrix(1_000_000, seed=0)
    Ad = spx.csr_from_host(A)
    assert spx.validate(Ad) == spx.OK
    assert spx.validate(spx.convert(Ad, spx.COO)) == spx.OK
    assert spx.validate(spx.convert(Ad, spx.HYB)) == spx.OK


def test_server_rejects_malformed_requests_before_queueing():
    A = S.poisson2d(20)
    b = np.ones(A.n)
    srv = spx.Server(max_slots=4, hbm_budget_bytes=64 << 20)
    try:
        col = A.col.copy()
        col[5] = A.n
        bad = S.CSR(A.n, A.rowptr, col, A.val)
        with pytest.raises(spx.SpxError) as e:
            srv.submit(bad, b)
        assert e.value.status == spx.ERR_RANGE
        rp = A.rowptr.copy()
        rp[3] = rp[4] + 1
        with pytest.raises(spx.SpxError) as e:
            srv.submit(S.CSR(A.n, rp, A.col, A.val), b)
        assert e.value.status == spx.ERR_FORMAT
        col = A.col.copy()
        col[1] = col[0]
        with pytest.raises(spx.SpxError) as e:
            srv.submit(S.CSR(A.n, A.rowptr, col, A.val), b)
        assert e.value.status == spx.ERR_DUPLICATE
        assert srv.stats()["submitted"] == 0
        t = srv.submit(A, b, tol=1e-8)
        _, info = srv.wait(t)
        assert info["status"] == spx.OK
    finally:
        srv.close()

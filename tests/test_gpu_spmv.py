"""GPU parity of the SpMV kernels (CSR, COO, ELL, HYB; float64, float32,
binary16 values) against the CPU oracle's Dot2-accurate product, through the
C ABI."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from paper_2006_14290_amd import synth as S

from gpu_util import U32, assert_spmv_f64, assert_spmv_low, dev, host

pytestmark = pytest.mark.gpu

spx = pytest.importorskip("paper_2006_14290_amd.spx")


def _round(v, dtype):
    if dtype == "f64":
        return np.asarray(v, np.float64)
    return np.asarray(v, {"f32": np.float32, "f16": np.float16}[dtype]).astype(np.float64)


def _long_and_empty():
    # long rows crossing several LDS passes between many empty rows
    rp = np.concatenate([[0], np.cumsum([0] * 12000 + [9000, 3, 0, 7000] + [1] * 3000 + [0] * 70)])
    n = len(rp) - 1
    rng = np.random.default_rng(9)
    col = np.concatenate([np.sort(rng.choice(n, l, replace=False)) for l in np.diff(rp)]).astype(np.int32)
    return S.CSR(n, rp.astype(np.int32), col, rng.uniform(-1, 1, rp[-1]))


MATS = [
    ("rand_empty_long", lambda: S.random_small(300, 0.03, seed=1, empty_rows=tuple(range(40, 140)),
                                               long_rows=(7, 299))),
    ("poisson64", lambda: S.poisson2d(64)),
    ("stencil27_n30", lambda: S.stencil27_random(30, seed=2)),
    ("zipf_2e4", lambda: S.zipf_matrix(20000, seed=3)),
    ("one_row", lambda: S.random_small(1, 1.0, seed=4)),
    ("ragged_n", lambda: S.random_small(1001, 0.01, seed=5, long_rows=(500,))),
    ("long_and_empty", _long_and_empty),
    ("all_empty", lambda: S.CSR(300, np.zeros(301, np.int32), np.zeros(0, np.int32), np.zeros(0))),
]
IDS = [m[0] for m in MATS]


def _device_matrix(fmt, A, dtype, sv):
    dt = spx.DTYPE_NAMES[dtype]
    if fmt == "csr":  # row-per-subwarp kernel where rows are short and even
        return spx.csr_from_host(A, dt)
    if fmt == "csr_lb":  # no row-length hint: always the load-balanced kernel
        M = spx.csr_from_host(A, dt)
        M.max_row_len = 0
        return M
    if fmt == "coo":
        return spx.coo_from_host(A.n, O.csr_to_coo_rows(A), A.col, A.val, dt)
    if fmt == "ell":
        E = O.csr_to_ell(A, ld=A.n + 3)
        return spx.ell_from_host(A.n, E.K, E.ld, E.col, E.val, dt)
    H = O.csr_to_hyb(A, sv=sv)
    return spx.hyb_from_host(A.n, H.ell.K, H.ell.ld, H.ell.col, H.ell.val, H.row, H.col, H.val, dt)


@pytest.mark.parametrize("fmt", ["csr", "csr_lb", "coo", "ell", "hyb"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
@pytest.mark.parametrize("mi", range(len(MATS)), ids=IDS)
def test_spmv_parity(fmt, dtype, mi):
    name, make = MATS[mi]
    A = make()
    if fmt == "ell" and name in ("long_and_empty", "zipf_2e4") and dtype != "f64":
        pytest.skip("padded ELL of a 9000-long row: covered once in float64")
    print(f"case {name} {fmt} {dtype}", flush=True)
    sv = {"f64": 8, "f32": 4, "f16": 2}[dtype]
    Ad = _device_matrix(fmt, A, dtype, sv)
    x = S.uniform_vector(A.n, seed=11)
    xr = _round(x, "f64" if dtype == "f64" else "f32")
    Ar = S.CSR(A.n, A.rowptr, A.col, _round(A.val, dtype))
    yref, absax = O.csr_spmv_dot2(Ar, xr)
    xd = dev(xr, Ad.vec_dtype)
    y = host(spx.spmv(Ad, xd))
    if dtype == "f64":
        assert_spmv_f64(y, yref, absax)
    else:
        assert_spmv_low(y, yref, absax, np.diff(A.rowptr))


@pytest.mark.parametrize("fmt", ["csr", "csr_lb", "coo", "ell", "hyb"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_spmv_alpha_beta(fmt, dtype):
    A = S.random_small(700, 0.02, seed=6, empty_rows=(3, 4, 5, 699), long_rows=(100,))
    sv = {"f64": 8, "f32": 4}[dtype]
    Ad = _device_matrix(fmt, A, dtype, sv)
    x = _round(S.uniform_vector(A.n, seed=1), dtype)
    y0 = _round(S.uniform_vector(A.n, seed=2), dtype)
    Ar = S.CSR(A.n, A.rowptr, A.col, _round(A.val, dtype))
    yref, absax = O.csr_spmv_dot2(Ar, x, y0, alpha=-2.5, beta=0.75)
    y = host(spx.spmv(Ad, dev(x, Ad.vec_dtype), dev(y0, Ad.vec_dtype), alpha=-2.5, beta=0.75))
    if dtype == "f64":
        assert_spmv_f64(y, yref, 2.5 * absax, beta_y=0.75 * y0)
    else:
        assert_spmv_low(y, yref, 2.5 * absax, np.diff(A.rowptr), beta_y=0.75 * y0)
    # beta == 0: y is write-only, NaN does not propagate
    ynan = torch.full((A.n,), float("nan"), dtype=Ad.vec_dtype, device="cuda")
    y = host(spx.spmv(Ad, dev(x, Ad.vec_dtype), ynan, alpha=1.0, beta=0.0))
    assert np.all(np.isfinite(y))


@pytest.mark.parametrize("mi", range(len(MATS)), ids=IDS)
def test_csr_analysed_partition(mi):
    """The precomputed partition gives the same tiles as the in-kernel search,
    hence bitwise the same result, and it matches the oracle."""
    name, make = MATS[mi]
    A = make()
    Ad = spx.csr_from_host(A, spx.F64)
    Ad.max_row_len = 0  # the partition belongs to the load-balanced kernel
    x = S.uniform_vector(A.n, seed=4)
    xd = dev(x)
    y0 = host(spx.spmv(Ad, xd))
    spx.csr_analyse(Ad)
    part = host(Ad.csr_part)
    # partition pins: tile k starts at the first row whose offset is >= 2048*k
    ntiles = max(1, -(-A.nnz // 2048))
    rp = A.rowptr.astype(np.int64)
    for k in range(ntiles + 1):
        row = A.n if k == ntiles else int(np.searchsorted(rp, 2048 * k, side="left"))
        assert part[2 * k] == row and part[2 * k + 1] == rp[row], k
    y1 = host(spx.spmv(Ad, xd))
    np.testing.assert_array_equal(y0.view(np.uint64), y1.view(np.uint64))
    yref, absax = O.csr_spmv_dot2(A, x)
    assert_spmv_f64(y1, yref, absax)


@pytest.mark.parametrize("make", [lambda: S.zipf_matrix(30000, seed=8), lambda: S.stencil27_random(40, seed=8)],
                         ids=["zipf_load_balanced", "stencil27_rows"])
def test_csr_bitwise_reproducible(make):
    A = make()
    Ad = spx.csr_from_host(A, spx.F64)
    xd = dev(S.uniform_vector(A.n, seed=3))
    y1 = host(spx.spmv(Ad, xd, csr_only=True))
    y2 = host(spx.spmv(Ad, xd, csr_only=True))
    np.testing.assert_array_equal(y1.view(np.uint64), y2.view(np.uint64))


def test_csr_row_hint_too_small_still_correct():
    """max_row_len is only a hint: a wrong (too small) value selects the
    row-per-subwarp kernel for rows longer than its first chunk, which must
    still be exact to the tolerance."""
    A = S.random_small(500, 0.05, seed=21, long_rows=(17, 300))
    Ad = spx.csr_from_host(A, spx.F64)
    Ad.max_row_len = 8
    x = S.uniform_vector(A.n, seed=2)
    y = host(spx.spmv(Ad, dev(x)))
    yref, absax = O.csr_spmv_dot2(A, x)
    assert_spmv_f64(y, yref, absax)


def test_stencil_closed_form_on_gpu():
    # (A*1)_i = 0 at interior rows of the isotropic Poisson operator, exactly
    A = S.poisson3d_7pt(40)
    for fmt in ("csr", "coo", "ell", "hyb"):
        Ad = _device_matrix(fmt, A, "f64", 8)
        y = host(spx.spmv(Ad, torch.ones(A.n, dtype=torch.float64, device="cuda")))
        lens = np.diff(A.rowptr)
        assert np.all(y[lens == 7] == 0.0), fmt
        assert np.all(y[lens == 4] == 3.0), fmt  # corners miss 3 neighbours


def test_error_paths():
    A = spx.csr_from_host(S.poisson2d(8))
    x = torch.zeros(A.nrows, dtype=torch.float64, device="cuda")
    with pytest.raises(spx.SpxError, match="aliases"):
        spx.spmv(A, x, x)
    bad = spx.csr_from_host(S.poisson2d(8))
    bad.dtype = 7
    y = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    st = spx._lib.spx_spmv(ctypes.byref(bad.desc()), x.data_ptr(), y.data_ptr(), 1.0, 0.0, None)
    assert st == spx.ERR_ARG and b"val_type" in spx._lib.spx_last_error()
    coo = spx.coo_from_host(4, np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.ones(2))
    coo.rowidx = None
    st = spx._lib.spx_spmv(ctypes.byref(coo.desc()), x.data_ptr(), y.data_ptr(), 1.0, 0.0, None)
    assert st == spx.ERR_ARG
    with pytest.raises(spx.SpxError, match="not CSR"):
        spx.spmv(spx.coo_from_host(4, np.array([0], np.int32), np.array([0], np.int32), np.ones(1)),
                 x[:4], y[:4], csr_only=True)


# ------------------------------------------------------------------ full size
@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_27pt_all_formats(dtype):
    """27-point stencil on 100^3 (n = 1e6, nnz = 26,463,592), uniform[-1,1)
    values, every format, compared row by row with the oracle."""
    print(f"case 27pt-100^3 {dtype}", flush=True)
    A = S.stencil27_random(100, seed=0)
    assert A.nnz == 26463592
    x = S.uniform_vector(A.n, seed=0)
    sv = 8 if dtype == "f64" else 4
    xr = _round(x, dtype)
    Ar = S.CSR(A.n, A.rowptr, A.col, _round(A.val, dtype))
    yref, absax = O.csr_spmv_dot2(Ar, xr)
    for fmt in ("csr", "coo", "ell", "hyb"):
        Ad = _device_matrix(fmt, A, dtype, sv)
        y = host(spx.spmv(Ad, dev(xr, Ad.vec_dtype)))
        if dtype == "f64":
            assert_spmv_f64(y, yref, absax)
        else:
            assert_spmv_low(y, yref, absax, np.diff(A.rowptr))
        del Ad
        torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_full_size_zipf_csr_coo_hyb():
    """Zipf(1.5) row lengths clipped to [1, 10000], n = 1e6 (nnz ~ 1.5e8),
    float64; CSR, COO and HYB (auto width) compared row by row."""
    print("case zipf-1e6 f64", flush=True)
    A = S.zipf_matrix(10**6, seed=0)
    x = S.uniform_vector(A.n, seed=0)
    yref, absax = O.csr_spmv_dot2(A, x)
    for fmt in ("csr", "coo", "hyb"):
        Ad = _device_matrix(fmt, A, "f64", 8)
        y = host(spx.spmv(Ad, dev(x)))
        assert_spmv_f64(y, yref, absax)
        del Ad
        torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_full_size_zipf_ell_int64_slots():
    """The Zipf(1.5) matrix (n = 1e6, longest rows 10,000 entries) in ELL:
    1e10 slots, so every slot offset is past 2^31 for most slot columns.
    Device CSR -> ELL -> CSR round trip compared bitwise on the host, the
    ELL slots of every 10,000-entry row and of a row sample checked against
    the canonical layout, and the ELL product compared row by row with the
    oracle."""
    print("case zipf-1e6 ell f64 (1e10 slots)", flush=True)
    A = S.zipf_matrix(10**6, seed=0)
    lens = np.diff(A.rowptr)
    long_rows = np.flatnonzero(lens == 10000)
    assert long_rows.size > 1000
    x = S.uniform_vector(A.n, seed=0)
    yref, absax = O.csr_spmv_dot2(A, x)
    Ad = spx.csr_from_host(A)
    E = spx.convert(Ad, spx.ELL)
    K, ld = E.ell_width, E.ell_ld
    assert K == 10000 and K * ld > 2 ** 31
    y = host(spx.spmv(E, dev(x)))
    assert_spmv_f64(y, yref, absax)
    rows = np.unique(np.concatenate([long_rows, S.rng(5, "x").choice(A.n, 4000, replace=False)]))
    ri = torch.from_numpy(rows).cuda()
    ecol = host(E.ell_col.view(K, ld)[:, ri])
    evbits = host(E.ell_val.view(K, ld)[:, ri]).view(np.uint64)
    for j, i in enumerate(rows):
        a, L = A.rowptr[i], lens[i]
        np.testing.assert_array_equal(ecol[:L, j], A.col[a:a + L])
        assert np.all(ecol[L:, j] == -1)
        np.testing.assert_array_equal(evbits[:L, j], A.val[a:a + L].view(np.uint64))
        assert np.all(evbits[L:, j] == 0)
    del ecol, evbits
    B = spx.convert(E, spx.CSR)
    del E
    np.testing.assert_array_equal(host(B.rowptr), A.rowptr)
    np.testing.assert_array_equal(host(B.colidx), A.col)
    np.testing.assert_array_equal(host(B.vals).view(np.uint64), A.val.view(np.uint64))
    del B, Ad
    torch.cuda.empty_cache()

"""The column-blocked CSR product (spx_csr_colblock: 8 column ranges, one per
XCD, partial row sums added in block order) against the oracle's
Dot2-accurate product, row by row, through the C ABI; its layout against
the definition (each block holds A's entries of its column range, in A's
order); bitwise reproducibility; the full-size Zipf(1.5) matrix."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2006_14290_amd import synth as S

from gpu_util import assert_spmv_f64, assert_spmv_low, dev, host

pytestmark = pytest.mark.gpu

spx = pytest.importorskip("paper_2006_14290_amd.spx")


def _one_block():
    # every column in the first of the 8 ranges: seven empty blocks
    rng = np.random.default_rng(3)
    n = 4000
    rows = [np.sort(rng.choice(n // 8, rng.integers(0, 9), replace=False)) for _ in range(n)]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    return S.CSR(n, rp, np.concatenate(rows).astype(np.int32), rng.uniform(-1, 1, rp[-1]))


MATS = [
    ("zipf_2e4", lambda: S.zipf_matrix(20000, seed=3)),
    ("stencil27_n24", lambda: S.stencil27_random(24, seed=2)),
    ("rand_empty_long", lambda: S.random_small(300, 0.03, seed=1, empty_rows=tuple(range(40, 140)),
                                               long_rows=(7, 299))),
    ("narrow_n5", lambda: S.random_small(5, 1.0, seed=8)),  # fewer columns than blocks
    ("one_row", lambda: S.random_small(1, 1.0, seed=4)),
    ("one_block", _one_block),
    ("all_empty", lambda: S.CSR(300, np.zeros(301, np.int32), np.zeros(0, np.int32), np.zeros(0))),
]
IDS = [m[0] for m in MATS]


def _round(v, dtype):
    if dtype == "f64":
        return np.asarray(v, np.float64)
    return np.asarray(v, {"f32": np.float32, "f16": np.float16}[dtype]).astype(np.float64)


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
@pytest.mark.parametrize("mi", range(len(MATS)), ids=IDS)
def test_colblock_parity(dtype, mi):
    name, make = MATS[mi]
    A = make()
    print(f"case colblock {name} {dtype}", flush=True)
    Ad = spx.csr_colblock(spx.csr_from_host(A, spx.DTYPE_NAMES[dtype]))
    x = S.uniform_vector(A.n, seed=11)
    xr = _round(x, "f64" if dtype == "f64" else "f32")
    Ar = S.CSR(A.n, A.rowptr, A.col, _round(A.val, dtype))
    yref, absax = O.csr_spmv_dot2(Ar, xr)
    y = host(spx.spmv(Ad, dev(xr, Ad.vec_dtype)))
    if dtype == "f64":
        assert_spmv_f64(y, yref, absax)
    else:
        # each row is summed in at most 8 block partials: the row-length bound
        # plus 8 further additions
        assert_spmv_low(y, yref, absax, np.diff(A.rowptr) + 8)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_colblock_alpha_beta(dtype):
    A = S.random_small(700, 0.02, seed=6, empty_rows=(3, 4, 5, 699), long_rows=(100,))
    Ad = spx.csr_colblock(spx.csr_from_host(A, spx.DTYPE_NAMES[dtype]))
    x = _round(S.uniform_vector(A.n, seed=1), dtype)
    y0 = _round(S.uniform_vector(A.n, seed=2), dtype)
    Ar = S.CSR(A.n, A.rowptr, A.col, _round(A.val, dtype))
    yref, absax = O.csr_spmv_dot2(Ar, x, y0, alpha=-2.5, beta=0.75)
    y = host(spx.spmv(Ad, dev(x, Ad.vec_dtype), dev(y0, Ad.vec_dtype), alpha=-2.5, beta=0.75))
    if dtype == "f64":
        assert_spmv_f64(y, yref, 2.5 * absax, beta_y=0.75 * y0)
    else:
        assert_spmv_low(y, yref, 2.5 * absax, np.diff(A.rowptr) + 8, beta_y=0.75 * y0)
    ynan = torch.full((A.n,), float("nan"), dtype=Ad.vec_dtype, device="cuda")
    y = host(spx.spmv(Ad, dev(x, Ad.vec_dtype), ynan, alpha=1.0, beta=0.0))
    assert np.all(np.isfinite(y))


def _a256(b):
    return (b + 255) // 256 * 256


def test_colblock_layout():
    """Block b of the copy holds exactly A's entries with column in
    [b*W, (b+1)*W), W = ceil(n/8), in A's row-major order, values bit for bit;
    its row pointer starts at 0 and counts them per row."""
    A = S.zipf_matrix(20000, seed=5)
    n, nnz = A.n, A.nnz
    Ad = spx.csr_colblock(spx.csr_from_host(A))
    buf = host(Ad.csr_cb)
    W = -(-n // 8)
    table = buf[:256].view(np.int64)
    base, bnnz = table[:9], table[9:17]
    off_rp = 256
    ntiles = max(1, -(-nnz // 2048))
    off_part = off_rp + _a256(8 * (n + 1) * 4)
    off_p = off_part + _a256(8 * 2 * (ntiles + 1) * 4)
    off_col = off_p + _a256(8 * n * 8)
    off_val = off_col + _a256((nnz + 128) * 4)
    brp = buf[off_rp:off_rp + 8 * (n + 1) * 4].view(np.int32).reshape(8, n + 1)
    col = buf[off_col:off_col + (nnz + 128) * 4].view(np.int32)
    val = buf[off_val:off_val + (nnz + 128) * 8].view(np.uint64)
    rows = np.repeat(np.arange(n), np.diff(A.rowptr))
    blk = A.col // W
    assert int(bnnz.sum()) == nnz
    for b in range(8):
        sel = np.flatnonzero(blk == b)
        assert bnnz[b] == sel.size and base[b] % 16 == 0
        np.testing.assert_array_equal(brp[b], np.concatenate([[0], np.cumsum(np.bincount(rows[sel], minlength=n))]))
        np.testing.assert_array_equal(col[base[b]:base[b] + sel.size], A.col[sel])
        np.testing.assert_array_equal(val[base[b]:base[b] + sel.size], A.val[sel].view(np.uint64))
    assert Ad.csr_cb_live == 0xFF


def test_colblock_reproducible_and_close_to_plain():
    A = S.zipf_matrix(30000, seed=7)
    x = dev(S.uniform_vector(A.n, seed=2))
    plain = spx.csr_from_host(A)
    Ad = spx.csr_colblock(spx.csr_from_host(A))
    y1, y2 = host(spx.spmv(Ad, x)), host(spx.spmv(Ad, x))
    np.testing.assert_array_equal(y1.view(np.uint64), y2.view(np.uint64))
    yp = host(spx.spmv(plain, x))
    _, absax = O.csr_spmv_dot2(A, host(x))
    assert np.all(np.abs(y1 - yp) <= 2e-14 * absax)


def test_colblock_errors():
    A = S.poisson2d(20)
    Ad = spx.csr_from_host(A)
    d = Ad.desc()
    need = spx._lib.spx_csr_colblock_bytes(d)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    st = spx._lib.spx_csr_colblock(d, spx._ptr(small), small.numel(), spx._stream())
    assert st == spx.ERR_ARG
    E = spx.convert(Ad, spx.ELL)
    with pytest.raises(spx.SpxError, match="ERR_ARG"):
        spx.csr_colblock(E)
    # columns out of order: the blocks' counts still add up (no fault), and
    # spx_validate is the check that reports it
    bad = S.CSR(A.n, A.rowptr, A.col.copy(), A.val)
    bad.col[[5, 6]] = bad.col[[6, 5]]
    Bd = spx.csr_from_host(bad)
    assert spx.validate(Bd) == spx.ERR_UNSORTED


@pytest.mark.timeout(900)
def test_full_size_zipf_colblock():
    """Zipf(1.5) n = 1e6 (rows clipped to 10,000): every row against the oracle."""
    print("case zipf-1e6 colblock f64", flush=True)
    A = S.zipf_matrix(10**6, seed=0)
    x = S.uniform_vector(A.n, seed=0)
    yref, absax = O.csr_spmv_dot2(A, x)
    Ad = spx.csr_colblock(spx.csr_analyse(spx.csr_from_host(A)))
    y = host(spx.spmv(Ad, dev(x)))
    assert_spmv_f64(y, yref, absax)
    del Ad
    torch.cuda.empty_cache()

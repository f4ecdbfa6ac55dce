"""GPU parity of the subwarp primitives (Section 3.3) against the oracle's
subwarp model: the butterfly sums must match bit for bit (the DPP steps pair
the same values as the xor butterfly), ballot/any/all exactly, and the
segmented scan within rounding (exactly on integer data)."""
import numpy as np
import pytest
import torch

import oracle as O

from gpu_util import dev, host

pytestmark = pytest.mark.gpu

spx = pytest.importorskip("paper_2006_14290_amd.spx")

SIZES = [1, 2, 4, 8, 16, 32, 64]


@pytest.mark.parametrize("size", SIZES)
def test_subwarp_sum_bitwise(size):
    rng = np.random.default_rng(size)
    data = rng.standard_normal(64 * 37) * np.exp(rng.uniform(-20, 20, 64 * 37))
    ref, steps = O.subwarp_reduce(data, size)
    assert steps == int(np.log2(size))
    out = host(spx.subwarp_sum(dev(data), size))
    np.testing.assert_array_equal(out.view(np.uint64), ref.view(np.uint64))


@pytest.mark.parametrize("size", [4, 64])
def test_subwarp_sum_inner_loops(size):
    data = np.arange(256, dtype=np.float64)
    ref = data.copy()
    for _ in range(3):
        ref, _ = O.subwarp_reduce(ref, size)
    out = host(spx.subwarp_sum(dev(data), size, inner_loops=3))
    np.testing.assert_array_equal(out, ref)


@pytest.mark.parametrize("size", SIZES)
def test_subwarp_vote_exact(size):
    rng = np.random.default_rng(100 + size)
    pred = (rng.random(64 * 9) < 0.5).astype(np.int32)
    pred[64:128] = 1
    pred[128:192] = 0
    b, a, l = O.subwarp_vote(pred, size)
    gb, ga, gl = spx.subwarp_vote(dev(pred), size)
    np.testing.assert_array_equal(host(gb).view(np.uint64), b)
    np.testing.assert_array_equal(host(ga), a)
    np.testing.assert_array_equal(host(gl), l)


def test_segscan_exact_on_integers_and_close_on_floats():
    rng = np.random.default_rng(7)
    n = 64 * 50
    head = (rng.random(n) < 0.15).astype(np.int32)
    head[64 * 3:64 * 4] = 0   # one wave with a single segment
    head[64 * 4:64 * 5] = 1   # one wave where every lane starts a segment
    ints = rng.integers(-1000, 1000, n).astype(np.float64)
    ref = O.segmented_scan(ints, head, 64)
    out = host(spx.wave_segscan(dev(ints), dev(head)))
    np.testing.assert_array_equal(out, ref)
    fl = rng.uniform(-1, 1, n)
    ref = O.segmented_scan(fl, head, 64)
    absref = O.segmented_scan(np.abs(fl), head, 64)
    out = host(spx.wave_segscan(dev(fl), dev(head)))
    assert np.all(np.abs(out - ref) <= 64 * 2.0 ** -53 * absref)


@pytest.mark.parametrize("n", [1, 2, 4095, 4096, 4097, 1_000_003])
def test_stream_copy(n):
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.full_like(x, float("nan"))
    spx.stream_copy(x, y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


def test_stream_read_writes_nothing():
    x = torch.randn(1_000_002, dtype=torch.float64, device="cuda")
    sink = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    spx.stream_read(x, sink)
    torch.cuda.synchronize()
    assert float(sink[0]) == 7.0

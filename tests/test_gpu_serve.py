"""Batched CG (one work-group per system) and the continuous-batching server:
every result meets the tolerance through the oracle's true residual, and a
system's solution is bitwise the same alone, in a batch, and in the served
mix (however its iterations are split across ticks). Admission, budget,
queueing, slot reuse and cancellation are exercised."""
import time

import numpy as np
import pytest
import torch

import oracle as O
from paper_2006_14290_amd import synth as S

from gpu_util import dev, host

pytestmark = pytest.mark.gpu

spx = pytest.importorskip("paper_2006_14290_amd.spx")


def _system(kind, size, seed):
    A = S.poisson2d(size) if kind == "poisson" else S.spd_diag_dominant(size, seed=seed)
    xs = S.uniform_vector(A.n, seed=seed, purpose="xstar")
    b, _ = O.csr_spmv_dot2(A, xs)
    return A, b


MIX = [("poisson", 32, 1), ("spd", 1000, 2), ("poisson", 47, 3), ("spd", 5000, 4), ("poisson", 64, 5),
       ("spd", 20000, 6), ("poisson", 90, 7), ("spd", 1500, 8), ("poisson", 33, 9), ("spd", 12345, 10)]


def _relres(A, b, x):
    _, rn = O.residual(A, b, x)
    return rn / np.linalg.norm(b)


def _alone(A, b, tol):
    Ad = spx.csr_from_host(A)
    xs, infos = spx.cg_batch([Ad], [dev(b)], tol=tol)
    return host(xs[0]), infos[0]


def test_cg_batch_mix_and_alone_bitwise():
    systems = [_system(*m) for m in MIX]
    mats = [spx.csr_from_host(A) for A, _ in systems]
    bs = [dev(b) for _, b in systems]
    xs, infos = spx.cg_batch(mats, bs, tol=1e-8)
    for (A, b), x, info in zip(systems, xs, infos):
        x = host(x)
        assert info["status"] == spx.OK, info
        assert _relres(A, b, x) <= 1e-8
        xa, ia = _alone(A, b, 1e-8)
        assert ia["iters"] == info["iters"]
        np.testing.assert_array_equal(xa.view(np.uint64), x.view(np.uint64))


def test_cg_batch_one_group_mix_alone_bitwise():
    # the one-work-group kernel for systems above the small-system range, asked
    # for explicitly (by default those systems take the wide path)
    systems = [(A, b) for A, b in (_system(*m) for m in MIX) if A.n > 4096]
    assert len(systems) == 4
    mats = [spx.csr_from_host(A) for A, _ in systems]
    xs, infos = spx.cg_batch(mats, [dev(b) for _, b in systems], tol=1e-8, path=spx.BATCH_ONE_GROUP)
    for (A, b), Ad, x, info in zip(systems, mats, xs, infos):
        assert info["status"] == spx.OK, info
        x = host(x)
        assert _relres(A, b, x) <= 1e-8
        xa, ia = spx.cg_batch([Ad], [dev(b)], tol=1e-8, path=spx.BATCH_ONE_GROUP)
        assert ia[0]["iters"] == info["iters"]
        np.testing.assert_array_equal(host(xa[0]).view(np.uint64), x.view(np.uint64))


def test_cg_batch_matches_oracle_iterations():
    A, b = _system("poisson", 64, 0)
    x, info = _alone(A, b, 1e-10)
    assert info["status"] == spx.OK
    assert _relres(A, b, x) <= 1e-10
    xo, io = O.cg(A, b, tol=1e-10)
    assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5


def test_cg_batch_many_identical_systems():
    """The 64x64 Poisson system 512 times over with different right-hand sides."""
    A = S.poisson2d(64)
    Ad = spx.csr_from_host(A)
    bs = []
    for s in range(512):
        xs = S.uniform_vector(A.n, seed=s, purpose="xstar")
        bs.append(O.csr_spmv_dot2(A, xs)[0])
    xs, infos = spx.cg_batch([Ad] * 512, [dev(b) for b in bs], tol=1e-10)
    for i in (0, 1, 255, 511):
        assert infos[i]["status"] == spx.OK
        assert _relres(A, bs[i], host(xs[i])) <= 1e-10
    assert all(inf["status"] == spx.OK for inf in infos)


def test_server_mix_alone_bitwise_and_stats():
    srv = spx.Server(max_slots=4, hbm_budget_bytes=256 << 20, tick_us=300)
    try:
        systems = [_system(*m) for m in MIX]
        tickets = [srv.submit(A, b, tol=1e-8) for A, b in systems]
        for t, (A, b) in zip(tickets, systems):
            x, info = srv.wait(t, timeout_s=120)
            assert info["status"] == spx.OK, info
            assert _relres(A, b, x) <= 1e-8
            xa, ia = _alone(A, b, 1e-8)
            assert ia["iters"] == info["iters"]
            np.testing.assert_array_equal(xa.view(np.uint64), x.view(np.uint64))
            assert info["device_ms"] > 0
        st = srv.stats()
        assert st["submitted"] == st["completed"] == len(MIX)
        assert st["active"] == 0 and st["queued"] == 0
        assert st["pool_bytes_peak"] <= st["pool_bytes_total"]
        assert st["ticks"] >= 1
    finally:
        srv.close()


def test_server_inflight_bound_fifo_same_bits():
    """A work bound smaller than any request: one system resident at a time,
    admitted in submission order (the queue drains FIFO), each result
    bitwise its solo solve."""
    systems = [_system(*m) for m in MIX[:6]]
    srv = spx.Server(max_slots=8, hbm_budget_bytes=256 << 20, inflight_bytes=1)
    try:
        tickets = [srv.submit(A, b, tol=1e-8) for A, b in systems]
        assert srv.stats()["queued"] >= 1
        done_ms = []
        for t, (A, b) in zip(tickets, systems):
            x, info = srv.wait(t, timeout_s=120)
            assert info["status"] == spx.OK, info
            xa, ia = _alone(A, b, 1e-8)
            np.testing.assert_array_equal(xa.view(np.uint64), x.view(np.uint64))
            done_ms.append(info["device_ms"])
        # submitted together, served one after another: completion times grow
        assert all(b > a for a, b in zip(done_ms, done_ms[1:])), done_ms
        st = srv.stats()
        assert st["active"] == 0 and st["queued"] == 0
    finally:
        srv.close()


def test_server_one_iteration_per_tick_same_bits():
    A, b = _system("poisson", 40, 11)
    srv = spx.Server(max_slots=2, hbm_budget_bytes=64 << 20, iters_per_tick=1)
    try:
        x, info = srv.wait(srv.submit(A, b, tol=1e-8), timeout_s=120)
        assert info["status"] == spx.OK
        xa, _ = _alone(A, b, 1e-8)
        np.testing.assert_array_equal(xa.view(np.uint64), x.view(np.uint64))
        assert srv.stats()["ticks"] >= info["iters"]
    finally:
        srv.close()


def test_server_budget_queueing_and_cancel():
    big = S.poisson2d(128)
    xs = S.uniform_vector(big.n, seed=1, purpose="xstar")
    bbig = O.csr_spmv_dot2(big, xs)[0]
    small, bsmall = _system("poisson", 32, 2)
    # a budget that holds one 128x128 system at a time
    one = 5 * 16384 * 8 + 16385 * 4 + big.nnz * 12 + 8 * 256
    srv = spx.Server(max_slots=8, hbm_budget_bytes=int(one * 1.5), iters_per_tick=5)
    try:
        with pytest.raises(spx.SpxError, match="BUDGET"):
            huge = S.poisson2d(300)
            srv.submit(huge, np.ones(huge.n))
        # a blocker with an unreachable tolerance holds the budget until it is
        # cancelled, so the requests behind it stay queued however fast the
        # others would converge
        blocker = srv.submit(big, bbig, tol=1e-300)
        tickets = [srv.submit(big, bbig, tol=1e-8) for _ in range(3)]
        assert srv.stats()["queued"] >= 3
        # an unreachable tolerance keeps the victim running (or queued) until
        # the cancel arrives, so the cancel must win
        victim = srv.submit(small, bsmall, tol=1e-300)
        time.sleep(0.05)
        srv.cancel(victim)
        x, info = srv.wait(victim, timeout_s=60)
        assert info["status"] == spx.CANCELLED
        # cancelled while still queued behind the budget
        queued = srv.submit(big, bbig, tol=1e-8)
        assert srv.stats()["queued"] >= 4
        srv.cancel(queued)
        x, info = srv.wait(queued, timeout_s=60)
        assert info["status"] == spx.CANCELLED
        p = srv.poll(blocker)
        assert p[1]["status"] == spx.PENDING and srv.stats()["queued"] >= 3
        srv.cancel(blocker)
        x, info = srv.wait(blocker, timeout_s=60)
        assert info["status"] == spx.CANCELLED
        for t in tickets:
            x, info = srv.wait(t, timeout_s=120)
            assert info["status"] == spx.OK
            assert _relres(big, bbig, x) <= 1e-8
        st = srv.stats()
        assert st["pool_bytes_peak"] <= st["pool_bytes_total"]
        assert st["rejected"] == 1
        assert st["completed"] == st["submitted"] == 6
    finally:
        srv.close()


def test_server_failure_ends_every_request():
    # the host makes the worker stop at its 4th tick as if a HIP call had
    # failed (no device fault): resident and queued requests must all end
    # with SPX_ERR_HIP, none may stay pending, later submissions are refused
    A, b = _system("poisson", 96, 3)
    srv = spx.Server(max_slots=2, hbm_budget_bytes=64 << 20, iters_per_tick=2, debug_fail_tick=4)
    try:
        tickets = [srv.submit(A, b, tol=1e-10) for _ in range(6)]
        for t in tickets:
            _, info = srv.wait(t, timeout_s=60)
            assert info["status"] == spx.ERR_HIP, info
        with pytest.raises(spx.SpxError, match="HIP"):
            srv.submit(A, b)
        st = srv.stats()
        assert st["completed"] == st["submitted"] == 6
        assert st["active"] == 0 and st["queued"] == 0 and st["pool_bytes_in_use"] == 0
    finally:
        srv.close()


def test_server_destroy_cancels_resident_requests():
    A, b = _system("poisson", 96, 4)
    srv = spx.Server(max_slots=2, hbm_budget_bytes=64 << 20, iters_per_tick=1)
    for _ in range(4):
        srv.submit(A, b, tol=1e-300)
    time.sleep(0.05)
    srv.close()  # must return: the worker ends every resident and queued request


def test_server_poll_and_slot_reuse():
    srv = spx.Server(max_slots=2, hbm_budget_bytes=64 << 20)
    try:
        systems = [_system("spd", 2000 + 100 * i, i) for i in range(10)]
        tickets = [srv.submit(A, b, tol=1e-8) for A, b in systems]
        pending = set(tickets)
        t0 = time.time()
        results = {}
        while pending and time.time() - t0 < 120:
            for t in list(pending):
                x, info = srv.poll(t)
                if info["status"] != spx.PENDING:
                    results[t] = (x, info)
                    pending.discard(t)
            time.sleep(0.001)
        assert not pending
        for t, (A, b) in zip(tickets, systems):
            x, info = results[t]
            assert info["status"] == spx.OK
            assert _relres(A, b, x) <= 1e-8
    finally:
        srv.close()


# ---------------------------------------------------------------- wide systems
WIDE_MIX = [("poisson", 160, 21), ("spd", 50000, 22), ("poisson", 40, 23), ("spd", 17000, 24), ("poisson", 129, 25)]


def test_cg_batch_wide_converges_like_oracle():
    for kind, size, seed in [("poisson", 160, 1), ("spd", 60000, 2)]:
        A, b = _system(kind, size, seed)
        assert A.n >= 16384
        x, info = _alone(A, b, 1e-10)
        assert info["status"] == spx.OK, info
        assert _relres(A, b, x) <= 1e-10
        _, io = O.cg(A, b, tol=1e-10)
        assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5


def test_cg_batch_wide_and_one_group_agree():
    A, b = _system("poisson", 130, 3)
    Ad = spx.csr_from_host(A)
    xw, iw = spx.cg_batch([Ad], [dev(b)], tol=1e-9, path=spx.BATCH_WIDE)
    xn, inn = spx.cg_batch([Ad], [dev(b)], tol=1e-9, path=spx.BATCH_ONE_GROUP)
    assert iw[0]["status"] == inn[0]["status"] == spx.OK
    for x in (host(xw[0]), host(xn[0])):
        assert _relres(A, b, x) <= 1e-9
    assert abs(iw[0]["iters"] - inn[0]["iters"]) <= 5


def test_cg_batch_wide_mix_alone_bitwise():
    systems = [_system(*m) for m in WIDE_MIX]
    mats = [spx.csr_from_host(A) for A, _ in systems]
    xs, infos = spx.cg_batch(mats, [dev(b) for _, b in systems], tol=1e-8)
    for (A, b), x, info in zip(systems, xs, infos):
        assert info["status"] == spx.OK, info
        x = host(x)
        assert _relres(A, b, x) <= 1e-8
        xa, ia = _alone(A, b, 1e-8)
        assert ia["iters"] == info["iters"]
        np.testing.assert_array_equal(xa.view(np.uint64), x.view(np.uint64))


def test_cg_batch_wide_status_codes():
    n = 20000
    # indefinite diagonal: p.A p <= 0 at some step
    d = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    rowptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    mk = lambda vals: spx.csr_from_host(S.CSR(n, rowptr, col, vals.astype(np.float64)))
    b = np.ones(n)
    _, inf = spx.cg_batch([mk(d)], [dev(b)], tol=1e-10, path=spx.BATCH_WIDE)
    assert inf[0]["status"] == spx.ERR_BREAKDOWN
    bn = b.copy()
    bn[7] = np.nan
    _, inf = spx.cg_batch([mk(np.ones(n))], [dev(bn)], tol=1e-10, path=spx.BATCH_WIDE)
    assert inf[0]["status"] == spx.ERR_NONFINITE
    xs, inf = spx.cg_batch([mk(np.ones(n))], [dev(np.zeros(n))], tol=1e-10, path=spx.BATCH_WIDE)
    assert inf[0]["status"] == spx.OK and inf[0]["iters"] == 0
    assert not host(xs[0]).any()
    A, bb = _system("poisson", 150, 4)
    _, inf = spx.cg_batch([spx.csr_from_host(A)], [dev(bb)], tol=1e-12, maxit=3, path=spx.BATCH_WIDE)
    assert inf[0]["status"] == spx.ERR_NOT_CONVERGED and inf[0]["iters"] == 3


def test_cg_batch_wide_true_residual_restarts():
    """A tolerance below the attainable accuracy: the recursive residual keeps
    passing it, each true-residual check fails and the recurrences restart
    from the true residual, until maxit; the iterate stays accurate."""
    A, b = _system("poisson", 130, 1)
    xs, inf = spx.cg_batch([spx.csr_from_host(A)], [dev(b)], tol=1e-17, maxit=800, path=spx.BATCH_WIDE)
    assert inf[0]["status"] == spx.ERR_NOT_CONVERGED and inf[0]["iters"] == 800, inf
    # one product per step; each failed check adds two (the product whose
    # step was not taken, and the check's), the stop at maxit one more
    assert inf[0]["spmv_count"] >= inf[0]["iters"] + 5, inf
    assert _relres(A, b, host(xs[0])) <= 1e-14


def test_server_wide_and_narrow_mix_bitwise():
    srv = spx.Server(max_slots=6, hbm_budget_bytes=512 << 20, tick_us=500)
    try:
        systems = [_system(*m) for m in WIDE_MIX + MIX[:4]]
        tickets = [srv.submit(A, b, tol=1e-8) for A, b in systems]
        for t, (A, b) in zip(tickets, systems):
            x, info = srv.wait(t, timeout_s=120)
            assert info["status"] == spx.OK, info
            assert _relres(A, b, x) <= 1e-8
            xa, ia = _alone(A, b, 1e-8)
            assert ia["iters"] == info["iters"]
            np.testing.assert_array_equal(xa.view(np.uint64), x.view(np.uint64))
    finally:
        srv.close()


def test_server_all_one_group_when_wide_disabled():
    A, b = _system("poisson", 130, 5)
    srv = spx.Server(max_slots=2, hbm_budget_bytes=64 << 20, wide_min_rows=-1)
    try:
        x, info = srv.wait(srv.submit(A, b, tol=1e-8), timeout_s=120)
        assert info["status"] == spx.OK
        Ad = spx.csr_from_host(A)
        xs, _ = spx.cg_batch([Ad], [dev(b)], tol=1e-8, path=spx.BATCH_ONE_GROUP)
        np.testing.assert_array_equal(host(xs[0]).view(np.uint64), x.view(np.uint64))
    finally:
        srv.close()


# ---------------------------------------------------------------- nonsymmetric requests
NONSYM = [(12, 21), (20, 22), (28, 23), (36, 24)]  # convection-diffusion N^3: n = 1,728 .. 46,656


def _nonsym(N, seed):
    A = S.convdiff3d_upwind(N)
    xs = S.uniform_vector(A.n, seed=seed, purpose="xstar")
    b, _ = O.csr_spmv_dot2(A, xs)
    return A, b


def _served_alone(A, b, solver, **cfg):
    srv = spx.Server(max_slots=2, hbm_budget_bytes=256 << 20, **cfg)
    try:
        return srv.wait(srv.submit(A, b, tol=1e-8, solver=solver), timeout_s=120)
    finally:
        srv.close()


def test_server_bicgstab_alone_mix_bitwise_and_oracle():
    """Nonsymmetric (upwind convection-diffusion) systems served by BiCGSTAB
    next to CG systems: each meets 1e-8 through the oracle's true residual,
    takes about the oracle's BiCGSTAB iteration count, and is bitwise the
    same served alone, in the mix, and with one iteration per tick."""
    systems = [_nonsym(N, s) for N, s in NONSYM]
    alone = [_served_alone(A, b, spx.SOLVER_BICGSTAB) for A, b in systems]
    cg = [_system(*m) for m in MIX[:6]]
    srv = spx.Server(max_slots=5, hbm_budget_bytes=512 << 20, tick_us=300)
    try:
        order = []
        for i in range(max(len(systems), len(cg))):
            if i < len(cg):
                order.append(("cg", i, srv.submit(*cg[i], tol=1e-8)))
            if i < len(systems):
                order.append(("bi", i, srv.submit(*systems[i], tol=1e-8, solver=spx.SOLVER_BICGSTAB)))
        for kind, i, t in order:
            x, info = srv.wait(t, timeout_s=120)
            assert info["status"] == spx.OK, (kind, i, info)
            A, b = (systems if kind == "bi" else cg)[i]
            assert _relres(A, b, x) <= 1e-8
            if kind == "bi":
                xa, ia = alone[i]
                assert ia["iters"] == info["iters"]
                np.testing.assert_array_equal(xa.view(np.uint64), x.view(np.uint64))
                _, io = O.bicgstab(A, b, tol=1e-8)
                assert io["status"] == O.OK
                assert abs(info["iters"] - io["iters"]) <= 0.1 * io["iters"] + 5, (info["iters"], io["iters"])
                assert info["spmv_count"] >= 2 * info["iters"] - 1
            else:
                xa, _ = _alone(A, b, 1e-8)
                np.testing.assert_array_equal(xa.view(np.uint64), x.view(np.uint64))
    finally:
        srv.close()
    # one BiCGSTAB step per tick: the state carried between launches gives the same bits
    A, b = systems[1]
    x1, i1 = _served_alone(A, b, spx.SOLVER_BICGSTAB, iters_per_tick=1)
    assert i1["status"] == spx.OK and i1["iters"] == alone[1][1]["iters"]
    np.testing.assert_array_equal(x1.view(np.uint64), alone[1][0].view(np.uint64))


def test_server_bicgstab_wide_and_one_group_agree():
    """Large nonsymmetric requests take the wide path (three product + vector
    pairs per BiCGSTAB step); the one-work-group path (wide path switched
    off) solves the same systems in about as many steps."""
    for N, seed in NONSYM[1:]:
        A, b = _nonsym(N, seed)
        assert A.n > 4096
        xw, iw = _served_alone(A, b, spx.SOLVER_BICGSTAB)
        xn, inn = _served_alone(A, b, spx.SOLVER_BICGSTAB, wide_min_rows=-1)
        assert iw["status"] == inn["status"] == spx.OK, (iw, inn)
        for x in (xw, xn):
            assert _relres(A, b, x) <= 1e-8
        assert abs(iw["iters"] - inn["iters"]) <= 0.1 * inn["iters"] + 5, (iw, inn)
        assert iw["spmv_count"] >= 2 * iw["iters"] - 1


def test_server_bicgstab_wide_status_codes():
    A, b = _nonsym(28, 5)
    srv = spx.Server(max_slots=4, hbm_budget_bytes=256 << 20)
    try:
        t1 = srv.submit(A, b, tol=1e-12, maxit=3, solver=spx.SOLVER_BICGSTAB)
        t2 = srv.submit(A, np.zeros(A.n), tol=1e-8, solver=spx.SOLVER_BICGSTAB)
        bn = b.copy()
        bn[11] = np.nan
        t3 = srv.submit(A, bn, tol=1e-8, solver=spx.SOLVER_BICGSTAB)
        _, i1 = srv.wait(t1, timeout_s=60)
        assert i1["status"] == spx.ERR_NOT_CONVERGED and i1["iters"] == 3, i1
        x2, i2 = srv.wait(t2, timeout_s=60)
        assert i2["status"] == spx.OK and i2["iters"] == 0 and not x2.any(), i2
        _, i3 = srv.wait(t3, timeout_s=60)
        assert i3["status"] == spx.ERR_NONFINITE, i3
    finally:
        srv.close()


def test_server_bicgstab_solves_spd_and_refuses_other_solvers():
    A, b = _system("spd", 3000, 31)
    x, info = _served_alone(A, b, spx.SOLVER_BICGSTAB)
    assert info["status"] == spx.OK and _relres(A, b, x) <= 1e-8
    srv = spx.Server(max_slots=2, hbm_budget_bytes=64 << 20)
    try:
        with pytest.raises(spx.SpxError, match="ERR_ARG"):
            srv.submit(A, b, solver=spx.SOLVER_GMRES)
        assert srv.stats()["submitted"] == 0
    finally:
        srv.close()

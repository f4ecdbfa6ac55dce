#!/usr/bin/env python3
"""Benchmark of the SpMV + Krylov hot path on one MI355X.

Headline workload (one "step"): y = A x on the 27-point stencil of a 100^3
grid (n = 1e6, nnz = 26,463,592, uniform[-1,1) values, float64, CSR), the
sparse format sweep's regular matrix. The matrix, x and y are replicated R
times so that R * footprint >= 1 GiB and step s uses copy s % R: the 256 MB
Infinity Cache cannot hold the working set between steps.

The same run also measures (each section can be switched off):
  - the attainable streaming copy and read bandwidths;
  - the format sweep: CSR / COO / ELL / HYB / SELL-P in float64 and float32
    (and CSR with binary16 values) on the 27-point matrix and on the
    Zipf(1.5) matrix (n = 1e6, rows clipped to 10,000), plus the device
    conversions;
  - CG on the 64x64 Poisson system (latency, one at a time and batched);
  - the full-size solvers: Jacobi-CG on the anisotropic 7-point 128^3 grid,
    BiCGSTAB and GMRES(30) on the convection-diffusion 128^3 grid, and
    float32 / binary16-value iterative refinement against float64 CG on the
    7-point 192^3 grid, with the error against the float64 oracle solution;
  - the serving stream (Poisson arrivals, p50/p99 latency, solves/s, against
    the same requests solved one by one; request arrays in pinned host
    memory, --serve-pageable for pageable ones);
  - the CPU oracle on the host's cores (one thread and all cores).

Prints ONE JSON line; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
T0 = time.time()


def progress(msg):
    print(f"[bench {time.time() - T0:6.1f} s] {msg}", file=sys.stderr, flush=True)


def csr_bytes(n, nnz, sv, sx, beta=False):
    return nnz * (sv + 4) + (n + 1) * 4 + n * sx + n * sx + (n * sx if beta else 0)


def coo_bytes(n, nnz, sv, sx):
    return nnz * (sv + 8) + 2 * n * sx


def ell_bytes(n, K, sv, sx):
    return n * K * (sv + 4) + 2 * n * sx


def sellp_bytes(n, slice_cols, C, sv, sx):
    return slice_cols * C * (sv + 4) + (-(-n // C) + 1) * 4 + 2 * n * sx


def hyb_bytes(n, K, coo_nnz, sv, sx):
    return n * K * (sv + 4) + coo_nnz * (sv + 8) + 2 * n * sx


def time_launches(fn, steps, warmup, torch):
    """Average device time per call (ms) over `steps` back-to-back calls on
    the current stream, bracketed by HIP events."""
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        fn(i)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cg_iter_bytes(n, nnz, sv, precond):
    """Algorithmic bytes of one CG iteration: the CSR product plus 9 (no
    preconditioner) or 11 (Jacobi) vector passes of n values."""
    return csr_bytes(n, nnz, sv, sv) + (11 if precond else 9) * n * sv


def format_sweep(spx, torch, dev, A, x_h, args, tag, ell=True):
    """Time y = A x in CSR, COO, ELL and HYB (automatic width), float64 and
    float32 values, plus CSR with binary16 values and CSR without the
    row-length hint. Each format is built on the device from the CSR upload
    by spx_convert. GB/s counts the format's own algorithmic bytes (ELL
    padding included); csr_equiv_GBs counts the CSR bytes of the same
    product, for comparison across formats."""
    n, nnz = A.n, A.nnz
    out = {}
    K = int(A.row_lengths().max())
    free = torch.cuda.mem_get_info()[0]
    for vt, sv, vname in ((spx.F64, 8, "f64"), (spx.F32, 4, "f32"), (spx.F16, 2, "f16")):
        base = spx.csr_from_host(A, vt, dev)
        sx = 8 if vt == spx.F64 else 4
        hyb = spx.convert(base, spx.HYB)
        hK, hC = hyb.ell_width, hyb.coo_nnz
        del hyb
        sp = spx.convert(base, spx.SELLP)
        scols = sp.slice_cols
        del sp
        variants = {"csr": (lambda: spx.csr_analyse(spx.csr_from_host(A, vt, dev)), csr_bytes(n, nnz, sv, sx))}
        if vt != spx.F16:
            variants.update({
                "coo": (lambda: spx.convert(base, spx.COO), coo_bytes(n, nnz, sv, sx)),
                "hyb": (lambda: spx.convert(base, spx.HYB), hyb_bytes(n, hK, hC, sv, sx)),
                "sellp": (lambda: spx.convert(base, spx.SELLP), sellp_bytes(n, scols, 64, sv, sx)),
            })
            if ell:
                variants["ell"] = (lambda: spx.convert(base, spx.ELL), ell_bytes(n, K, sv, sx))

        def no_hint():
            M = spx.csr_from_host(A, vt, dev)
            M.max_row_len = 0  # no row-length hint
            return spx.csr_analyse(M)

        if vt != spx.F16:
            variants["csr_lb"] = (no_hint, csr_bytes(n, nnz, sv, sx))
        # column-blocked copy (for the random-column matrix only: a banded
        # matrix already finds x in L2): its own bytes add 8 block row
        # pointers and the 8 partial vectors (written and read)
        if tag == "zipf":
            variants["csr_cb"] = (lambda: spx.csr_colblock(spx.csr_analyse(spx.csr_from_host(A, vt, dev))),
                                  csr_bytes(n, nnz, sv, sx) + 8 * (n + 1) * 4 + 2 * 8 * n * sx)
        for fmt, (make, vb) in variants.items():
            name = f"{tag}_{fmt}_{vname}"
            if vb > 0.8 * free:
                out[name] = {"skipped": f"needs {vb / 1e9:.1f} GB"}
                continue
            Rv = max(1, int(np.ceil((1 << 30) / vb)))
            Ms = [make() for _ in range(Rv)]
            vdt = Ms[0].vec_dtype
            Xs = [torch.from_numpy(x_h).to(dev).to(vdt) for _ in range(Rv)]
            Ys = [torch.empty(n, dtype=vdt, device=dev) for _ in range(Rv)]
            steps = args.steps if vb < (4 << 30) else max(3, args.steps // 20)
            vms = time_launches(lambda i: spx.spmv(Ms[i % Rv], Xs[i % Rv], Ys[i % Rv]), steps,
                                max(1, args.warmup // 4), torch)
            out[name] = {"ms": round(vms, 5), "GBs": round(vb / vms / 1e6, 1), "bytes": vb,
                         "pct_hbm_peak": round(100 * vb / vms / 1e6 / HBM_PEAK_GBS, 2),
                         "gflops": round(2 * nnz / vms / 1e6, 1),
                         "csr_equiv_GBs": round(csr_bytes(n, nnz, sv, sx) / vms / 1e6, 1)}
            if fmt == "hyb":
                out[name].update(ell_width=hK, coo_nnz=hC)
            del Ms, Xs, Ys
            torch.cuda.empty_cache()
        del base
        torch.cuda.empty_cache()
    return out


def conversion_sweep(spx, torch, dev, A, tag, steps=20):
    """Device format conversion, float64 values: CSR -> COO / ELL / HYB /
    SELL-P and back, timed with HIP events around spx_convert alone (outputs
    and workspace allocated by one untimed plan + conversion). GB/s counts one
    read of the source arrays and one write of the destination arrays. The
    float64 -> float32 value cast is timed around the (blocking) call."""
    import ctypes

    n, nnz = A.n, A.nnz
    base = spx.csr_from_host(A, spx.F64, dev)
    csr_b = (n + 1) * 4 + nnz * 12
    out = {}

    def fmt_bytes(M):
        if M.fmt == spx.COO:
            return nnz * 16
        if M.fmt == spx.SELLP:
            return M.slice_cols * M.slice_size * 12 + (-(-n // M.slice_size) + 1) * 4
        if M.fmt == spx.ELL:
            return M.ell_width * M.ell_ld * 12
        return M.ell_width * M.ell_ld * 12 + M.coo_nnz * 16

    def time_convert(src, dst):
        ws = getattr(dst, "_ws")
        d_src, d_dst = src.desc(), dst.desc()
        fn = lambda i: spx.check(spx._lib.spx_convert(ctypes.byref(d_src), ctypes.byref(d_dst), spx._ptr(ws),
                                                      ws.numel(), spx._stream()), "spx_convert")
        return time_launches(fn, steps, 2, torch)

    for fname, fmt in (("coo", spx.COO), ("ell", spx.ELL), ("hyb", spx.HYB), ("sellp", spx.SELLP)):
        M = spx.convert(base, fmt)
        ms = time_convert(base, M)
        fb = fmt_bytes(M)
        out[f"{tag}_csr_to_{fname}"] = {"ms": round(ms, 4), "GBs": round((csr_b + fb) / ms / 1e6, 1)}
        back = spx.convert(M, spx.CSR)
        ms = time_convert(M, back)
        out[f"{tag}_{fname}_to_csr"] = {"ms": round(ms, 4), "GBs": round((csr_b + fb) / ms / 1e6, 1)}
        del M, back
        torch.cuda.empty_cache()
    spx.cast_values(base, spx.F32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        spx.cast_values(base, spx.F32)
    ms = (time.perf_counter() - t0) / 5 * 1e3
    out[f"{tag}_cast_f64_to_f32"] = {"ms": round(ms, 4), "GBs": round(nnz * 12 / ms / 1e6, 1)}
    return out


def subwarp_sweep(spx, torch, dev):
    """Subwarp reduction cost versus subwarp size (the protocol of the paper's
    reduction benchmark, Section 3.3): every lane of 2^22 float64 values
    repeats the subwarp sum 1,000 times on its running value. The cost per
    reduction step (size 1 subtracted) should grow as log2(size)."""
    n = 1 << 22
    loops = 1000
    x = torch.from_numpy(np.random.default_rng(0).uniform(-1, 1, n)).to(dev)
    out = torch.empty_like(x)
    t = {}
    for size in (1, 2, 4, 8, 16, 32, 64):
        ms = time_launches(lambda i: spx.subwarp_sum(x, size, loops, out), 5, 2, torch)
        t[size] = ms
    base = t[1]
    res = {str(k): {"ms": round(v, 4), "ns_per_reduction_per_wave": round((v - base) * 1e6 / (loops * n / 64), 6)}
           for k, v in t.items()}
    res["ratio_4_over_64"] = round((t[4] - base) / (t[64] - base), 3)
    res["theory_4_over_64"] = round(2 / 6, 3)
    return res


def csr_kernel_name(M):
    """Name of the CSR kernel the library picks for M (mirrors its rule:
    row-per-subwarp when rows are short and even, else load-balanced)."""
    if M is None or M.max_row_len <= 0 or M.nnz <= 0 or M.nrows > 65536:
        return "csr_spmv_kernel (load-balanced)"
    mean = -(-M.nnz // M.nrows)
    sub = 4
    while sub < 64 and sub < mean:
        sub *= 2
    return f"csr_rows_kernel (subwarp {sub})" if M.max_row_len <= 2 * sub else "csr_spmv_kernel (load-balanced)"


def profile_traffic(name, algo_bytes):
    """Beyond-L2 bytes per launch measured by the FETCH_SIZE / WRITE_SIZE
    counter runs summarised in profiles/<name>.md, or None when the kernel
    sources listed there have changed since (their hash differs) or the
    launch moved a different number of algorithmic bytes."""
    import hashlib

    path = os.path.join(ROOT, "profiles", name + ".md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ": " in line and not line.startswith(("|", "#", " ")):
            k, v = line.strip().split(": ", 1)
            kv[k] = v
    try:
        h = hashlib.sha256()
        for f in sorted(kv["kernel_sources"].split(",")):
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != kv["kernel_source_sha256_16"] or int(kv["algorithmic_bytes_per_launch"]) != algo_bytes:
            return None
        return int(kv["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def rhs(spx, S, torch, Ad, seed=0):
    """b = A x* on the device, x* i.i.d. uniform[-1, 1) (the product is the
    library's own)."""
    xs = torch.from_numpy(S.uniform_vector(Ad.nrows, seed=seed, purpose="xstar")).to(Ad.vals.device)
    return spx.spmv(Ad, xs)


def bench_cg_small(spx, S, torch, dev, nsolves, nbatch):
    """2D 5-point 64x64 (n = 4096, nnz = 20,224), unpreconditioned CG to 1e-10
    relative residual. (1) One system at a time: `nsolves` blocking solves back
    to back, latency = host wall clock per call. (2) Batched: `nbatch`
    independent right-hand sides solved by one launch of the batched kernel
    (one work-group per system)."""
    A = S.poisson2d(64)
    Ad = spx.csr_analyse(spx.csr_from_host(A, spx.F64, dev))
    bd = rhs(spx, S, torch, Ad)
    # one product, 1,000 launches each bracketed by its own events
    xv = torch.from_numpy(S.uniform_vector(A.n, seed=0)).to(dev)
    yv = torch.empty_like(xv)
    for _ in range(20):
        spx.spmv(Ad, xv, yv)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(1000)]
    for e0, e1 in ev:
        e0.record()
        spx.spmv(Ad, xv, yv)
        e1.record()
    torch.cuda.synchronize()
    sl = np.array([e0.elapsed_time(e1) * 1e3 for e0, e1 in ev])
    spmv_lat = {"p50_us": round(float(np.percentile(sl, 50)), 2), "p99_us": round(float(np.percentile(sl, 99)), 2),
                "launches": len(ev)}
    for _ in range(3):
        spx.cg_solve(Ad, bd, tol=1e-10)
    torch.cuda.synchronize()
    lat, iters = [], 0
    t0 = time.perf_counter()
    for _ in range(nsolves):
        t1 = time.perf_counter()
        x, info = spx.cg_solve(Ad, bd, tol=1e-10)
        lat.append(time.perf_counter() - t1)
        iters = info["iters"]
        assert info["status"] == 0 and info["relres_true"] <= 1e-10, info
    tot = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    out = {"spmv": spmv_lat,
           "single": {"solves_per_s": round(nsolves / tot, 2), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat, 99)), 3), "iters": iters, "solves": nsolves,
                      "relres_true": info["relres_true"]}}
    # the same blocking solves with pipelined CG (three launches per
    # iteration against five: the small system is launch-bound)
    for _ in range(3):
        spx.pipecg_solve(Ad, bd, tol=1e-10)
    torch.cuda.synchronize()
    plat = []
    t0 = time.perf_counter()
    for _ in range(nsolves):
        t1 = time.perf_counter()
        x, pinfo = spx.pipecg_solve(Ad, bd, tol=1e-10)
        plat.append(time.perf_counter() - t1)
        assert pinfo["status"] == 0 and pinfo["relres_true"] <= 1e-10, pinfo
    ptot = time.perf_counter() - t0
    plat = np.array(plat) * 1e3
    out["single_pipecg"] = {"solves_per_s": round(nsolves / ptot, 2), "p50_ms": round(float(np.percentile(plat, 50)), 3),
                            "p99_ms": round(float(np.percentile(plat, 99)), 3), "iters": pinfo["iters"],
                            "solves": nsolves, "relres_true": pinfo["relres_true"]}
    if nbatch > 0:
        bs = [rhs(spx, S, torch, Ad, seed=s) for s in range(nbatch)]
        spx.cg_batch([Ad] * nbatch, bs, tol=1e-10)
        torch.cuda.synchronize()
        reps, lat = 5, []
        for _ in range(reps):
            t1 = time.perf_counter()
            xs, infos = spx.cg_batch([Ad] * nbatch, bs, tol=1e-10)
            lat.append(time.perf_counter() - t1)
            assert all(i["status"] == 0 and i["relres_true"] <= 1e-10 for i in infos)
        lat = np.array(lat)
        out["batched"] = {"systems": nbatch, "solves_per_s": round(nbatch / float(np.median(lat)), 1),
                          "batch_ms_p50": round(1e3 * float(np.median(lat)), 3),
                          "batch_ms_max": round(1e3 * float(lat.max()), 3), "iters": infos[0]["iters"]}
    return out


def _solve_rec(info, nbytes=None, **extra):
    r = {"ms": round(info["device_ms"], 2), "iters": info["iters"], "spmv": info["spmv_count"],
         "us_per_iter": round(1e3 * info["device_ms"] / max(info["iters"], 1), 2),
         "relres_true": info["relres_true"], "status": info["status"]}
    if nbytes is not None:
        r["GBs"] = round(nbytes / (1e3 * info["device_ms"] / max(info["iters"], 1)) / 1e3, 1)
        r["pct_hbm_peak"] = round(100 * r["GBs"] / HBM_PEAK_GBS, 2)
    r.update(extra)
    return r


def bench_solvers(spx, S, torch, dev, cpu=True):
    """Krylov solvers at full size: CG+Jacobi on the anisotropic 7-point 128^3
    grid, BiCGSTAB and GMRES(30) + Jacobi on the upwind convection-diffusion
    128^3 grid, and mixed-precision IR (float32 / binary16 values) against
    plain float64 CG on the 7-point 192^3 grid; all to 1e-10. After the GPU
    timings (never beside them: the solvers' host-side loops must not compete
    with the oracle's threads for the CPU), the float64 oracle (all-core CG)
    solves the 192^3 system on the host and the IR and CG solutions are
    compared with its solution."""
    out = {}
    nrm = torch.linalg.vector_norm
    P192 = S.poisson3d_7pt(192)
    xstar192 = S.uniform_vector(P192.n, seed=0, purpose="xstar")
    oracle = {}

    def run_oracle():
        import oracle as O

        b = O.csr_spmv_omp(P192, xstar192)
        t = time.perf_counter()
        x, info = O.cg_omp(P192, b, tol=1e-10, maxit=5000)
        oracle.update(x=x, info=info, s=time.perf_counter() - t, threads=O.omp_threads())

    progress("solvers: CG + Jacobi, anisotropic 128^3")
    A = S.poisson3d_7pt(128, 1, 1, 0.01)
    Ad = spx.csr_analyse(spx.csr_from_host(A, spx.F64, dev))
    bd = rhs(spx, S, torch, Ad)
    cg_b = cg_iter_bytes(A.n, A.nnz, 8, True)
    spx.cg_solve(Ad, bd, tol=1e-10, precond=1, maxit=5000)
    x, info = spx.cg_solve(Ad, bd, tol=1e-10, precond=1, maxit=5000)
    out["cg_jacobi_aniso128"] = _solve_rec(info, cg_b, bytes_per_iter=cg_b)
    t_cg = info["device_ms"]
    spx.pipecg_solve(Ad, bd, tol=1e-10, precond=1, maxit=5000)
    x, info = spx.pipecg_solve(Ad, bd, tol=1e-10, precond=1, maxit=5000)
    out["pipecg_jacobi_aniso128"] = _solve_rec(info, time_vs_cg=round(info["device_ms"] / t_cg, 3))
    for bs in (8, 32):
        spx.cg_solve(Ad, bd, tol=1e-10, precond=bs, maxit=5000)
        x, info = spx.cg_solve(Ad, bd, tol=1e-10, precond=bs, maxit=5000)
        out[f"cg_blockjacobi{bs}_aniso128"] = _solve_rec(info)
    Ps = spx.convert(Ad, spx.SELLP)
    spx.cg_solve(Ps, bd, tol=1e-10, precond=1, maxit=5000)
    x, info = spx.cg_solve(Ps, bd, tol=1e-10, precond=1, maxit=5000)
    out["cg_jacobi_aniso128_sellp"] = _solve_rec(info)
    del Ad, A, Ps

    progress("solvers: BiCGSTAB, GMRES(30), BiCG, convection-diffusion 128^3")
    A = S.convdiff3d_upwind(128)
    Ad = spx.csr_analyse(spx.csr_from_host(A, spx.F64, dev))
    bd = rhs(spx, S, torch, Ad)
    spx.csr_transpose(Ad)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tms = []
    for _ in range(10):
        e0.record()
        spx.csr_transpose(Ad)
        e1.record()
        torch.cuda.synchronize()
        tms.append(e0.elapsed_time(e1))
    tmin = 2 * (4 * (A.n + 1) + 12 * A.nnz)  # read A, write A^T
    out["csr_transpose_convdiff128"] = {"ms_p50": round(float(np.median(tms)), 3), "nnz": A.nnz,
                                        "GBs_min_bytes": round(tmin / float(np.median(tms)) / 1e6, 1)}
    spmv_b = csr_bytes(A.n, A.nnz, 8, 8)
    for nm, fn, nb in (("bicgstab_jacobi_convdiff128", spx.bicgstab_solve, 2 * spmv_b + 20 * A.n * 8),
                       ("gmres30_jacobi_convdiff128", spx.gmres_solve, None),
                       ("bicg_jacobi_convdiff128", spx.bicg_solve, None)):
        fn(Ad, bd, tol=1e-10, precond=1, maxit=5000)
        x, info = fn(Ad, bd, tol=1e-10, precond=1, maxit=5000)
        out[nm] = _solve_rec(info, nb)
    del Ad, A

    progress("solvers: IR float32 / binary16 values against float64 CG, 192^3")
    A = P192
    A64 = spx.csr_analyse(spx.csr_from_host(A, spx.F64, dev))
    xstar = torch.from_numpy(xstar192).to(dev)
    bd = spx.spmv(A64, xstar)
    spx.cg_solve(A64, bd, tol=1e-10, maxit=5000)
    x, info = spx.cg_solve(A64, bd, tol=1e-10, maxit=5000)
    t64 = info["device_ms"]
    cg192_b = cg_iter_bytes(A.n, A.nnz, 8, False)
    out["cg_fp64_poisson192"] = _solve_rec(info, cg192_b)
    x64 = x.clone()
    out["cg_fp64_poisson192"]["rel_err_vs_xstar"] = float(nrm(x64 - xstar) / nrm(xstar))
    sols = {}
    for nm, low in (("ir_fp32_poisson192", spx.F32), ("ir_fp16v_poisson192", spx.F16)):
        Alow = spx.cast_values(A64, low)
        sweep = {}
        for itol in (1e-3, 1e-4, 1e-6):
            spx.ir_solve(A64, Alow, bd, tol=1e-10, inner_tol=itol)
            x, info = spx.ir_solve(A64, Alow, bd, tol=1e-10, inner_tol=itol)
            sweep[f"{itol:.0e}"] = {
                "ms": round(info["device_ms"], 2), "inner_iters": info["iters"], "outer": info["outer_iters"],
                "speedup_vs_fp64_cg": round(t64 / info["device_ms"], 3), "relres_true": info["relres_true"],
                "status": info["status"], "rel_err_vs_gpu_fp64_cg": float(nrm(x - x64) / nrm(x64)),
                "rel_err_vs_xstar": float(nrm(x - xstar) / nrm(xstar))}
            sols[(nm, f"{itol:.0e}")] = x.cpu().numpy()
        ok = {k: v for k, v in sweep.items() if v["status"] == 0}
        best = min(ok, key=lambda k: ok[k]["ms"]) if ok else None
        out[nm] = dict(ok[best], inner_tol=best) if best else {"status": "failed"}
        out[nm]["inner_tol_sweep"] = sweep
        del Alow
    # the same comparison with every matrix in ELL
    E64 = spx.convert(A64, spx.ELL)
    spx.cg_solve(E64, bd, tol=1e-10, maxit=5000)
    x, info = spx.cg_solve(E64, bd, tol=1e-10, maxit=5000)
    te = info["device_ms"]
    out["cg_fp64_poisson192_ell"] = _solve_rec(info)
    for nm, low in (("ir_fp32_poisson192_ell", spx.F32), ("ir_fp16v_poisson192_ell", spx.F16)):
        Elow = spx.cast_values(E64, low)
        spx.ir_solve(E64, Elow, bd, tol=1e-10, inner_tol=1e-6)
        x, info = spx.ir_solve(E64, Elow, bd, tol=1e-10, inner_tol=1e-6)
        out[nm] = {"ms": round(info["device_ms"], 2), "inner_iters": info["iters"], "outer": info["outer_iters"],
                   "speedup_vs_fp64_ell": round(te / info["device_ms"], 3),
                   "speedup_vs_fp64_csr": round(t64 / info["device_ms"], 3), "relres_true": info["relres_true"],
                   "status": info["status"], "rel_err_vs_xstar": float(nrm(x - xstar) / nrm(xstar))}
        sols[(nm, "1e-06")] = x.cpu().numpy()
        del Elow
    x64h = x64.cpu().numpy()
    del A64, E64
    torch.cuda.empty_cache()
    if cpu:
        progress("solvers: the host oracle's 192^3 CG (all cores)")
        run_oracle()
        xo = oracle["x"]
        no = np.linalg.norm(xo)
        out["oracle_fp64_cg_poisson192"] = {
            "s": round(oracle["s"], 2), "iters": oracle["info"]["iters"], "threads": oracle["threads"],
            "relres_true": oracle["info"]["relres_true"], "status": oracle["info"]["status"]}
        out["cg_fp64_poisson192"]["rel_err_vs_fp64_oracle"] = float(np.linalg.norm(x64h - xo) / no)
        for (nm, itol), xs_ in sols.items():
            rec = out[nm] if nm.endswith("_ell") else out[nm]["inner_tol_sweep"][itol]
            rec["rel_err_vs_fp64_oracle"] = float(np.linalg.norm(xs_ - xo) / no)
        for nm in ("ir_fp32_poisson192", "ir_fp16v_poisson192"):
            if "inner_tol" in out[nm]:
                out[nm]["rel_err_vs_fp64_oracle"] = out[nm]["inner_tol_sweep"][out[nm]["inner_tol"]]["rel_err_vs_fp64_oracle"]
    return out


def serve_workload(S, nreq, seed):
    """Request mix of the serving workload, every size drawn from its law:
    half 2D 5-point Poisson systems on N x N grids with N ~ U{32..512}, half
    random symmetric diagonally dominant SPD systems with n log-uniform in
    [1e3, 1e6] (5..30 entries per row, the pattern seeded per request). Every
    request has its own right-hand side b = A x* (x* seeded per request)."""
    r = S.rng(seed, "sizes")
    kinds = r.random(nreq) < 0.5
    pN = r.integers(32, 513, nreq)
    sn = np.floor(np.exp(r.uniform(np.log(1e3), np.log(1e6), nreq))).astype(int)
    return [("poisson", int(pN[i])) if kinds[i] else ("spd", int(sn[i])) for i in range(nreq)]


_PINNED = []  # torch tensors whose pinned host memory the request arrays view


def _pinned_copy(torch, a):
    """A numpy view of a pinned (page-locked) host copy of a; the tensor that
    owns the memory is kept in _PINNED."""
    t = torch.empty(a.shape, dtype=torch.from_numpy(a[:0]).dtype, pin_memory=True)
    out = t.numpy()
    out[...] = a
    _PINNED.append(t)
    return out


def build_requests(spx, S, torch, dev, reqs, seed, pinned=False):
    """Host CSR matrices and right-hand sides of every request (Poisson
    matrices shared by equal N; each SPD matrix generated for its request).
    pinned: every array in page-locked host memory (as a receive path would
    hold requests), so the server's uploads are plain DMA transfers."""
    pois = {}
    out = []
    t0 = time.time()
    pin = (lambda a: _pinned_copy(torch, a)) if pinned else (lambda a: a)
    for i, (kind, size) in enumerate(reqs):
        if kind == "poisson":
            if size not in pois:
                P = S.poisson2d(size)
                pois[size] = S.CSR(P.n, pin(P.rowptr), pin(P.col), pin(P.val))
            A = pois[size]
        else:
            A = S.spd_diag_dominant(size, seed=1_000_000 + seed * 100_000 + i, device=dev)
            A = S.CSR(A.n, pin(A.rowptr), pin(A.col), pin(A.val))
        Ad = spx.csr_from_host(A, spx.F64, dev)
        b = pin(rhs(spx, S, torch, Ad, seed=seed * 100_000 + i).cpu().numpy())
        out.append((A, b))
        if (i + 1) % 500 == 0:
            progress(f"serve: {i + 1}/{len(reqs)} requests built ({time.time() - t0:.1f} s)")
    return out


def cpu_serve_sample(systems, nsample=200):
    """The oracle's CG (plain C, float64, one solve per thread) on the first
    `nsample` requests of the serving stream, as many solves at once as the
    host has cores for this process (at most 16): sampled CPU solves/s. The
    C calls release the interpreter lock, so threads run them in parallel."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle as O

    ncores = max(1, min(16, len(os.sched_getaffinity(0))))
    sample = systems[: min(len(systems), nsample)]
    progress(f"serve cpu: {len(sample)} oracle CG solves on {ncores} threads")
    t0 = time.perf_counter()
    with ThreadPoolExecutor(ncores) as ex:
        infos = list(ex.map(lambda ab: O.cg(ab[0], ab[1], tol=1e-8, maxit=100000)[1], sample))
    dt = time.perf_counter() - t0
    assert all(i["status"] == O.OK for i in infos)
    return {"value": round(len(sample) / dt, 2), "unit": "solves/s", "cores": ncores, "kind": "oracle",
            "sample": f"first {len(sample)} requests of the stream, oracle CG to 1e-8, one solve per thread"}


def bench_serve(spx, S, torch, dev, nreq, seed, fracs, budget_gb=32, cpu=False, pinned=True):
    """Serving: (1) all `nreq` requests submitted at once (capacity, solves/s);
    (2) open-loop Poisson arrival streams at `fracs` x that capacity (latency
    = completion - scheduled arrival, p50/p99; completion is the server's own
    submit-to-done time added to the submission time); (3) a sample of the
    same requests solved one by one with the blocking float64 CG
    (spx_cg_solve), for comparison. Tolerance 1e-8. The request arrays are
    in pinned host memory unless pinned=False (pageable numpy arrays, which
    the runtime stages through its own buffers on the server's thread)."""
    reqs = serve_workload(S, nreq, seed)
    t0 = time.time()
    systems = build_requests(spx, S, torch, dev, reqs, seed, pinned=pinned)
    # result buffers, pinned as well (the server copies each solution there)
    xouts = [_pinned_copy(torch, np.zeros(A.n)) if pinned else None for A, _ in systems]
    gen_s = time.time() - t0
    nnz = np.array([A.nnz for A, _ in systems])
    n = np.array([A.n for A, _ in systems])
    srv = spx.Server(max_slots=2048, hbm_budget_bytes=int(budget_gb * (1 << 30)))

    def run(arrivals, label):
        progress(f"serve {label}: submitting {nreq} requests")
        tickets, t_sched, t_sub = [], [], []
        start = time.perf_counter()
        for i, (A, b) in enumerate(systems):
            if arrivals is not None:
                while time.perf_counter() - start < arrivals[i]:
                    time.sleep(0.0002)
            t_sub.append(time.perf_counter())
            tickets.append(srv.submit(A, b, tol=1e-8, x_out=xouts[i]))
            t_sched.append(start + (arrivals[i] if arrivals is not None else 0.0))
        lat, iters, worst, last = [], [], 0.0, start
        for i, (t, ts, tu) in enumerate(zip(tickets, t_sched, t_sub)):
            x, info = srv.wait(t, timeout_s=900)
            assert info["status"] == 0, info
            done = tu + info["device_ms"] * 1e-3
            last = max(last, done)
            lat.append(done - ts)
            iters.append(info["iters"])
            worst = max(worst, info["relres_true"])
        total = last - start
        lat = np.array(lat) * 1e3
        iters = np.array(iters)
        kinds = np.array([k for k, _ in reqs])
        fam = {}
        for k in ("poisson", "spd"):
            sel = kinds == k
            if sel.any():
                fam[k] = {"p50_ms": round(float(np.percentile(lat[sel], 50)), 2),
                          "p99_ms": round(float(np.percentile(lat[sel], 99)), 2),
                          "mean_iters": round(float(iters[sel].mean()), 1)}
        # the slowest 1%: what they are (size, iterations)
        slow = np.argsort(lat)[-max(1, nreq // 100):]
        return {"requests": nreq, "solves_per_s": round(nreq / total, 2), "wall_s": round(total, 3),
                "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "p99_over_p50": round(float(np.percentile(lat, 99) / np.percentile(lat, 50)), 2),
                "mean_iters": round(float(np.mean(iters)), 1), "max_relres_true": worst, "by_family": fam,
                "slowest_1pct": {"n_median": int(np.median(n[slow])), "iters_median": int(np.median(iters[slow])),
                                 "poisson_share": round(float(np.mean(kinds[slow] == "poisson")), 2)},
                "_lat": lat, "_iters": iters}

    progress(f"serve: {nreq} requests built in {gen_s:.1f} s")
    burst = run(None, "burst")
    burst_iters = burst.pop("_iters")
    burst.pop("_lat")
    streams = {}
    for frac in fracs:
        rate = frac * burst["solves_per_s"]
        r = run(S.poisson_arrivals(nreq, rate, seed=seed), f"{frac:.1f}x")
        r.pop("_iters")
        r.pop("_lat")
        r["rate_per_s"] = round(rate, 2)
        streams[f"{frac:.1f}x"] = r
    # unloaded latency of the heaviest requests (iterations x entries), each
    # alone on the server: the floor the tail of a loaded stream sits on
    heavy = np.argsort(burst_iters * (nnz + n))[-10:]
    alone = []
    for i in heavy:
        A, b = systems[i]
        t = srv.submit(A, b, tol=1e-8)
        _, info = srv.wait(t, timeout_s=900)
        alone.append(info["device_ms"])
    light = np.argsort(burst_iters * (nnz + n))[nreq // 2 - 5:nreq // 2 + 5]
    alone_mid = []
    for i in light:
        A, b = systems[i]
        t = srv.submit(A, b, tol=1e-8)
        _, info = srv.wait(t, timeout_s=900)
        alone_mid.append(info["device_ms"])
    unloaded = {"heaviest10_ms_median": round(float(np.median(alone)), 2),
                "median_work10_ms_median": round(float(np.median(alone_mid)), 2),
                "ratio": round(float(np.median(alone) / max(np.median(alone_mid), 1e-9)), 2)}
    st = srv.stats()
    srv.close()
    # sequential blocking float64 CG on a sample of the same requests
    sample = systems[: min(nreq, 200)]
    progress(f"serve: {len(sample)} sequential blocking solves")
    t1 = time.perf_counter()
    for A, b in sample:
        Ad = spx.csr_from_host(A, spx.F64, dev)
        x, info = spx.cg_solve(Ad, torch.from_numpy(b).to(dev), tol=1e-8, maxit=100000)
        assert info["status"] == 0
    seq = len(sample) / (time.perf_counter() - t1)
    # the served throughput over the same first requests
    out = {"burst": burst, "open_loop": streams, "unloaded": unloaded,
           "sequential_cg_solves_per_s": round(seq, 2), "sequential_sample": len(sample), "served_over_sequential": round(burst["solves_per_s"] / seq, 2),
           "server": {k: st[k] for k in ("ticks", "pool_bytes_peak", "pool_bytes_total")}, "budget_gb": budget_gb,
           "mix": {"poisson": int(sum(k == "poisson" for k, _ in reqs)), "spd": int(sum(k == "spd" for k, _ in reqs)),
                   "n_median": int(np.median(n)), "n_max": int(n.max()), "nnz_mean": int(nnz.mean()),
                   "nnz_max": int(nnz.max())},
           "gen_s": round(gen_s, 1), "host_memory": "pinned" if pinned else "pageable"}
    if cpu:
        out["cpu_oracle"] = cpu_serve_sample(systems)
    del systems
    _PINNED.clear()
    return out


def cpu_spmv_baseline(A, x_h, b, desc):
    """The oracle's plain float64 CSR product on the host: one thread (about
    10 s of repetitions) and all cores (the OpenMP variant, about 5 s)."""
    import oracle as O

    out = {}
    O.csr_spmv(A, x_h)
    reps, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < 10.0:
        O.csr_spmv(A, x_h)
        reps += 1
    cs = (time.perf_counter() - t1) / reps
    one = {"value": round(b / cs / 1e9, 2), "unit": "GB/s", "cores": 1, "kind": "oracle",
           "sample": f"{reps} plain float64 CSR products of the full {desc} matrix, {cs * 1e3:.1f} ms each, 1 thread"}
    th = O.omp_threads()
    O.csr_spmv_omp(A, x_h)
    reps, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < 5.0:
        O.csr_spmv_omp(A, x_h)
        reps += 1
    cs = (time.perf_counter() - t1) / reps
    allc = {"value": round(b / cs / 1e9, 2), "unit": "GB/s", "cores": th, "kind": "oracle",
            "sample": f"{reps} plain float64 CSR products of the full {desc} matrix, {cs * 1e3:.2f} ms each, "
                      f"rows shared by {th} OpenMP threads"}
    return allc, one


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--grid", type=int, default=100, help="27-point grid edge (100 -> n = 1e6)")
    ap.add_argument("--matrix", choices=("27pt", "zipf"), default="27pt",
                    help="matrix of the headline CSR product (27-point stencil or the Zipf(1.5) rows)")
    ap.add_argument("--quick", action="store_true", help="headline product only (no sweep, solvers, serving)")
    ap.add_argument("--colblock", action="store_true",
                    help="headline product through the column-blocked copy (spx_csr_colblock); GB/s stays CSR bytes")
    ap.add_argument("--no-sweep", action="store_true", help="skip the format sweep and conversions")
    ap.add_argument("--no-zipf", action="store_true", help="skip the Zipf(1.5) formats of the sweep")
    ap.add_argument("--zipf-ell", action="store_true", help="also time the 1e10-slot Zipf ELL (120 GB)")
    ap.add_argument("--no-solvers", action="store_true", help="skip the full-size Krylov solvers")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--cg-solves", type=int, default=50, help="solves of the 64x64 CG latency run (0 = skip)")
    ap.add_argument("--cg-batch", type=int, default=1024, help="systems in the batched 64x64 CG run (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests of the serving run (0 = skip)")
    ap.add_argument("--serve-fracs", default="0.5,0.7,0.9", help="open-loop arrival rates, fractions of capacity")
    ap.add_argument("--serve-budget-gb", type=float, default=32.0, help="HBM budget of the serving run")
    ap.add_argument("--serve-pageable", action="store_true",
                    help="requests in pageable host memory (default: pinned, as a receive path holds them)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-subwarp", action="store_true", help="skip the subwarp reduction sweep")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.quick:
        args.no_sweep = args.no_solvers = args.no_subwarp = True
        args.serve_requests = 0

    import torch

    from paper_2006_14290_amd import spx
    from paper_2006_14290_amd import synth as S

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    if args.matrix == "zipf":
        A = S.zipf_matrix(1_000_000, seed=0)
        mdesc, mtag = "Zipf(1.5) rows clipped to 10,000, n=1e6", "zipf"
    else:
        A = S.stencil27_random(args.grid, seed=0)
        mdesc, mtag = f"27-point stencil {args.grid}^3", f"27pt{args.grid}"
    x_h = S.uniform_vector(A.n, seed=0)
    n, nnz = A.n, A.nnz
    gen_s = time.time() - t0

    # replicate so that the rotated working set exceeds the Infinity Cache
    progress(f"headline: CSR float64, {mdesc}")
    fp = csr_bytes(n, nnz, 8, 8)
    R = max(2, int(np.ceil((1 << 30) / fp)))
    mats = [spx.csr_analyse(spx.csr_from_host(A, spx.F64, dev)) for _ in range(R)]
    kname = csr_kernel_name(mats[0])
    if args.colblock:
        mats = [spx.csr_colblock(M) for M in mats]
        kname = "cb_spmv_kernel (column-blocked, + cb_finish_kernel)"
        mdesc += ", column-blocked copy"
    xs = [torch.from_numpy(x_h).to(dev) for _ in range(R)]
    ys = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(R)]

    def csr_step(i):
        k = i % R
        spx.spmv(mats[k], xs[k], ys[k], csr_only=True)

    results = {}
    ms = time_launches(csr_step, args.steps, args.warmup, torch)
    b = csr_bytes(n, nnz, 8, 8)
    results["csr_f64"] = {"ms": ms, "GBs": b / ms / 1e6, "bytes": b}
    del mats, xs, ys
    torch.cuda.empty_cache()

    # attainable streaming bandwidths (1 GiB read + 1 GiB written; 2 GiB read)
    cn = (1 << 30) // 8
    src = torch.empty(cn, dtype=torch.float64, device=dev).uniform_()
    dst = torch.empty_like(src)
    cms = time_launches(lambda i: spx.stream_copy(src, dst), 20, 3, torch)
    copy_gbs = 2 * cn * 8 / cms / 1e6
    del dst
    src2 = torch.empty(2 * cn, dtype=torch.float64, device=dev).uniform_()
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    rms = time_launches(lambda i: spx.stream_read(src2, sink), 20, 3, torch)
    read_gbs = 2 * cn * 8 / rms / 1e6
    del src, src2
    torch.cuda.empty_cache()

    conversions = None
    if not args.no_sweep:
        progress("sweep: 27-point formats")
        results.update(format_sweep(spx, torch, dev, S.stencil27_random(100, seed=0) if mtag != "27pt100" else A,
                                    x_h if mtag == "27pt100" else S.uniform_vector(10**6, seed=0), args, "27pt"))
        progress("sweep: conversions")
        conversions = conversion_sweep(spx, torch, dev, A if mtag == "27pt100" else S.stencil27_random(100, seed=0),
                                       "27pt")
        if not args.no_zipf:
            progress("sweep: Zipf formats")
            Z = A if mtag == "zipf" else S.zipf_matrix(1_000_000, seed=0)
            zx = S.uniform_vector(Z.n, seed=0)
            results.update(format_sweep(spx, torch, dev, Z, zx, args, "zipf", ell=args.zipf_ell))
            del Z

    progress("64x64 CG")
    cg_small = bench_cg_small(spx, S, torch, dev, args.cg_solves, args.cg_batch) if args.cg_solves > 0 else None
    solvers = bench_solvers(spx, S, torch, dev, cpu=not args.no_cpu) if not args.no_solvers else None
    serve = None
    if args.serve_requests > 0:
        fracs = [float(f) for f in args.serve_fracs.split(",") if f]
        serve = bench_serve(spx, S, torch, dev, args.serve_requests, args.seed, fracs, args.serve_budget_gb,
                            not args.no_cpu, pinned=not args.serve_pageable)
    subwarp = None
    if not args.no_subwarp:
        progress("subwarp sweep")
        subwarp = subwarp_sweep(spx, torch, dev)

    cpu = None
    if not args.no_cpu:
        import oracle as O

        progress("cpu baseline: oracle CSR product")
        cpu, cpu1 = cpu_spmv_baseline(A, x_h, b, mdesc)
        cpu["single_thread"] = cpu1
        if solvers is not None and "oracle_fp64_cg_poisson192" in solvers:
            o = solvers["oracle_fp64_cg_poisson192"]
            cpu["solver_cg_poisson192"] = {
                "value": o["s"], "unit": "s to 1e-10", "cores": o["threads"], "kind": "oracle",
                "iters": o["iters"], "gpu_fp64_cg_s": round(solvers["cg_fp64_poisson192"]["ms"] / 1e3, 4),
                "sample": "one oracle CG solve (all-core variant) of the 7-point 192^3 system, run on the host after the GPU timings"}
        if cg_small is not None:
            # the oracle's CG on the 64x64 Poisson system (unpreconditioned, 1e-10), 1 thread
            P = S.poisson2d(64)
            pb = O.csr_spmv(P, S.uniform_vector(P.n, seed=0, purpose="xstar"))
            cnt, t1 = 0, time.perf_counter()
            while time.perf_counter() - t1 < 3.0:
                _, oinfo = O.cg(P, pb, tol=1e-10)
                cnt += 1
            cg_small["cpu_oracle"] = {"value": round(cnt / (time.perf_counter() - t1), 2), "unit": "solves/s",
                                      "cores": 1, "kind": "oracle", "iters": oinfo["iters"],
                                      "sample": f"{cnt} oracle CG solves of the 64x64 Poisson system, 1 thread"}

    r = results["csr_f64"]
    line = {
        "metric": "SpMV GB/s (% HBM peak); CG solves/sec + p50/p99 latency at 1e-10 rel. residual",
        "value": round(r["GBs"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"SpMV y=Ax, CSR float64, {mdesc} (n={n}, nnz={nnz}), "
                               f"uniform[-1,1) values, {R} rotated copies"},
        "pct_hbm_peak": round(100 * r["GBs"] / HBM_PEAK_GBS, 2),
        "gflops": round(2 * nnz / r["ms"] / 1e6, 2),
        "copy_GBs": round(copy_gbs, 1),
        "read_GBs": round(read_gbs, 1),
        "pct_of_copy": round(100 * r["GBs"] / copy_gbs, 2),
        "pct_of_read": round(100 * r["GBs"] / read_gbs, 2),
        "roofline": {"bound": "hbm", "achieved": round(r["GBs"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(r["GBs"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": kname, "bytes_per_launch": b},
        "sweep": {k: ({kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()})
                  for k, v in results.items()},
        "conversions": conversions,
        "cg_poisson64": cg_small,
        "solvers": solvers,
        "serve": serve,
        "subwarp": subwarp,
        "cpu_baseline": cpu,
        "gen_s": round(gen_s, 1),
        "wall_s": round(time.time() - T0, 1),
    }
    traffic = profile_traffic(f"csr_spmv_f64_{mtag}" + ("_colblock" if args.colblock else ""), b)
    if traffic is not None:
        line["roofline"]["traffic"] = traffic
        line["roofline"]["traffic_over_algorithmic"] = round(traffic / b, 4)
        line["roofline"]["traffic_kind"] = "beyond-L2 bytes (FETCH_SIZE, WRITE_SIZE counters, copy-calibrated)"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

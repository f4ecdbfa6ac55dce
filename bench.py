#!/usr/bin/env python3
"""Benchmark of the SpMV hot path on one MI355X.

Workload (one "step"): y = A x on the 27-point stencil of a 100^3 grid
(n = 1e6, nnz = 26,463,592, uniform[-1,1) values, float64, CSR), the sparse
format sweep's regular matrix. The matrix, x and y are replicated R times so
that R * footprint >= 1 GiB and step s uses copy s % R: the 256 MB
Infinity Cache cannot hold the working set between steps.

Prints ONE JSON line: SpMV GB/s (algorithmic bytes / time) and its fraction
of the 8 TB/s HBM peak, the other formats and precisions of the sweep, a
measured streaming-copy bandwidth, the roofline record of the CSR kernel and
the CPU oracle's rate on the host.
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


def csr_bytes(n, nnz, sv, sx, beta=False):
    return nnz * (sv + 4) + (n + 1) * 4 + n * sx + n * sx + (n * sx if beta else 0)


def coo_bytes(n, nnz, sv, sx):
    return nnz * (sv + 8) + 2 * n * sx


def ell_bytes(n, K, sv, sx):
    return n * K * (sv + 4) + 2 * n * sx


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


def bench_cg_small(spx, S, O, torch, dev, nsolves):
    """2D 5-point 64x64 (n = 4096, nnz = 20,224), unpreconditioned CG to 1e-10
    relative residual, solved `nsolves` times back to back (blocking calls);
    latency is the host wall clock of each call."""
    A = S.poisson2d(64)
    xs = S.uniform_vector(A.n, seed=0, purpose="xstar")
    b, _ = O.csr_spmv_dot2(A, xs)
    Ad = spx.csr_analyse(spx.csr_from_host(A, spx.F64, dev))
    bd = torch.from_numpy(b).to(dev)
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
    return {"solves_per_s": round(nsolves / tot, 2), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "iters": iters, "solves": nsolves,
            "relres_true": info["relres_true"]}


def bench_solvers(spx, S, O, torch, dev):
    """Krylov solvers at full size: CG+Jacobi on the anisotropic 7-point 128^3
    grid, BiCGSTAB and GMRES(30) + Jacobi on the upwind convection-diffusion
    128^3 grid, and mixed-precision IR (float32 / binary16 values) against
    plain float64 CG on the 7-point 192^3 grid; all to 1e-10."""
    out = {}

    def prob(A):
        xs = S.uniform_vector(A.n, seed=0, purpose="xstar")
        b, _ = O.csr_spmv_dot2(A, xs)
        return torch.from_numpy(b).to(dev)

    A = S.poisson3d_7pt(128, 1, 1, 0.01)
    bd = prob(A)
    Ad = spx.csr_analyse(spx.csr_from_host(A, spx.F64, dev))
    spx.cg_solve(Ad, bd, tol=1e-10, precond=1, maxit=5000)
    x, info = spx.cg_solve(Ad, bd, tol=1e-10, precond=1, maxit=5000)
    it_us = 1e3 * info["device_ms"] / max(info["iters"], 1)
    out["cg_jacobi_aniso128"] = {"ms": round(info["device_ms"], 2), "iters": info["iters"],
                                 "us_per_iter": round(it_us, 2),
                                 "GBs": round(cg_iter_bytes(A.n, A.nnz, 8, True) / it_us / 1e3, 1),
                                 "relres_true": info["relres_true"]}
    del Ad, A
    A = S.convdiff3d_upwind(128)
    bd = prob(A)
    Ad = spx.csr_analyse(spx.csr_from_host(A, spx.F64, dev))
    for nm, fn in (("bicgstab_jacobi_convdiff128", spx.bicgstab_solve), ("gmres30_jacobi_convdiff128", spx.gmres_solve)):
        fn(Ad, bd, tol=1e-10, precond=1, maxit=5000)
        x, info = fn(Ad, bd, tol=1e-10, precond=1, maxit=5000)
        out[nm] = {"ms": round(info["device_ms"], 2), "iters": info["iters"], "spmv": info["spmv_count"],
                   "relres_true": info["relres_true"]}
    del Ad, A
    A = S.poisson3d_7pt(192)
    bd = prob(A)
    A64 = spx.csr_analyse(spx.csr_from_host(A, spx.F64, dev))
    spx.cg_solve(A64, bd, tol=1e-10, maxit=5000)
    x, info = spx.cg_solve(A64, bd, tol=1e-10, maxit=5000)
    t64 = info["device_ms"]
    out["cg_fp64_poisson192"] = {"ms": round(t64, 2), "iters": info["iters"], "relres_true": info["relres_true"]}
    x64 = x.clone()
    for nm, low in (("ir_fp32_poisson192", spx.F32), ("ir_fp16v_poisson192", spx.F16)):
        Alow = spx.cast_values(A64, low)
        spx.ir_solve(A64, Alow, bd, tol=1e-10, inner_tol=1e-3)
        x, info = spx.ir_solve(A64, Alow, bd, tol=1e-10, inner_tol=1e-3)
        err = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))
        out[nm] = {"ms": round(info["device_ms"], 2), "inner_iters": info["iters"], "outer": info["outer_iters"],
                   "speedup_vs_fp64": round(t64 / info["device_ms"], 3), "relres_true": info["relres_true"],
                   "rel_err_vs_fp64_cg": err}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--grid", type=int, default=100, help="27-point grid edge (100 -> n = 1e6)")
    ap.add_argument("--sweep", action="store_true", help="also time COO/ELL/HYB and float32")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--solvers", action="store_true", help="also time the full-size Krylov solvers")
    ap.add_argument("--cg-solves", type=int, default=50, help="solves of the 64x64 CG latency run (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2006_14290_amd import spx
    from paper_2006_14290_amd import synth as S

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    A = S.stencil27_random(args.grid, seed=0)
    x_h = S.uniform_vector(A.n, seed=0)
    n, nnz = A.n, A.nnz
    gen_s = time.time() - t0

    # replicate so that the rotated working set exceeds the Infinity Cache
    fp = csr_bytes(n, nnz, 8, 8)
    R = max(2, int(np.ceil((1 << 30) / fp)))
    mats = [spx.csr_analyse(spx.csr_from_host(A, spx.F64, dev)) for _ in range(R)]
    xs = [torch.from_numpy(x_h).to(dev) for _ in range(R)]
    ys = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(R)]

    def csr_step(i):
        k = i % R
        spx.spmv(mats[k], xs[k], ys[k], csr_only=True)

    results = {}
    ms = time_launches(csr_step, args.steps, args.warmup, torch)
    b = csr_bytes(n, nnz, 8, 8)
    results["csr_f64"] = {"ms": ms, "GBs": b / ms / 1e6, "bytes": b}

    # attainable streaming bandwidth (copy of a 2 GiB buffer, read + write)
    cn = (1 << 30) // 8
    src = torch.empty(cn, dtype=torch.float64, device=dev).uniform_()
    dst = torch.empty_like(src)
    cms = time_launches(lambda i: spx.stream_copy(src, dst), 20, 3, torch)
    copy_gbs = 2 * cn * 8 / cms / 1e6
    del src, dst

    if args.sweep:
        import oracle as O  # host-side format conversion for the inputs only

        E = O.csr_to_ell(A)
        H = O.csr_to_hyb(A)
        crow = O.csr_to_coo_rows(A)
        variants = {
            "coo_f64": (lambda: spx.coo_from_host(n, crow, A.col, A.val, spx.F64, dev), coo_bytes(n, nnz, 8, 8)),
            "ell_f64": (lambda: spx.ell_from_host(n, E.K, E.ld, E.col, E.val, spx.F64, dev), ell_bytes(n, E.K, 8, 8)),
            "hyb_f64": (lambda: spx.hyb_from_host(n, H.ell.K, H.ell.ld, H.ell.col, H.ell.val, H.row, H.col, H.val,
                                                  spx.F64, dev), hyb_bytes(n, H.ell.K, len(H.row), 8, 8)),
            "csr_f32": (lambda: spx.csr_analyse(spx.csr_from_host(A, spx.F32, dev)), csr_bytes(n, nnz, 4, 4)),
            "csr_f16": (lambda: spx.csr_analyse(spx.csr_from_host(A, spx.F16, dev)), csr_bytes(n, nnz, 2, 4)),
            "csr_f64_nopart": (lambda: spx.csr_from_host(A, spx.F64, dev), csr_bytes(n, nnz, 8, 8)),
        }
        del mats
        torch.cuda.empty_cache()
        for name, (make, vb) in variants.items():
            Rv = max(2, int(np.ceil((1 << 30) / vb)))
            Ms = [make() for _ in range(Rv)]
            vdt = Ms[0].vec_dtype
            Xs = [torch.from_numpy(x_h).to(dev).to(vdt) for _ in range(Rv)]
            Ys = [torch.empty(n, dtype=vdt, device=dev) for _ in range(Rv)]
            vms = time_launches(lambda i: spx.spmv(Ms[i % Rv], Xs[i % Rv], Ys[i % Rv]), args.steps, args.warmup,
                                torch)
            results[name] = {"ms": vms, "GBs": vb / vms / 1e6, "bytes": vb}
            del Ms, Xs, Ys
            torch.cuda.empty_cache()

    import oracle as O  # inputs (b = A x*) and the CPU baseline only

    cg_small = bench_cg_small(spx, S, O, torch, dev, args.cg_solves) if args.cg_solves > 0 else None
    solvers = bench_solvers(spx, S, O, torch, dev) if args.solvers else None

    cpu = None
    if not args.no_cpu:
        import oracle as O

        # the oracle's plain float64 CSR product, single thread, repeated for ~10 s
        O.csr_spmv(A, x_h)
        reps, t1 = 0, time.perf_counter()
        while time.perf_counter() - t1 < 10.0:
            O.csr_spmv(A, x_h)
            reps += 1
        cs = (time.perf_counter() - t1) / reps
        cpu = {"value": b / cs / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} plain float64 CSR products of the full 27-point 100^3 matrix, "
                         f"{cs * 1e3:.1f} ms each, 1 thread"}

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
        "config": {"workload": f"SpMV y=Ax, CSR float64, 27-point stencil {args.grid}^3 (n={n}, nnz={nnz}), "
                               f"uniform[-1,1) values, {R} rotated copies"},
        "pct_hbm_peak": round(100 * r["GBs"] / HBM_PEAK_GBS, 2),
        "gflops": round(2 * nnz / r["ms"] / 1e6, 2),
        "copy_GBs": round(copy_gbs, 1),
        "pct_of_copy": round(100 * r["GBs"] / copy_gbs, 2),
        "roofline": {"bound": "hbm", "achieved": round(r["GBs"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(r["GBs"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "csr_spmv_kernel<double,double,false>", "bytes_per_launch": b},
        "sweep": {k: {"GBs": round(v["GBs"], 2), "ms": round(v["ms"], 5)} for k, v in results.items()},
        "cg_poisson64": cg_small,
        "solvers": solvers,
        "cpu_baseline": cpu,
        "gen_s": round(gen_s, 1),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

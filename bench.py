#!/usr/bin/env python3
"""Benchmark of the block Krylov hot path on one MI355X.

Workload (the headline): 3D 7-point Laplacian on a 128^3 grid (n = 2,097,152,
nnz = 14,581,760), p = 8 right-hand sides uniform in [-1, 1] (seed 1002),
block CG over the block subalgebra with adaptive re-orthonormalisation
(eta = 1e4), X0 = 0, relative residual tolerance 1e-10 per column.

One step = one complete solve to 1e-10 (time-to-tolerance).  The reported
value is block-CG iterations per second over the K timed solves; the solve
time is ms_per_step.  Inputs are resident in HBM before timing starts.

roofline: the dominant kernel is the SpMM fused with the alpha Gram partials
(spmm_ell_kernel<double, 8, 2, 1>, streaming the padded row-major copy of A);
its average duration comes from HIP events the library records around every
launch in four of that kernel on the solve's stream during the timed region
(bkry_profile with only that kernel selected and a sampling stride of 4, so
the other kernels and three launches in four run without events).  Algorithmic bytes per launch = the CSR form of the product:
rowptr + colind + values + X read + Y write (the ELL padding is not counted).
traffic: measured HBM bytes per launch from the committed rocprofv3 counter
summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
for a plain 1 GiB device copy), used only while the kernel sources hash to
the value recorded there.

cpu_baseline: the oracle (plain C, one thread) on a bounded sample of the
same solve (the difference of two runs of 2 and 16 block iterations, about
10-20 s of CPU work), as iterations per second.

extras: the other hot-path rows measured on their own workloads (hybrid
subalgebra, BDOT, block GMRes(30) cycle with TSQR, standalone TSQR
4,194,304 x 32, FP32-inner iterative refinement, adjoint solve).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
METRIC = "block-CG iters/s + SpMM/BDOT HBM GB/s (p=8, 128³ Laplacian); time-to-1e-10"
PMC_FILE = os.path.join(ROOT, "profiles", "spmm_laplace3d_128_s8_pmc.txt")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2104_02494_amd", "csrc", f) for f in ("kernels_block.hip", "common.hpp")]
ROOFLINE_KERNEL = "spmm_ell_kernel<double, 8, 2, 1>"
PROF_EVERY = 8          # HIP events around one SpMM launch in 8 of the timed solves


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


SPMM_END_MARK = b"// ------------------------------------------------------------------ Gram --"


def kernel_hash():
    """Hash of the sources of the roofline kernel: kernels_block.hip up to the
    end of its SpMM section (the SpMM kernels, their launchers and the
    helpers above them) and common.hpp."""
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        data = open(f, "rb").read()
        if f.endswith("kernels_block.hip"):
            data = data[:data.index(SPMM_END_MARK)]
        h.update(data)
    return h.hexdigest()[:16]


def pmc_traffic():
    """HBM bytes per launch of the fused SpMM from the committed rocprofv3
    counter summary, or None if absent or taken on a different kernel source."""
    if not os.path.exists(PMC_FILE):
        return None
    vals = {}
    for line in open(PMC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def spmm_bytes(A, s, elem=8):
    return (A.n + 1) * 4 + A.nnz * 4 + A.nnz * elem + 2 * A.n * s * elem


def cpu_baseline(A, B, iters_a=2, iters_b=36):
    """Oracle block CG on the same workload; the per-iteration time is the
    difference of two bounded runs, so set-up is excluded."""
    import oracle
    t0 = time.perf_counter()
    oracle.bcg(A, B, kind="block", tol=0.0, maxit=iters_a, eta=1e4)
    t1 = time.perf_counter()
    oracle.bcg(A, B, kind="block", tol=0.0, maxit=iters_b, eta=1e4)
    t2 = time.perf_counter()
    per_it = ((t2 - t1) - (t1 - t0)) / (iters_b - iters_a)
    return dict(value=1.0 / per_it, unit="block-iter/s", cores=1, kind="oracle",
                sample=f"128^3 Laplacian, p=8, block subalgebra, eta=1e4: {iters_b} vs {iters_a} block iterations "
                       f"(difference), single-threaded C oracle; {t2 - t0:.1f} s of CPU work",
                seconds_per_iter=per_it)


def run(args):
    import numpy as np
    import torch

    import paper_2104_02494_amd as P
    import workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    h = P.Handle(0)
    log("building 128^3 Laplacian workload")
    A, B, _ = W.build_workload("laplace3d_128_s8")
    s = B.shape[1]
    Ad = P.CsrMatrix.from_numpy(A.n, A.rowptr, A.colind, A.val, device=dev)
    Bd = torch.as_tensor(B).to(dev)
    opts = dict(kind="block", q=1, tol=1e-10, maxit=args.maxit, eta=1e4)
    solve = P.bkry_cg1r_solve if args.solver == "cg1r" else P.bkry_cg_solve

    for w in range(args.warmup):
        X, info = solve(h, Ad, Bd, **opts)
        log(f"warmup {w}: iters {info['iters']} reorth {info['reorth']} {info['seconds']*1e3:.1f} ms")
    P.bkry_profile(h, True, kernels=[P.PROF_CG_SPMM], every=PROF_EVERY)
    for k in range(4):
        P.bkry_profile_read(h, k, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    infos = []
    for k in range(args.steps):
        X, info = solve(h, Ad, Bd, **opts)
        iters += info["iters"]
        infos.append(info)
        log(f"step {k}: iters {info['iters']} reorth {info['reorth']} {info['seconds']*1e3:.1f} ms "
            f"true relres {max(info['true_relres']):.2e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    spmm_ms, spmm_n = P.bkry_profile_read(h, P.PROF_CG_SPMM)
    elapsed = t1 - t0
    value = iters / elapsed
    ms_per_step = elapsed / args.steps * 1e3
    # one more (untimed) solve with every streaming kernel timed, for the
    # per-kernel rates reported beside the roofline
    P.bkry_profile(h, True)
    for k in range(4):
        P.bkry_profile_read(h, k, reset=True)
    solve(h, Ad, Bd, **opts)
    upd_ms, upd_n = P.bkry_profile_read(h, P.PROF_CG_UPDATE)
    pup_ms, pup_n = P.bkry_profile_read(h, P.PROF_CG_PUPDATE)
    sp2_ms, sp2_n = P.bkry_profile_read(h, P.PROF_CG_SPMM)
    P.bkry_profile(h, False)
    blk = A.n * s * 8
    sp_bytes = spmm_bytes(A, s)
    sp_avg = spmm_ms / max(spmm_n, 1) * 1e-3
    achieved = sp_bytes / sp_avg / 1e9
    if args.solver == "cg1r":
        # fused pass: R, U, P, Q read, P, Q, R written, X read and written every
        # other iteration: 8 blocks on average
        upd_gbs = 8 * blk / (upd_ms / max(upd_n, 1) * 1e-3) / 1e9
        iter_bytes = sp_bytes + 8 * blk
        per_kernel = {"fused_pass": round(upd_gbs, 1)}
    else:
        upd_gbs = 3 * blk / (upd_ms / max(upd_n, 1) * 1e-3) / 1e9
        # the direction update moves 3 blocks (P, R read, P_{k+1} written) and, every
        # other iteration, 3 more (X read and written, P_{k-1} read): 4.5 on average
        pup_gbs = 4.5 * blk / (pup_ms / max(pup_n, 1) * 1e-3) / 1e9
        iter_bytes = sp_bytes + 7.5 * blk        # + residual pass (3 blocks) + direction pass (4.5 blocks)
        per_kernel = {"residual_update_gram": round(upd_gbs, 1), "direction_update": round(pup_gbs, 1)}
    traffic = pmc_traffic()
    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "block-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "laplace3d_128_s8: 3D 7-point Laplacian 128^3 (n=2097152, nnz=14581760), "
                               "p=8 uniform[-1,1] seed 1002, "
                               + ("one-reduction block CG" if args.solver == "cg1r" else "block CG")
                               + ", block subalgebra, eta=1e4, tol=1e-10, X0=0",
                   "global_batch": s, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "kernel": ROOFLINE_KERNEL + " (SpMM fused with the alpha Gram partials)",
                     "algorithmic_bytes_per_launch": sp_bytes,
                     "avg_launch_us": round(sp_avg * 1e6, 2), "launches_timed": spmm_n},
        "time_to_tol_s": round(ms_per_step / 1e3, 4),
        "iters_per_solve": infos[-1]["iters"],
        "reorth_per_solve": infos[-1]["reorth"],
        "true_relres_max": max(infos[-1]["true_relres"]),
        "cg_iteration_GBps_algorithmic": round(iter_bytes * value / 1e9, 1),
        "kernels_GBps": {"spmm_alpha_gram": round(achieved, 1),
                         "spmm_alpha_gram_all_timed": round(sp_bytes / (sp2_ms / max(sp2_n, 1) * 1e-3) / 1e9, 1),
                         **per_kernel},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(A, B)
        result["cpu_baseline"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in cb.items()
                                  if k != "seconds_per_iter"}
    if args.extras:
        result["extras"] = extras(P, W, h, dev, A, Ad, Bd, args)
    h.close()
    print(json.dumps(result), flush=True)


def timed(fn, reps):
    import torch
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    out = None
    for _ in range(reps):
        out = fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps, out


def extras(P, W, h, dev, A, Ad, Bd, args):
    import numpy as np
    import torch

    ex = {}
    s = Bd.shape[1]
    # hybrid subalgebra, q = 2 groups of 4
    X, info = P.bkry_cg_solve(h, Ad, Bd, kind="hybrid", q=2, tol=1e-10, maxit=args.maxit, eta=1e4)
    ex["cg_hybrid_q2"] = dict(iters=info["iters"], reorth=info["reorth"], seconds=round(info["seconds"], 4),
                              iters_per_s=round(info["iters"] / info["seconds"], 1),
                              true_relres_max=max(info["true_relres"]))
    log("hybrid", ex["cg_hybrid_q2"])
    # BDOT alone (block subalgebra), 2 blocks read
    Y = torch.randn_like(Bd)
    ms, _ = timed(lambda: P.bkry_bdot(h, Bd, Y, "block"), 20)
    ex["bdot_block_GBps"] = round(2 * A.n * s * 8 / (ms * 1e-3) / 1e9, 1)
    ex["bdot_block_us"] = round(ms * 1e3, 2)
    # SpMM alone (mode 0)
    ms, _ = timed(lambda: P.bkry_spmm(h, Ad, Bd, Y), 20)
    ex["spmm_plain_GBps"] = round(spmm_bytes(A, s) / (ms * 1e-3) / 1e9, 1)
    del Y
    # attainable HBM bandwidth: a plain device copy of 1 GiB
    try:
        xa = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        ya = torch.empty_like(xa)
        ms, _ = timed(lambda: ya.copy_(xa), 10)
        ex["hbm_copy_GBps"] = round(2 * xa.numel() * 8 / (ms * 1e-3) / 1e9, 1)
        del xa, ya
    except Exception as e:
        ex["hbm_copy_GBps"] = dict(error=str(e))
    # standalone TSQR 4,194,304 x 32
    try:
        Xt = torch.as_tensor(W.tsqr_input()).to(dev)
        Xw = torch.empty_like(Xt)

        def tsqr_once():
            Xw.copy_(Xt)
            return P.bkry_tsqr(h, Xw, "block")
        ms_copy, _ = timed(lambda: Xw.copy_(Xt), 5)
        ms, R = timed(tsqr_once, 5)
        ms -= ms_copy
        m, c = Xt.shape
        gbps = 2 * m * c * 8 / (ms * 1e-3) / 1e9
        tfl = 4 * m * c * c / (ms * 1e-3) / 1e12
        ex["tsqr_4194304x32"] = dict(ms=round(ms, 3), GBps_algorithmic=round(gbps, 1),
                                     TFLOPs_algorithmic=round(tfl, 2), hbm_frac=round(gbps / 8000.0, 4),
                                     fp64_mfma_frac=round(tfl / 78.6, 4),
                                     orth_err=float((Xw.T @ Xw - torch.eye(c, device=dev, dtype=Xw.dtype))
                                                    .abs().max()))
        del Xt, Xw
        log("tsqr", ex["tsqr_4194304x32"])
    except Exception as e:  # report, do not hide
        ex["tsqr_4194304x32"] = dict(error=str(e))
    # one-reduction block CG on the same 128^3 workload (same options as the headline solve)
    try:
        P.bkry_cg1r_solve(h, Ad, Bd, kind="block", tol=1e-10, maxit=args.maxit, eta=1e4)
        X1, i1 = P.bkry_cg1r_solve(h, Ad, Bd, kind="block", tol=1e-10, maxit=args.maxit, eta=1e4)
        P.bkry_profile(h, True)
        for k in range(4):
            P.bkry_profile_read(h, k, reset=True)
        P.bkry_cg1r_solve(h, Ad, Bd, kind="block", tol=1e-10, maxit=args.maxit, eta=1e4)
        sp_ms, sp_n = P.bkry_profile_read(h, P.PROF_CG_SPMM)
        fu_ms, fu_n = P.bkry_profile_read(h, P.PROF_CG_UPDATE)
        P.bkry_profile(h, False)
        blk = A.n * s * 8
        # fused pass: R, U, P, Q read, P, Q, R written, X read and written every
        # other iteration: 8 blocks on average
        ex["cg1r_laplace3d_128_s8"] = dict(
            iters=i1["iters"], reorth=i1["reorth"], seconds=round(i1["seconds"], 4),
            iters_per_s=round(i1["iters"] / i1["seconds"], 1), converged=i1["converged"],
            true_relres_max=max(i1["true_relres"]),
            spmm_us=round(sp_ms / max(sp_n, 1) * 1e3, 2),
            spmm_GBps=round(spmm_bytes(A, s) / (sp_ms / max(sp_n, 1) * 1e-3) / 1e9, 1),
            fused_pass_us=round(fu_ms / max(fu_n, 1) * 1e3, 2),
            fused_pass_GBps=round(8 * blk / (fu_ms / max(fu_n, 1) * 1e-3) / 1e9, 1))
        log("cg1r", ex["cg1r_laplace3d_128_s8"])
        del X1
    except Exception as e:
        ex["cg1r_laplace3d_128_s8"] = dict(error=str(e))
    # Gropp's block CG (Q and Z by recurrences) on the same 128^3 workload
    try:
        P.bkry_gropp_solve(h, Ad, Bd, kind="block", tol=1e-10, maxit=args.maxit, eta=1e4)
        Xg, ig = P.bkry_gropp_solve(h, Ad, Bd, kind="block", tol=1e-10, maxit=args.maxit, eta=1e4)
        ex["gropp_laplace3d_128_s8"] = dict(iters=ig["iters"], reorth=ig["reorth"], seconds=round(ig["seconds"], 4),
                                            iters_per_s=round(ig["iters"] / ig["seconds"], 1),
                                            converged=ig["converged"], true_relres_max=max(ig["true_relres"]))
        log("gropp", ex["gropp_laplace3d_128_s8"])
        del Xg
    except Exception as e:
        ex["gropp_laplace3d_128_s8"] = dict(error=str(e))
    # block GMRes(30): one cycle on the convection-diffusion workload
    try:
        Ac, Bc, _ = W.build_workload("convdiff2d_1024_s8")
        Acd = P.CsrMatrix.from_numpy(Ac.n, Ac.rowptr, Ac.colind, Ac.val, device=dev)
        Bcd = torch.as_tensor(Bc).to(dev)
        P.bkry_gmres_solve(h, Acd, Bcd, kind="block", tol=0.0, maxit=30, restart=30)
        Xg, gi = P.bkry_gmres_solve(h, Acd, Bcd, kind="block", tol=0.0, maxit=30, restart=30)
        Xg, gt = P.bkry_gmres_solve(h, Acd, Bcd, kind="block", tol=1e-10, maxit=6000, restart=30)
        ex["gmres30_convdiff1024"] = dict(cycle_ms=round(gi["seconds"] * 1e3, 2), solve_s=round(gt["seconds"], 3),
                                          steps=gt["iters"], cycles=gt["outer_iters"], converged=gt["converged"],
                                          true_relres_max=max(gt["true_relres"]), orthogonalisation="CGS2")
        log("gmres", ex["gmres30_convdiff1024"])
        # the same with the pipelined Gram-Schmidt of the thesis's experiment (window 3)
        P.bkry_gmres_solve(h, Acd, Bcd, kind="block", tol=0.0, maxit=30, restart=30, pipelined=3)
        Xg, pi = P.bkry_gmres_solve(h, Acd, Bcd, kind="block", tol=0.0, maxit=30, restart=30, pipelined=3)
        Xg, pt = P.bkry_gmres_solve(h, Acd, Bcd, kind="block", tol=1e-10, maxit=6000, restart=30, pipelined=3)
        ex["gmres30_pipelined3_convdiff1024"] = dict(
            cycle_ms=round(pi["seconds"] * 1e3, 2), solve_s=round(pt["seconds"], 3), steps=pt["iters"],
            cycles=pt["outer_iters"], converged=pt["converged"], true_relres_max=max(pt["true_relres"]),
            orthogonalisation="pipelined Gram-Schmidt, window 3")
        log("gmres pipelined", ex["gmres30_pipelined3_convdiff1024"])
        del Acd, Bcd, Xg
    except Exception as e:
        ex["gmres30_convdiff1024"] = dict(error=str(e))
    # block BiCGStab with adaptive re-orthonormalisation on the same workload
    try:
        Ac, Bc, _ = W.build_workload("convdiff2d_1024_s8")
        Acd = P.CsrMatrix.from_numpy(Ac.n, Ac.rowptr, Ac.colind, Ac.val, device=dev)
        Bcd = torch.as_tensor(Bc).to(dev)
        P.bkry_bicgstab_solve(h, Acd, Bcd, tol=0.0, maxit=10, eta=1e4)
        Xb, bi = P.bkry_bicgstab_solve(h, Acd, Bcd, tol=0.0, maxit=100, eta=1e4)
        Xb, bt = P.bkry_bicgstab_solve(h, Acd, Bcd, tol=1e-10, maxit=20000, eta=1e4)
        ex["bicgstab_convdiff1024"] = dict(ms_per_iter=round(bi["seconds"] / 100 * 1e3, 3),
                                           solve_s=round(bt["seconds"], 3), iters=bt["iters"],
                                           reorth=bt["reorth"], restarts=bt["outer_iters"],
                                           converged=bt["converged"], true_relres_max=max(bt["true_relres"]))
        log("bicgstab", ex["bicgstab_convdiff1024"])
        del Acd, Bcd, Xb
    except Exception as e:
        ex["bicgstab_convdiff1024"] = dict(error=str(e))
    # FP32-inner iterative refinement vs FP64 on the 27-point variable-coefficient workload
    try:
        A3, B3, _ = W.build_workload("diffusion27_96_s16")
        A3d = P.CsrMatrix.from_numpy(A3.n, A3.rowptr, A3.colind, A3.val, device=dev)
        B3d = torch.as_tensor(B3).to(dev)
        X64, i64 = P.bkry_cg_solve(h, A3d, B3d, kind="block", tol=1e-10, maxit=20000, eta=1e4)
        X32, i32 = P.bkry_cg_solve(h, A3d, B3d, kind="block", tol=1e-10, maxit=20000, eta=1.0, prec=P.F32_IR)
        err = float(torch.linalg.norm(X32 - X64) / torch.linalg.norm(X64))
        # the oracle takes minutes per iteration here: the reference of this
        # error is the FP64 solve on the same GPU (the oracle comparison runs in
        # the GPU tests on a 32^3 instance of the same generator)
        ex["ir_diffusion27_96_s16"] = dict(fp64_s=round(i64["seconds"], 3), fp64_iters=i64["iters"],
                                           ir_s=round(i32["seconds"], 3), ir_inner_iters=i32["iters"],
                                           ir_outer=i32["outer_iters"], ir_converged=i32["converged"],
                                           ir_true_relres_max=max(i32["true_relres"]),
                                           fp64_true_relres_max=max(i64["true_relres"]),
                                           speedup_vs_fp64=round(i64["seconds"] / i32["seconds"], 3),
                                           rel_err_vs_gpu_fp64_solve=err)
        log("ir", ex["ir_diffusion27_96_s16"])
        del A3d, B3d, X64, X32
    except Exception as e:
        ex["ir_diffusion27_96_s16"] = dict(error=str(e))
    # Jacobi-preconditioned block CG vs no preconditioner, 64^3 variable-coefficient workload
    try:
        A5, B5, _ = W.build_workload("diffusion7var_64_s32")
        A5d = P.CsrMatrix.from_numpy(A5.n, A5.rowptr, A5.colind, A5.val, device=dev)
        B5d = torch.as_tensor(B5).to(dev)
        minv = P.bkry_jacobi_minv(h, A5d)
        P.bkry_pcg_solve(h, A5d, B5d, minv, tol=1e-10, maxit=5000, eta=1e4)
        Xp, ip = P.bkry_pcg_solve(h, A5d, B5d, minv, tol=1e-10, maxit=5000, eta=1e4)
        Xn, i0 = P.bkry_cg_solve(h, A5d, B5d, tol=1e-10, maxit=5000, eta=1e4)
        # the unpreconditioned forward solve of the differentiable workload,
        # with the per-iteration split of its kernels
        P.bkry_profile(h, True)
        for k in range(4):
            P.bkry_profile_read(h, k, reset=True)
        Xn, i0p = P.bkry_cg_solve(h, A5d, B5d, tol=1e-10, maxit=5000, eta=1e4)
        kt = {nm: P.bkry_profile_read(h, k) for nm, k in (("spmm", P.PROF_CG_SPMM), ("update", P.PROF_CG_UPDATE),
                                                             ("pupdate", P.PROF_CG_PUPDATE))}
        P.bkry_profile(h, False)
        ex["cg_diffusion7var_64_s32"] = dict(
            iters=i0["iters"], seconds=round(i0["seconds"], 4),
            us_per_iter=round(i0["seconds"] / i0["iters"] * 1e6, 1),
            kernel_us={nm: round(ms / max(cnt, 1) * 1e3, 2) for nm, (ms, cnt) in kt.items()})
        log("cg s=32", ex["cg_diffusion7var_64_s32"])
        ex["pcg_jacobi_diffusion7var_64_s32"] = dict(
            iters=ip["iters"], reorth=ip["reorth"], seconds=round(ip["seconds"], 4),
            iters_per_s=round(ip["iters"] / ip["seconds"], 1), converged=ip["converged"],
            true_relres_max=max(ip["true_relres"]), unpreconditioned_iters=i0["iters"],
            unpreconditioned_seconds=round(i0["seconds"], 4))
        log("pcg", ex["pcg_jacobi_diffusion7var_64_s32"])
        # multicolour SSOR (omega = 1) on the same system
        prio = torch.as_tensor(W.color_priorities(A5.n, 64).view(np.int32)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        colors, ncol = P.bkry_color(h, A5d, prio)
        torch.cuda.synchronize()
        t_color = time.perf_counter() - t0
        P.bkry_pcg_ssor_solve(h, A5d, B5d, colors, 1.0, tol=1e-10, maxit=5000, eta=1e4)
        Xs, isr = P.bkry_pcg_ssor_solve(h, A5d, B5d, colors, 1.0, tol=1e-10, maxit=5000, eta=1e4)
        Y = torch.randn_like(B5d)
        ms_apply, _ = timed(lambda: P.bkry_ssor_apply(h, A5d, colors, 1.0, Y), 10)
        # per-iteration split inside the solve: the residual-update stage holds
        # the update pass, both colour sweeps, the <Z, R~> Gram and the reduction
        P.bkry_profile(h, True)
        for k in range(4):
            P.bkry_profile_read(h, k, reset=True)
        P.bkry_pcg_ssor_solve(h, A5d, B5d, colors, 1.0, tol=1e-10, maxit=5000, eta=1e4)
        up_ms, up_n = P.bkry_profile_read(h, P.PROF_CG_UPDATE)
        P.bkry_profile(h, False)
        ex["pcg_ssor_diffusion7var_64_s32"] = dict(
            iters=isr["iters"], reorth=isr["reorth"], seconds=round(isr["seconds"], 4),
            iters_per_s=round(isr["iters"] / isr["seconds"], 1), converged=isr["converged"],
            true_relres_max=max(isr["true_relres"]), colours=ncol, colouring_ms=round(t_color * 1e3, 2),
            ssor_apply_call_ms=round(ms_apply, 3),
            update_sweeps_gram_reduce_us=round(up_ms / max(up_n, 1) * 1e3, 1))
        log("pcg ssor", ex["pcg_ssor_diffusion7var_64_s32"])
        del A5d, B5d, Xp, Xn, minv, Xs, Y, colors
    except Exception as e:
        ex["pcg_jacobi_diffusion7var_64_s32"] = dict(error=str(e))
    # differentiable solve: forward + adjoint on the 64^3 variable-coefficient workload
    try:
        A5, B5, e5 = W.build_workload("diffusion7var_64_s32")
        A5d = P.CsrMatrix.from_numpy(A5.n, A5.rowptr, A5.colind, A5.val, device=dev)
        vals = A5d.val.clone().requires_grad_(True)
        B5d = torch.as_tensor(B5).to(dev).requires_grad_(True)
        T5 = torch.as_tensor(e5["target"]).to(dev)
        # two rounds, the second timed: the first backward pass of a process
        # also starts autograd and loads torch's elementwise kernels
        for _ in range(2):
            vals.grad = None
            B5d.grad = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X5 = P.block_solve(vals, B5d, A5d, h, tol=1e-10, eta=1e4)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            loss = 0.5 * ((X5 - T5) ** 2).sum()
            loss.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        ex["adjoint_diffusion7var_64_s32"] = dict(forward_s=round(t1 - t0, 4), backward_s=round(t2 - t1, 4))
        log("adjoint", ex["adjoint_diffusion7var_64_s32"])
    except Exception as e:
        ex["adjoint_diffusion7var_64_s32"] = dict(error=str(e))
    return ex


def copy_probe():
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = 1 << 27  # 1 GiB of float64
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8}))


PROFILE_WORKLOADS = ("cg32", "ir96", "tsqr", "gmres")


def profile_run(which):
    """Two runs of one workload, for kernel traces (rocprofv3 --kernel-trace):
    cg32   block CG, 64^3 variable-coefficient problem, 32 right-hand sides;
    ir96   FP64 block CG and FP32-inner IR, 27-point 96^3 problem, 16 right-hand sides;
    tsqr   the normaliser of a 4,194,304 x 32 Gaussian block (six calls);
    gmres  two GMRes(30) cycles on the 1024^2 convection-diffusion problem,
           classical Gram-Schmidt twice, then the pipelined form (window 3)."""
    import torch
    import paper_2104_02494_amd as P
    import workloads as W
    h = P.Handle(0)

    def dev(name):
        A, B, _ = W.build_workload(name)
        return P.CsrMatrix.from_numpy(A.n, A.rowptr, A.colind, A.val), torch.as_tensor(B).cuda()
    if which == "cg32":
        Ad, Bd = dev("diffusion7var_64_s32")
        for r in range(2):
            _, info = P.bkry_cg_solve(h, Ad, Bd, tol=1e-10, maxit=5000, eta=1e4)
            log("profile cg32", r, info["iters"], info["reorth"], round(info["seconds"], 4))
    elif which == "ir96":
        Ad, Bd = dev("diffusion27_96_s16")
        for r in range(2):
            _, i64 = P.bkry_cg_solve(h, Ad, Bd, tol=1e-10, maxit=20000, eta=1e4)
            _, i32 = P.bkry_cg_solve(h, Ad, Bd, tol=1e-10, maxit=20000, eta=1.0, prec=P.F32_IR)
            log("profile ir96", r, "fp64", i64["iters"], round(i64["seconds"], 4), "ir", i32["outer_iters"],
                i32["iters"], round(i32["seconds"], 4))
    elif which == "tsqr":
        Xt = torch.as_tensor(W.tsqr_input()).cuda()
        Xw = torch.empty_like(Xt)
        for r in range(6):
            Xw.copy_(Xt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.bkry_tsqr(h, Xw, "block")
            torch.cuda.synchronize()
            log("profile tsqr", r, round((time.perf_counter() - t0) * 1e3, 3), "ms")
    elif which == "gmres":
        Ad, Bd = dev("convdiff2d_1024_s8")
        for r in range(2):
            _, info = P.bkry_gmres_solve(h, Ad, Bd, tol=0.0, maxit=60, restart=30)
            log("profile gmres", r, info["iters"], round(info["seconds"], 4))
        for r in range(2):
            _, info = P.bkry_gmres_pipelined_solve(h, Ad, Bd, 3, tol=0.0, maxit=60, restart=30)
            log("profile gmres pipelined", r, info["iters"], round(info["seconds"], 4))
    h.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--maxit", type=int, default=5000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", dest="extras", action="store_true", default=True)
    ap.add_argument("--no-extras", dest="extras", action="store_false")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--profile", choices=PROFILE_WORKLOADS, default=None,
                    help="run one workload twice for a kernel trace and exit (no JSON line)")
    ap.add_argument("--solver", choices=["cg", "cg1r"], default="cg",
                    help="block CG of the timed solves: two reductions per iteration (default) or one")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solvers run on a single MI355X "
              "(no multi-GPU path); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.profile:
        profile_run(args.profile)
        return
    run(args)


if __name__ == "__main__":
    main()

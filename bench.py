#!/usr/bin/env python
"""Benchmark: FGMRES time-to-1e-6 and cell-iterations/s of CPTR-preconditioned
solves of the 64x64x32 two-phase thermal Jacobian (131,072 cells, 3x3 BSR
blocks, Gaussian ln k field, heated zone), FP32 preconditioner against FP64,
on one MI355X.

A step is one fgmres_solve of the resident system from a zero initial guess
to rtol 1e-6 (restriction, block preconditioner with three AMG V-cycles,
two-stage residual, BILU(0), FP64 Arnoldi with CGS2, Givens, solution update
and FP64 true-residual check).  The preconditioner setup is timed separately.

Prints one JSON line (see the keys below).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_roofline(pr, solver, reps=50):
    """Average duration of the FP64 BSR product (the Arnoldi w = A z of every
    step), timed with HIP events on the stream it is launched on, and its
    algorithmic bytes: values + column indices + row pointers + x + y.
    Repeated launches on one system: at 131k cells the 65 MB matrix fits the
    256 MB last-level cache, so the figure can exceed what HBM alone gives."""
    import torch
    from paper_1907_04229_amd import cptr
    n, nv = pr.n, pr.nv
    x = torch.randn(n * nv, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    st = torch.cuda.current_stream()
    for _ in range(5):
        cptr.cptr_bsr_spmv(n, nv, solver.rp, solver.ci, solver.vals, x, y, st)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        cptr.cptr_bsr_spmv(n, nv, solver.rp, solver.ci, solver.vals, x, y, st)
    e1.record(st)
    e1.synchronize()
    avg_s = e0.elapsed_time(e1) / reps * 1e-3
    nnzb = pr.nnzb
    algo = nnzb * (nv * nv * 8 + 4) + 4 * (n + 1) + 2 * 8 * n * nv
    gbs = algo / avg_s / 1e9
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4), traffic=None,
                kernel=f"k_bsr_spmv<{nv},double> (FP64 BSR y = A x)",
                bytes_per_launch=int(algo), avg_us=round(avg_s * 1e6, 2))


def cpu_baseline(pr, iters):
    """The FP64 oracle on the same system: setup excluded, FGMRES(30) capped at
    `iters` inner iterations (a bounded sample of the same solve)."""
    from oracle import oracle as O
    O.build(force=False)
    t0 = time.perf_counter()
    o = O.Oracle.from_problem(pr, first="cptr", second="bilu0_mc")
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, info = o.fgmres(pr.b, m=30, rtol=1e-6, maxit=iters)
    t = time.perf_counter() - t0
    o.close()
    return dict(value=round(pr.n * info["iters"] / t, 1), unit="cell-iters/s", cores=1,
                kind="oracle",
                sample=f"same {pr.n:,}-cell system, FP64 CPTR-Block(AMG)+BILU0(multicolour), "
                       f"FGMRES(30), {info['iters']} inner iterations (cap {iters}) in {t:.1f} s "
                       f"(setup {t_setup:.1f} s excluded), single thread")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="medium")
    ap.add_argument("--second", default="bilu0_mc")
    ap.add_argument("--cpu-iters", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the solver is a single-GPU library); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1907_04229_amd import cptr
    from paper_1907_04229_amd.synth import make_problem
    from paper_1907_04229_amd.synth.problem import CONFIGS

    cfg = CONFIGS[args.config]
    t0 = time.perf_counter()
    pr = make_problem(config=args.config)
    log(f"generated {args.config} {cfg['shape']} nv={pr.nv} nnzb={pr.nnzb} in "
        f"{time.perf_counter() - t0:.1f} s")
    restart = cfg["restart"]
    b = torch.as_tensor(pr.b, device="cuda")
    bnorm = float(np.linalg.norm(pr.b))

    def run(solver, steps, warmup, tag):
        for _ in range(warmup):
            solver.solve(b, restart=restart, rtol=1e-6)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(steps):
            x, info = solver.solve(b, restart=restart, rtol=1e-6)
            infos.append(info)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        it = infos[-1]["iters"]
        log(f"{tag}: {dt * 1e3:.2f} ms/solve, {it} iterations, true relres "
            f"{infos[-1]['relres_true']:.2e}")
        return dt, infos[-1], x

    t0 = time.perf_counter()
    s32 = cptr.Solver(pr, precision="fp32", second_stage=args.second)
    torch.cuda.synchronize()
    setup32 = time.perf_counter() - t0
    st32 = s32.stats()
    log(f"fp32 setup {setup32:.2f} s, AMG levels {st32['level_rows']}")
    dt32, info32, x32 = run(s32, args.steps, args.warmup, "fp32")
    assert info32["converged"] and info32["relres_true"] <= 1e-6

    res64 = None
    if not args.no_fp64:
        t0 = time.perf_counter()
        s64 = cptr.Solver(pr, precision="fp64", second_stage=args.second)
        torch.cuda.synchronize()
        setup64 = time.perf_counter() - t0
        dt64, info64, x64 = run(s64, max(1, min(args.steps, 3)), 1, "fp64")
        err = float(torch.linalg.vector_norm(x32 - x64) / torch.linalg.vector_norm(x64))
        res64 = dict(time_to_tol_s=round(dt64, 5), iters=info64["iters"],
                     cell_iters_per_s=round(pr.n * info64["iters"] / dt64, 1),
                     setup_s=round(setup64, 3), relres_true=info64["relres_true"],
                     fp32_vs_fp64_solution_rel_diff=err)
        s64.close()

    roof = kernel_roofline(pr, s32)
    log(f"roofline: {roof}")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(pr, args.cpu_iters)
        log(f"cpu baseline: {cpu}")
    out = {
        "metric": "FGMRES time-to-1e-6 (s) & cell-iters/s: learned/FP32 vs FP64 CPTR; HBM GB/s",
        "value": round(pr.n * info32["iters"] / dt32, 1),
        "unit": "cell-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt32 * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 preconditioner, f64 Krylov",
        "data": "synthetic (seeded thermal Jacobian of the first implicit step, Gaussian ln k field)",
        "config": {"workload": f"{args.config}: {'x'.join(map(str, cfg['shape']))} cells, "
                               f"nv={pr.nv}, FGMRES({restart}) rtol 1e-6, CPTR-Block(AMG)+"
                               f"{'BILU0 multicolour' if args.second == 'bilu0_mc' else 'BILU0'}",
                   "cells": pr.n, "nnzb": pr.nnzb, "restart": restart},
        "time_to_tol_s": round(dt32, 5),
        "iters": info32["iters"],
        "relres_true": info32["relres_true"],
        "setup_s": round(setup32, 3),
        "fp64": res64,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    s32.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

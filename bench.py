#!/usr/bin/env python
"""Benchmark: FGMRES time-to-1e-6 of the 128x128x64 two-phase thermal Jacobian
(1,048,576 cells, 3x3 BSR blocks, Gaussian ln k field with correlation length
8 cells and std 2.0) preconditioned by CPTR with the learned second stage and
an FP32 preconditioner, against plain FP64 CPTR (AMG V-cycles and BILU(0) in
natural order, all FP64), on one MI355X.

A step is one fgmres_solve of the resident system from a zero initial guess
to rtol 1e-6: restriction to p/T, the block preconditioner with three AMG
V-cycles, the two-stage residual, the learned second stage (three
message-passing layers), FP64 Arnoldi with CGS2, Givens rotations, the
solution update and the FP64 true-residual check.  Setup and training are
done before the timed region and reported separately.

Training (not timed): the network starts from the Neumann-series
initialisation and is trained by the library's own kernels on FGMRES Arnoldi
vectors of eight 64x64x32 systems with seeds 100-107 of the same field model
(the solved system, seed 200, is held out), keeping the parameters whose
learned-stage FGMRES solves of two validation systems of the solved size
(seeds 190, 191) take the fewest iterations in total.  After the timed run the 128x128x64 systems of seeds
200-204 are solved with the trained network, the untrained one and the
BILU(0) second stages, and their iterations and times reported (skipped with
`--no-held-out`).

Prints one JSON line (keys below).  `--probe` runs only a short learned
forward pass, the layer kernel and a plain device copy, for hardware-counter
runs of the profiler.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "learned_layer_traffic.json")
LAYER_SRC = os.path.join(ROOT, "paper_1907_04229_amd", "csrc", "learned_kernels.hip")
FIRST_NAME = {"cptr": "CPTR-Block", "cptr_lower": "CPTR-BlockLower", "cpr": "CPR", "cptr_bd": "CPTR-BD",
              "cptr_uamg": "CPTR-uAMG"}
TRAIN_SEED0 = 100  # --train-systems N takes the seeds 100 .. 100 + N - 1
VAL_SEEDS = (190, 191)  # validation fields of the model selection, at full size
HELD_OUT_SEEDS = (200, 201, 202, 203, 204)
TRAIN_SHAPE = (64, 64, 32)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def layer_source_hash():
    with open(LAYER_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def recorded_traffic(cells, nv):
    """HBM bytes per launch of the middle layer from the committed counter
    runs, if they were taken on the current kernel source, cell count and
    number of unknowns per cell."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if (rec.get("source_sha256") != layer_source_hash() or rec.get("cells") != cells
            or f"<{nv}," not in rec.get("kernel", "")):
        return None
    return rec.get("bytes_per_launch")


def layer_roofline(solver, reps=50):
    """Average duration of the middle layer kernel of the learned stage (BF16
    activations), timed with HIP events on the stream it is launched on,
    against its algorithmic HBM bytes: BF16 activations read and written
    (2 x 64 x 2 B) and six BF16 edge blocks (6 x 16 x 2 B) per cell, plus the
    presence mask (1 B) for the tile-order kernel.  On a grid whose planes are
    whole tiles of 16 cells the library runs the z-column kernel, which reads
    no mask."""
    import torch
    from paper_1907_04229_amd import cptr
    n, nv = solver.problem.n, solver.problem.nv
    nx, ny, _ = solver.problem.shape
    column = (nx * ny) % 16 == 0
    st = torch.cuda.current_stream()
    for _ in range(3):
        cptr.cptr_learn_rerun_layer(solver, 1, None, st)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        cptr.cptr_learn_rerun_layer(solver, 1, None, st)
    e1.record(st)
    e1.synchronize()
    avg_s = e0.elapsed_time(e1) / reps * 1e-3
    algo = n * (2 * 64 * 2 + 6 * 16 * 2 + (0 if column else 1))
    gbs = algo / avg_s / 1e9
    name = (f"k_lrn_layer_col<{nv},false,false,bf16> (message-passing layer, inference, z-column schedule)"
            if column else f"k_lrn_layer<{nv},false,false,bf16> (message-passing layer, inference)")
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4), traffic=recorded_traffic(n, nv), kernel=name,
                bytes_per_launch=int(algo), avg_us=round(avg_s * 1e6, 2), launches=reps)


def spmv_roofline(pr, solver, reps=50):
    """FP64 BSR product y = A x (the Arnoldi w = A z of every step, on the
    solver's sliced copy of A): average duration with HIP events, algorithmic
    bytes = values + column indices + row pointers + x + y of the BSR matrix."""
    import torch
    from paper_1907_04229_amd import cptr
    n, nv = pr.n, pr.nv
    x = torch.randn(n * nv, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    st = torch.cuda.current_stream()
    for _ in range(5):
        cptr.cptr_matvec(solver.h, x, y, st)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        cptr.cptr_matvec(solver.h, x, y, st)
    e1.record(st)
    e1.synchronize()
    avg_s = e0.elapsed_time(e1) / reps * 1e-3
    algo = pr.nnzb * (nv * nv * 8 + 4) + 4 * (n + 1) + 2 * 8 * n * nv
    gbs = algo / avg_s / 1e9
    return dict(kernel=f"k_bsr_spmv_sliced<{nv},double>", achieved=round(gbs, 1), unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4), bytes_per_launch=int(algo), avg_us=round(avg_s * 1e6, 2))


def cpu_baseline(pr, iters):
    """The FP64 oracle (plain CPTR: AMG + BILU(0) natural order) on the same
    system: setup excluded, FGMRES(30) capped at `iters` inner iterations."""
    from oracle import oracle as O
    O.build(force=False)
    t0 = time.perf_counter()
    o = O.Oracle.from_problem(pr, first="cptr", second="bilu0")
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, info = o.fgmres(pr.b, m=30, rtol=1e-6, maxit=iters)
    t = time.perf_counter() - t0
    o.close()
    return dict(value=round(pr.n * info["iters"] / t, 1), unit="cell-iters/s", cores=1,
                kind="oracle",
                sample=f"same {pr.n:,}-cell system, FP64 CPTR-Block(AMG)+BILU0(natural), FGMRES(30), "
                       f"first {info['iters']} inner iterations in {t:.1f} s (setup {t_setup:.1f} s "
                       f"excluded), single thread")


def train_model(cfg, steps, lr, systems, pairs, batch, first, log_fn, lr_final=None, rollback=None):
    from paper_1907_04229_amd.learned import train
    from paper_1907_04229_amd.synth import make_problem
    kw = {k: v for k, v in cfg.items() if k not in ("shape", "seed", "restart")}
    t0 = time.perf_counter()
    seeds = tuple(range(TRAIN_SEED0, TRAIN_SEED0 + systems))
    probs = [make_problem(shape=TRAIN_SHAPE, seed=s, **kw) for s in seeds]
    # model selection at the size of the solved system (one validation field)
    vseeds = VAL_SEEDS
    vprobs = [make_problem(shape=cfg["shape"], seed=s, **kw) for s in vseeds]
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    model, hist = train(probs, probs[0].nv, steps=steps, batch=batch, pairs=pairs, lr=lr, seed=1,
                        eval_every=50, val_problems=vprobs, val_restart=cfg["restart"], rollback=rollback,
                        lr_final=lr_final, precision="fp32", second_stage="bilu0_mc", first_stage=first)
    t_train = time.perf_counter() - t0
    log_fn(f"trained {steps} steps in {t_train:.1f} s (data {t_gen:.1f} s); validation "
           f"{[(k, round(v, 4), it) for k, v, it in hist['val']]}, kept step {hist['best_step']}")
    info = dict(train_s=round(t_train, 2), data_s=round(t_gen, 2), steps=steps, lr=lr, lr_final=lr_final,
                rollback=rollback, rollbacks=hist["rollbacks"],
                systems=f"{len(seeds)} x {'x'.join(map(str, TRAIN_SHAPE))}, seeds {seeds}", pairs=pairs,
                batch=batch,
                validation_systems=f"{len(vseeds)} x {'x'.join(map(str, cfg['shape']))}, seeds {vseeds}",
                val_loss_init=round(hist["val"][0][1], 5), val_iters_init=hist["val"][0][2],
                val_kept=[(k, round(v, 5), it) for k, v, it in hist["val"] if k == hist["best_step"]][0],
                kept_step=hist["best_step"])
    return model, info


def held_out_eval(cfg, model, restart, first, log_fn):
    """FGMRES iterations and time-to-1e-6 on the held-out 128x128x64 systems:
    learned (trained and untrained) with the FP32 preconditioner, BILU(0)
    natural order in FP64 (plain CPTR) and BILU(0) multicolour in FP32."""
    import torch
    from paper_1907_04229_amd import cptr
    from paper_1907_04229_amd.learned_init import neumann_params
    from paper_1907_04229_amd.synth import make_problem
    kw = {k: v for k, v in cfg.items() if k not in ("seed", "restart")}
    rows = []
    for seed in HELD_OUT_SEEDS:
        pr = make_problem(seed=seed, **kw)
        b = torch.as_tensor(pr.b, device="cuda")
        row = {"seed": seed}
        untrained = cptr.LearnModel(pr.nv, neumann_params(pr.nv, seed=1))
        for tag, opt, mdl in (("learned", dict(precision="fp32", second_stage="learned", first_stage=first), model),
                              ("untrained", dict(precision="fp32", second_stage="learned", first_stage=first),
                               untrained),
                              ("fp64_bilu0", dict(precision="fp64", second_stage="bilu0", first_stage="cptr"), None),
                              ("fp32_bilu0_mc", dict(precision="fp32", second_stage="bilu0_mc", first_stage=first),
                               None)):
            s = cptr.Solver(pr, **opt)
            if mdl is not None:
                mdl.attach(s)
            s.solve(b, restart=restart, rtol=1e-6)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = s.solve(b, restart=restart, rtol=1e-6)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            s.close()
            row[tag] = dict(iters=info["iters"], time_s=round(dt, 5), fell_back=info["fell_back"],
                            converged=bool(info["converged"] and info["relres_true"] <= 1e-6))
        untrained.close()
        log_fn(f"held-out seed {seed}: " + ", ".join(f"{k} {v['iters']} its {v['time_s'] * 1e3:.1f} ms"
                                                      for k, v in row.items() if k != "seed"))
        rows.append(row)
    return rows


def probe(cfg_name):
    """Short run for the hardware-counter passes: one learned forward, the
    middle layer three more times, and a 256 MiB device copy three times."""
    import torch
    from paper_1907_04229_amd import cptr
    from paper_1907_04229_amd.learned_init import neumann_params
    from paper_1907_04229_amd.synth import make_problem
    pr = make_problem(config=cfg_name)
    s = cptr.Solver(pr, precision="fp32", second_stage="learned")
    m = cptr.LearnModel(pr.nv, neumann_params(pr.nv, seed=1))
    m.attach(s)
    b1 = torch.randn(pr.n * pr.nv, dtype=torch.float64, device="cuda")
    cptr.cptr_learn_forward(s, b1)
    for _ in range(3):
        cptr.cptr_learn_rerun_layer(s, 1)
    a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    s.close()
    m.close()
    log(f"probe done: {pr.n} cells, copy of {a.numel() * 4} bytes")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="learned")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--train-lr", type=float, default=1e-5)
    ap.add_argument("--train-lr-final", type=float, default=1e-6,
                    help="step size at the last step (half-cosine decay from --train-lr)")
    ap.add_argument("--train-rollback", type=float, default=3.0,
                    help="continue from the kept parameters when the validation loss exceeds this "
                         "multiple of its lowest value (0: off)")
    ap.add_argument("--train-systems", type=int, default=8)
    ap.add_argument("--train-pairs", type=int, default=48)
    ap.add_argument("--train-batch", type=int, default=8)
    ap.add_argument("--first", default="cptr", choices=["cptr", "cptr_lower", "cpr", "cptr_bd", "cptr_uamg"],
                    help="first stage of the learned and BILU(0)-FP32 legs (plain FP64 CPTR stays cptr)")
    ap.add_argument("--cpu-iters", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 and BILU(0) legs")
    ap.add_argument("--no-held-out", action="store_true", help="skip the held-out seed evaluation")
    ap.add_argument("--probe", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the solver is a single-GPU library); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.probe:
        probe(args.config)
        return

    import torch
    from paper_1907_04229_amd import cptr
    from paper_1907_04229_amd.learned_init import neumann_params
    from paper_1907_04229_amd.synth import make_problem
    from paper_1907_04229_amd.synth.problem import CONFIGS

    cfg = CONFIGS[args.config]
    restart = cfg["restart"]
    t0 = time.perf_counter()
    pr = make_problem(config=args.config)
    log(f"generated {args.config} {cfg['shape']} nv={pr.nv} nnzb={pr.nnzb} in "
        f"{time.perf_counter() - t0:.1f} s")
    b = torch.as_tensor(pr.b, device="cuda")

    def run(solver, steps, warmup, tag, measured=False):
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
        info = infos[-1]
        log(f"{tag}: {dt * 1e3:.2f} ms/solve, {info['iters']} iterations, true relres "
            f"{info['relres_true']:.2e}, fell back {info['fell_back']}")
        # the measured configuration must converge; a comparison leg that does
        # not is reported as such
        if measured:
            assert info["converged"] and info["relres_true"] <= 1e-6, f"{tag} did not converge"
        return dt, info, x

    def setup(**opt):
        t0 = time.perf_counter()
        s = cptr.Solver(pr, **opt)
        torch.cuda.synchronize()
        return s, time.perf_counter() - t0

    def leg(dt, info, setup_s):
        return dict(time_to_tol_s=round(dt, 5), iters=info["iters"],
                    cell_iters_per_s=round(pr.n * info["iters"] / dt, 1), setup_s=round(setup_s, 3),
                    relres_true=info["relres_true"],
                    converged=bool(info["converged"] and info["relres_true"] <= 1e-6),
                    fell_back=info["fell_back"])

    model, train_info = train_model(cfg, args.train_steps, args.train_lr, args.train_systems,
                                    args.train_pairs, args.train_batch, args.first, log,
                                    lr_final=args.train_lr_final, rollback=args.train_rollback or None)

    # the measured configuration: learned second stage, FP32 preconditioner
    sl, setup_l = setup(precision="fp32", second_stage="learned", first_stage=args.first)
    model.attach(sl)
    dt, info, x_l = run(sl, args.steps, args.warmup, "learned+fp32", measured=True)
    roof = layer_roofline(sl)
    log(f"layer roofline: {roof}")

    compare = {}
    x64 = None
    if not args.no_compare:
        s64, su = setup(precision="fp64", second_stage="bilu0")
        d64, i64, x64 = run(s64, 1, 1, "plain fp64 (bilu0 natural)")
        compare["fp64_cptr_bilu0"] = leg(d64, i64, su)
        spmv = spmv_roofline(pr, s64)
        s64.close()
        smc, su = setup(precision="fp32", second_stage="bilu0_mc", first_stage=args.first)
        dmc, imc, _ = run(smc, 2, 1, "fp32 bilu0 multicolour")
        compare["fp32_cptr_bilu0_mc"] = leg(dmc, imc, su)
        smc.close()
        sn, su = setup(precision="fp32", second_stage="learned", first_stage=args.first)
        mn = cptr.LearnModel(pr.nv, neumann_params(pr.nv, seed=1))
        mn.attach(sn)
        dn, inn, _ = run(sn, 1, 1, "fp32 learned, untrained (Neumann init)")
        compare["fp32_cptr_learned_untrained"] = leg(dn, inn, su)
        sn.close()
        mn.close()
        # context: the same stages behind the CPR first stage (one A_pp V-cycle)
        # (also with the True-IMPES decoupling operator, Section 3.1), behind
        # the block-diagonal CPTR-BD(AMG) first stage (V-cycles on A_pp and
        # A_TT, Section 4.4), behind CPTR-uAMG (one V-cycle of the unknown-based
        # hierarchy of A_00, Section 3.4; also with True-IMPES extended to the
        # pressure-temperature system, Section 3.2), and CPTR with the BILU(1)
        # second stage
        for tag, first, opt, mdl_needed in (
                ("fp64_cpr_bilu0", "cpr", dict(precision="fp64", second_stage="bilu0"), False),
                ("fp32_cpr_bilu0_mc", "cpr", dict(precision="fp32", second_stage="bilu0_mc"), False),
                ("fp32_cpr_learned_untrained", "cpr", dict(precision="fp32", second_stage="learned"), True),
                ("fp64_cptr_bd_bilu0", "cptr_bd", dict(precision="fp64", second_stage="bilu0"), False),
                ("fp32_cptr_bd_bilu0_mc", "cptr_bd", dict(precision="fp32", second_stage="bilu0_mc"), False),
                ("fp64_cptr_uamg_bilu0", "cptr_uamg", dict(precision="fp64", second_stage="bilu0"), False),
                ("fp32_cptr_uamg_bilu0_mc", "cptr_uamg", dict(precision="fp32", second_stage="bilu0_mc"), False),
                ("fp64_cptr_uamg_ti_bilu0", "cptr_uamg", dict(precision="fp64", second_stage="bilu0",
                                                              decoupling="ti"), False),
                ("fp32_cptr_uamg_ti_bilu0_mc", "cptr_uamg", dict(precision="fp32", second_stage="bilu0_mc",
                                                                 decoupling="ti"), False),
                ("fp64_cpr_ti_bilu0", "cpr", dict(precision="fp64", second_stage="bilu0", decoupling="ti"),
                 False),
                ("fp32_cpr_ti_bilu0_mc", "cpr", dict(precision="fp32", second_stage="bilu0_mc", decoupling="ti"),
                 False),
                ("fp64_cptr_bilu1", args.first, dict(precision="fp64", second_stage="bilu0", ilu_level=1), False),
                ("fp32_cptr_bilu1_mc", args.first, dict(precision="fp32", second_stage="bilu0_mc", ilu_level=1),
                 False)):
            sc, su = setup(first_stage=first, **opt)
            mc_ = None
            if mdl_needed:
                mc_ = cptr.LearnModel(pr.nv, neumann_params(pr.nv, seed=1))
                mc_.attach(sc)
            dc, ic, _ = run(sc, 1, 1, tag)
            compare[tag] = leg(dc, ic, su)
            sc.close()
            if mc_ is not None:
                mc_.close()
        compare["speedup_vs_fp64"] = round(d64 / dt, 3)
        compare["solution_rel_diff_vs_fp64"] = float(torch.linalg.vector_norm(x_l - x64) /
                                                     torch.linalg.vector_norm(x64))
        compare["spmv_fp64"] = spmv
    held = None
    if not args.no_held_out:
        held = held_out_eval(cfg, model, restart, args.first, log)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(pr, args.cpu_iters)
        log(f"cpu baseline: {cpu}")
    out = {
        "metric": "FGMRES time-to-1e-6 (s) & cell-iters/s: learned/FP32 vs FP64 CPTR; HBM GB/s",
        "value": round(dt, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 preconditioner (bf16 MFMA in the learned stage), f64 Krylov",
        "data": "synthetic (seeded thermal Jacobian of the first implicit step, Gaussian ln k field)",
        "config": {"workload": f"{args.config}: {'x'.join(map(str, cfg['shape']))} cells, nv={pr.nv}, "
                               f"FGMRES({restart}) rtol 1e-6, {FIRST_NAME[args.first]}(AMG) + learned "
                               f"second stage, FP32 preconditioner",
                   "first_stage": args.first,
                   "cells": pr.n, "nnzb": pr.nnzb, "restart": restart},
        "iters": info["iters"],
        "cell_iters_per_s": round(pr.n * info["iters"] / dt, 1),
        "relres_true": info["relres_true"],
        "fell_back": info["fell_back"],
        "setup_s": round(setup_l, 3),
        "training": train_info,
        "compare": compare,
        "held_out": held,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    sl.close()
    model.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

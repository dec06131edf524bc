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
(seeds 190, 191) take the fewest iterations in total.  With `--held-out` the
128x128x64 systems of seeds 200-204 are then solved with the trained network,
the untrained one and the BILU(0) second stages, and their iterations and
times reported.

A second block measures the 128x128x64 three-phase case (nv = 4, ln k field
with std 2.5): plain FP64 CPTR with natural-order BILU(0) against CPTR with
the FP32 preconditioner whose BILU(0) is split into block-Jacobi parts of
whole grid columns (`--parts`, the parallel ILU(0) of the paper's
multi-process runs), with the two-stage residual and the rows of the ILU
solves summed in FP64.

Context of the Newton use (`newton` key): cptr_update_values on the measured
solver's options, on the GPU and on the host, and one implicit Euler step of
the thermal model on the workload's grid from its initial state with the
device Newton loop (assembly, GPU re-setup, CPTR-FGMRES, line search).

Prints one JSON line (keys below).  `--probe` runs only a short learned
forward pass, each layer kernel three more times, the FP64 BSR product and
a plain 1 GiB device copy, for hardware-counter runs of the profiler; `--traffic FETCH_DB WRITE_DB` turns
the two counter databases of such runs into the per-kernel traffic record.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "kernel_traffic_1M.json")
LAYER_SRC = os.path.join(ROOT, "paper_1907_04229_amd", "csrc", "learned_kernels.hip")
SPMV_SRC = os.path.join(ROOT, "paper_1907_04229_amd", "csrc", "device_kernels.hip")
COPY_BYTES = 1 << 30  # the reference copy of the counter runs (larger than the last-level cache)
FIRST_NAME = {"cptr": "CPTR-Block", "cptr_lower": "CPTR-BlockLower", "cptr_upper": "CPTR-BlockUpper", "cpr": "CPR",
              "cptr_bd": "CPTR-BD", "cptr_uamg": "CPTR-uAMG"}
TRAIN_SEED0 = 100  # --train-systems N takes the seeds 100 .. 100 + N - 1
VAL_SEEDS = (190, 191)  # validation fields of the model selection, at full size
HELD_OUT_SEEDS = (200, 201, 202, 203, 204)
TRAIN_SHAPE = (64, 64, 32)
HIDDEN = 64


# options of every solver the benchmark sets up (and of the oracle's
# hierarchy), from the command line
AMG_OPTS = {}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def layer_source_hash():
    return source_hash(LAYER_SRC)


def spmv_source_hash():
    return source_hash(SPMV_SRC)


def layer_method_bytes(layer, nv):
    """Bytes per cell that one inference launch of learned layer `layer`
    moves inside a solve (the method's, not the kernel's): the six nv x nv
    edge blocks in BF16; layer 0 reads r = D^{-1} b1 (nv FP32) and writes h1
    (64 BF16); layer 1 reads h1 and writes h2; layer 2 reads h2, r and the p
    and T components of the first stage's x1 (FP32) and writes z (nv FP32)."""
    edges = 6 * nv * nv * 2
    if layer == 0:
        return 4 * nv + edges + HIDDEN * 2
    if layer == 1:
        return HIDDEN * 2 + edges + HIDDEN * 2
    return HIDDEN * 2 + edges + 4 * nv + 2 * 4 + 4 * nv


def product_method_bytes(n, nnzb, nv, z_bytes=4):
    """The Arnoldi product w = A z inside the FP32-preconditioner solve: FP64
    blocks and block column indices, row pointers, z (FP32), w (FP64)."""
    return nnzb * (nv * nv * 8 + 4) + 4 * (n + 1) + n * nv * (z_bytes + 8)


def recorded_traffic(kernel, cells, nv):
    """HBM bytes per launch of a kernel (a learned layer 0, 1, 2, or "spmv",
    the FP64 BSR product) from the committed counter runs, if they were taken
    on the current kernel source, cell count and number of unknowns per cell."""
    try:
        with open(TRAFFIC_FILE) as f:
            recs = json.load(f)
    except (OSError, ValueError):
        return None
    src = spmv_source_hash() if kernel == "spmv" else layer_source_hash()
    for rec in recs.get("kernels", []):
        if (rec.get("layer") == kernel and rec.get("source_sha256") == src
                and rec.get("cells") == cells and rec.get("nv") == nv):
            return rec.get("bytes_per_launch")
    return None


LAYER_KERNEL = {0: "k_lrn_layer_first<{nv},true,false,short,float,float>",
                1: "k_lrn_layer_col<{nv},false,false,short,float,float>",
                2: "k_lrn_layer_col<{nv},false,true,short,float,float>"}
PRODUCT_KERNEL = "k_bsr_spmv_sliced<{nv},float,false>"


def in_solve_rooflines(solver, rhs, restart, solves=2):
    """Average duration of the Krylov product and of each learned layer as
    they run inside solves of the workload (cptr_kernel_timing: HIP events
    recorded by the library around every launch on the solve's stream; the
    timed solves run without graph replay), against the method's bytes per
    launch.  Returns one row per kernel."""
    from paper_1907_04229_amd import cptr
    n, nv, nnzb = solver.problem.n, solver.problem.nv, solver.problem.nnzb
    cptr.cptr_kernel_timing(solver.h, True)
    for _ in range(solves):
        solver.solve(rhs, restart=restart, rtol=1e-6)
    us, cnt = cptr.cptr_get_kernel_times(solver.h)
    cptr.cptr_kernel_timing(solver.h, False)
    rows = []
    for kid in range(4):
        # a kernel that did not run (the layers, once the learned stage has
        # fallen back to BILU(0)) has no row
        if cnt[kid] == 0 or not us[kid] > 0.0:
            continue
        if kid == 0:
            algo = product_method_bytes(n, nnzb, nv)
            name, per_cell, key = PRODUCT_KERNEL.format(nv=nv), None, "spmv"
        else:
            algo = n * layer_method_bytes(kid - 1, nv)
            name, per_cell, key = LAYER_KERNEL[kid - 1].format(nv=nv), layer_method_bytes(kid - 1, nv), kid - 1
        gbs = algo / (us[kid] * 1e-6) / 1e9
        rows.append(dict(kernel=name, layer=None if kid == 0 else kid - 1, achieved=round(gbs, 1), unit="GB/s",
                         frac=round(gbs / HBM_PEAK_GBS, 4), bytes_per_launch=int(algo),
                         method_bytes_per_cell=per_cell, avg_us=round(us[kid], 2), launches=int(cnt[kid]),
                         traffic=recorded_traffic(key, n, nv)))
    return rows


def resetup_times(pr, solver_opts):
    """cptr_update_values on the measured solver's options: the GPU re-setup
    (three calls, the last timed) and the host re-setup (one call), in ms."""
    import copy
    from paper_1907_04229_amd import cptr
    out = {}
    for tag, dev in (("gpu_ms", 1), ("host_ms", 0)):
        s = cptr.Solver(pr, resetup_device=dev, **AMG_OPTS, **solver_opts)
        for _ in range(3 if dev else 1):
            s.update_values(copy.copy(pr))
        out[tag] = round(cptr.cptr_get_stats(s.h)["setup_ms"], 1)
        s.close()
    return out


def newton_leg(cfg_name, log_fn):
    """One implicit Euler step of the thermal model on the device at the
    workload's grid (cptr_newton_solve: TPFA assembly, GPU re-setup,
    CPTR-FGMRES, line search), from the initial state, with two
    preconditioners; and the assembly kernel's time."""
    import torch
    from paper_1907_04229_amd import cptr
    from paper_1907_04229_amd.synth.problem import CONFIGS, build_model
    kw = dict(CONFIGS[cfg_name])
    shape = kw.pop("shape")
    m = build_model(shape, **kw)
    g, w = m.g, m.wells
    d = cptr.Model((g.nx, g.ny, g.nz), m.perm, m.poro, three_phase=m.three_phase, dt=m.dt, inj=w.inj,
                   prod=w.prod, heat=w.heat, dx=g.dx)
    x0 = torch.as_tensor(m.initial_state().reshape(-1), device="cuda")
    out = {"grid": "x".join(map(str, shape)), "cells": g.n, "dt_days": m.dt / 86400.0}
    st = torch.cuda.current_stream()
    for _ in range(2):
        d.assemble(x0, x0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(10):
        d.assemble(x0, x0)
    e1.record(st)
    e1.synchronize()
    out["assemble_ms"] = round(e0.elapsed_time(e1) / 10, 3)
    for tag, opts in (("fp32_cptr_bilu0_mc", dict(precision="fp32", second_stage="bilu0_mc")),
                      ("fp64_cptr_bilu0", dict(precision="fp64", second_stage="bilu0"))):
        x = x0.clone()
        s = d.solver(x, x0, **AMG_OPTS, **opts)
        info = d.newton(s, x, x0, max_it=20)
        log_fn(f"newton {tag}: {info['iters']} iterations ({info['lin_iters']} linear, {info['backtracks']} "
               f"halvings), {info['solve_ms']:.0f} ms, |F| {info['fnorm0']:.3e} -> {info['fnorm']:.3e}")
        out[tag] = dict(info, solve_ms=round(info["solve_ms"], 1))
        s.close()
    d.close()
    return out


def cpu_baseline(pr, maxit=None):
    """The FP64 oracle (plain CPTR: AMG + BILU(0) in natural order, FGMRES(30)
    to rtol 1e-6) on the same system, single thread, setup timed apart;
    `maxit` caps the inner iterations (None: to the tolerance)."""
    from oracle import oracle as O
    O.build(force=False)
    t0 = time.perf_counter()
    cs = AMG_OPTS.get("amg_coarse_size", 512)
    sw = AMG_OPTS.get("amg_sweeps", 2)
    swT = AMG_OPTS.get("amg_sweeps_T", 0) or sw
    o = O.Oracle.from_problem(pr, first="cptr", second="bilu0", coarse_size=cs, sweeps=sw, sweeps_T=swT)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, info = o.fgmres(pr.b, m=30, rtol=1e-6, maxit=maxit or 1000)
    t = time.perf_counter() - t0
    o.close()
    try:
        host = len(os.sched_getaffinity(0))
    except AttributeError:
        host = os.cpu_count()
    done = "to rtol 1e-6" if info["converged"] else f"capped at {info['iters']} inner iterations"
    return dict(value=round(t, 3), unit="s", cores=1, host_cores=host, kind="oracle",
                iters=info["iters"], converged=info["converged"], relres_true=info["relres_true"],
                setup_s=round(t_setup, 2), cell_iters_per_s=round(pr.n * info["iters"] / t, 1),
                sample=f"the whole {pr.n:,}-cell system, FP64 CPTR-Block(AMG, coarsest level <= {cs} rows, "
                       f"{sw} sweeps on A_pp, {swT} on S~_T)"
                       f"+BILU0(natural), FGMRES(30) "
                       f"{done} ({info['iters']} inner iterations), setup ({t_setup:.1f} s) excluded, "
                       f"one thread of the host's {host}")


def train_model(cfg, steps, lr, systems, pairs, batch, first, log_fn, lr_final=None, rollback=None,
                init="neumann"):
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
    from paper_1907_04229_amd.learned_init import init_params
    theta0 = init_params(probs[0].nv, seed=1) if init == "jacobi" else None
    model, hist = train(probs, probs[0].nv, steps=steps, batch=batch, pairs=pairs, lr=lr, seed=1, theta0=theta0,
                        eval_every=50, val_problems=vprobs, val_restart=cfg["restart"], rollback=rollback,
                        lr_final=lr_final, precision="fp32", second_stage="bilu0_mc", first_stage=first,
                        log=log_fn, **AMG_OPTS)
    t_train = time.perf_counter() - t0
    log_fn(f"trained {steps} steps in {t_train:.1f} s (data {t_gen:.1f} s); validation "
           f"{[(k, round(v, 4), it) for k, v, it in hist['val']]}, kept step {hist['best_step']}")
    info = dict(train_s=round(t_train, 2), data_s=round(t_gen, 2), steps=steps, init=init, lr=lr, lr_final=lr_final,
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
            s = cptr.Solver(pr, **AMG_OPTS, **opt)
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
    """Short run for the hardware-counter passes: a learned+FP32 solve of the
    workload cut at four FGMRES iterations (the Krylov product and the three
    layers as they run in the timed solve), and a 1 GiB device copy three
    times."""
    import torch
    from paper_1907_04229_amd import cptr
    from paper_1907_04229_amd.learned_init import neumann_params
    from paper_1907_04229_amd.synth import make_problem
    pr = make_problem(config=cfg_name)
    s = cptr.Solver(pr, precision="fp32", second_stage="learned", **AMG_OPTS)
    m = cptr.LearnModel(pr.nv, neumann_params(pr.nv, seed=1))
    m.attach(s)
    s.solve(torch.as_tensor(pr.b, device="cuda"), restart=30, rtol=1e-6, maxit=4)
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    s.close()
    m.close()
    log(f"probe done: {pr.n} cells, copy of {a.numel() * 4} bytes")


def trace_solves(cfg_name):
    """Two learned+FP32 solves of the workload (Neumann-series network), the
    second one to be read from a kernel trace (trace_summary)."""
    import torch
    from paper_1907_04229_amd import cptr
    from paper_1907_04229_amd.learned_init import neumann_params
    from paper_1907_04229_amd.synth import make_problem
    pr = make_problem(config=cfg_name)
    b = torch.as_tensor(pr.b, device="cuda")
    s = cptr.Solver(pr, precision="fp32", second_stage="learned", **AMG_OPTS)
    m = cptr.LearnModel(pr.nv, neumann_params(pr.nv, seed=1))
    m.attach(s)
    for k in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = s.solve(b, restart=30, rtol=1e-6)
        torch.cuda.synchronize()
        log(f"trace solve {k}: {info['iters']} iterations, {(time.perf_counter() - t0) * 1e3:.1f} ms")
    s.close()
    m.close()


def trace_summary(csv_path):
    """Markdown table of the kernels of the last FGMRES solve in a rocprofv3
    kernel trace (CSV) of `bench.py --trace`: the solve starts at the second
    half of the restart-cycle initialisations (k_cycle_init)."""
    import csv
    import re
    with open(csv_path) as f:
        rows = list(csv.DictReader(f))
    name_key = "Kernel_Name" if "Kernel_Name" in rows[0] else "Kernel Name"
    rows = [(r[name_key], int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows]
    rows.sort(key=lambda r: r[1])
    inits = [r[1] for r in rows if "k_cycle_init" in r[0]]
    t0 = inits[len(inits) // 2]
    # the solve's first kernels (the norm of b, the residual) come before its first cycle
    norms = [r[1] for r in rows if r[1] < t0 and "k_norm2_partial" in r[0]]
    t0 = norms[-2] if len(norms) >= 2 else t0
    sel = [r for r in rows if r[1] >= t0]
    iters = sum(1 for r in sel if "k_givens" in r[0])
    agg = {}
    for n, a, b in sel:
        k = re.sub(r"\(.*", "", n).replace("void ", "")
        c, t = agg.get(k, (0, 0.0))
        agg[k] = (c + 1, t + (b - a) / 1e3)
    tot = sum(t for _, t in agg.values())
    span = (sel[-1][2] - sel[0][1]) / 1e3
    out = [f"one solve: {iters} Arnoldi steps, {len(sel)} kernels, kernel time {tot:.0f} us, "
           f"span {span:.0f} us ({tot / max(iters, 1):.0f} us of kernels per step)", "",
           "| kernel | launches | total us | us per launch | us per step |", "|---|---|---|---|---|"]
    for k, (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| `{k}` | {c} | {t:.1f} | {t / c:.2f} | {t / max(iters, 1):.1f} |")
    return "\n".join(out)


def _counter_dispatches(db, counter):
    """(grid size, value) of every dispatch, by kernel name, for one hardware
    counter of a rocprofv3 database (rocpd schema)."""
    import sqlite3
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, grid_size, value from counters_collection where counter_name = ?",
                     (counter,)).fetchall()
    acc = {}
    for name, grid, v in rows:
        acc.setdefault(name, []).append((int(grid), float(v)))
    return acc


def _mean_of(disp, name, largest_grid=False):
    """Mean counter value per dispatch of kernel `name` (only the dispatches
    of its largest grid with largest_grid) and the number of dispatches."""
    d = disp[name]
    if largest_grid:
        g = max(x[0] for x in d)
        d = [x for x in d if x[0] == g]
    return sum(x[1] for x in d) / len(d), len(d)


def record_traffic(fetch_db, write_db, cells, nv, nnzb=None):
    """Per-launch HBM bytes of the three learned layers and the Krylov
    product, as they run in the timed solve, from a FETCH_SIZE and a
    WRITE_SIZE pass over `bench.py --probe`,
    each scaled by what the same counter reads for the probe's 1 GiB device
    copy (its largest-grid dispatches: COPY_BYTES read and written); written
    to TRAFFIC_FILE."""
    fetch = _counter_dispatches(fetch_db, "FETCH_SIZE")
    write = _counter_dispatches(write_db, "WRITE_SIZE")
    # the runtime's copy kernel (not the fill that made the source tensor)
    copy = [k for k in fetch if "copyBuffer" in k] or [k for k in fetch if "copy" in k.lower()]
    assert copy, "no device copy in the counter runs"
    ck = max(copy, key=lambda k: max(x[0] for x in fetch[k]))
    kib = COPY_BYTES / 1024.0
    fcopy, nfc = _mean_of(fetch, ck, True)
    wcopy, nwc = _mean_of(write, ck, True)
    fscale, wscale = kib / fcopy, kib / wcopy
    norm = lambda k: k.replace(" ", "")  # noqa: E731
    want = [(q, LAYER_KERNEL[q].format(nv=nv), "layer", cells * layer_method_bytes(q, nv)) for q in (0, 1, 2)]
    want.append(("spmv", PRODUCT_KERNEL.format(nv=nv), "spmv",
                 product_method_bytes(cells, nnzb, nv) if nnzb else None))
    kernels = []
    for key, tag, kind, method in want:
        names = [k for k in fetch if tag in norm(k)]
        assert len(names) == 1, (key, names)
        kn = names[0]
        f_kib, nf = _mean_of(fetch, kn)
        w_kib, nw = _mean_of(write, kn)
        fb, wb = f_kib * 1024 * fscale, w_kib * 1024 * wscale
        kernels.append(dict(layer=key, kernel=kn.split("(")[0], cells=cells, nv=nv,
                            source_sha256=spmv_source_hash() if kind == "spmv" else layer_source_hash(),
                            fetch_kib_raw=round(f_kib, 1), write_kib_raw=round(w_kib, 1),
                            fetch_bytes=int(fb), write_bytes=int(wb), bytes_per_launch=int(fb + wb),
                            launches_fetch=nf, launches_write=nw,
                            method_bytes=method))
    rec = dict(copy_kernel=ck.split("(")[0], copy_bytes=COPY_BYTES, copy_dispatches=[nfc, nwc],
               copy_fetch_kib_raw=round(fcopy, 1), copy_write_kib_raw=round(wcopy, 1),
               fetch_scale=round(fscale, 4), write_scale=round(wscale, 4),
               commands=["rocprofv3 --pmc FETCH_SIZE -d <dir> -o probe -- python3 -u bench.py --probe",
                         "rocprofv3 --pmc WRITE_SIZE -d <dir> -o probe -- python3 -u bench.py --probe"],
               kernels=kernels)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


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
    ap.add_argument("--train-batch", type=int, default=16)
    ap.add_argument("--train-init", default="neumann", choices=["neumann", "jacobi"],
                    help="start of training: the truncated Neumann series of block Jacobi, or block Jacobi "
                         "itself (random hidden layers, zero read-out)")
    ap.add_argument("--first", default="cptr",
                    choices=["cptr", "cptr_lower", "cptr_upper", "cpr", "cptr_bd", "cptr_uamg"],
                    help="first stage of the learned and BILU(0)-FP32 legs (plain FP64 CPTR stays cptr)")
    ap.add_argument("--amg-coarse-size", type=int, default=1024,
                    help="rows up to which an AMG level is the coarsest, solved with its explicit inverse "
                         "(every solver of the run and the oracle's hierarchy)")
    ap.add_argument("--amg-sweeps", type=int, default=3,
                    help="smoother sweeps before and after the coarse correction on every AMG level "
                         "(every solver of the run and the oracle's hierarchy)")
    ap.add_argument("--amg-sweeps-T", type=int, default=1,
                    help="smoother sweeps of the second (S~_T) hierarchy; 0: --amg-sweeps "
                         "(every solver of the run and the oracle's hierarchy)")
    ap.add_argument("--parts", default="16x16x1",
                    help="block-Jacobi grid parts of the partitioned BILU(0) legs (px x py x pz)")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="cap of the oracle's inner iterations in the CPU baseline (0: to the tolerance)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 and BILU(0) legs")
    ap.add_argument("--no-large", action="store_true", help="skip the three-phase 128x128x64 block")
    ap.add_argument("--no-newton", action="store_true",
                    help="skip the re-setup timings and the implicit step with the device Newton loop")
    ap.add_argument("--context", action="store_true",
                    help="also the context legs (CPR, CPTR-BD, CPTR-uAMG, decoupling, BILU(1))")
    ap.add_argument("--held-out", action="store_true", help="evaluate the held-out seeds 200-204")
    ap.add_argument("--probe", action="store_true")
    ap.add_argument("--trace", action="store_true",
                    help="only two learned+FP32 solves of the workload (untrained network), for a kernel trace")
    ap.add_argument("--trace-summary", metavar="KERNEL_TRACE_CSV",
                    help="per-kernel time of the last solve in a rocprofv3 kernel trace of --trace")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_DB", "WRITE_DB"))
    args = ap.parse_args()
    AMG_OPTS["amg_coarse_size"] = args.amg_coarse_size
    AMG_OPTS["amg_sweeps"] = args.amg_sweeps
    AMG_OPTS["amg_sweeps_T"] = args.amg_sweeps_T
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the solver is a single-GPU library); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.probe:
        probe(args.config)
        return
    if args.trace:
        trace_solves(args.config)
        return
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        return
    parts = tuple(int(q) for q in args.parts.split("x"))
    if args.traffic:
        from paper_1907_04229_amd.synth.problem import CONFIGS
        nx, ny, nz = CONFIGS[args.config]["shape"]
        nv = 4 if CONFIGS[args.config]["three_phase"] else 3
        # blocks of the 7-point pattern: the diagonal and both directions of every face
        nnzb = nx * ny * nz + 2 * ((nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1))
        print(json.dumps(record_traffic(args.traffic[0], args.traffic[1], nx * ny * nz, nv, nnzb), indent=1))
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

    def run(solver, steps, warmup, tag, rhs, measured=False):
        for _ in range(warmup):
            solver.solve(rhs, restart=restart, rtol=1e-6)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(steps):
            x, info = solver.solve(rhs, restart=restart, rtol=1e-6)
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

    def setup(prob, **opt):
        t0 = time.perf_counter()
        s = cptr.Solver(prob, **AMG_OPTS, **opt)
        torch.cuda.synchronize()
        return s, time.perf_counter() - t0

    def leg(dt, info, setup_s, n):
        return dict(time_to_tol_s=round(dt, 5), iters=info["iters"],
                    cell_iters_per_s=round(n * info["iters"] / dt, 1), setup_s=round(setup_s, 3),
                    relres_true=info["relres_true"],
                    converged=bool(info["converged"] and info["relres_true"] <= 1e-6),
                    fell_back=info["fell_back"])

    model, train_info = train_model(cfg, args.train_steps, args.train_lr, args.train_systems,
                                    args.train_pairs, args.train_batch, args.first, log,
                                    lr_final=args.train_lr_final, rollback=args.train_rollback or None,
                                    init=args.train_init)

    # the measured configuration: learned second stage, FP32 preconditioner
    sl, setup_l = setup(pr, precision="fp32", second_stage="learned", first_stage=args.first)
    model.attach(sl)
    dt, info, x_l = run(sl, args.steps, args.warmup, "learned+fp32", b, measured=True)
    kernels = in_solve_rooflines(sl, b, restart)
    for r in kernels:
        log(f"{r['kernel']}: {r['avg_us']} us in the solve, {r['achieved']} GB/s ({r['frac']:.2f} of peak)")
    resetup = None
    if not args.no_newton:
        resetup = resetup_times(pr, dict(precision="fp32", second_stage="learned", first_stage=args.first))
        log(f"re-setup (cptr_update_values): GPU {resetup['gpu_ms']} ms, host {resetup['host_ms']} ms")

    compare = {}
    x64 = None
    if not args.no_compare:
        s64, su = setup(pr, precision="fp64", second_stage="bilu0")
        d64, i64, x64 = run(s64, 1, 1, "plain fp64 (bilu0 natural)", b)
        compare["fp64_cptr_bilu0"] = leg(d64, i64, su, pr.n)
        s64.close()
        for tag, opt, mdl in (
                ("fp32_cptr_bilu0_mc", dict(precision="fp32", second_stage="bilu0_mc", first_stage=args.first),
                 False),
                ("fp32_cptr_learned_untrained", dict(precision="fp32", second_stage="learned",
                                                     first_stage=args.first), True),
                ("fp32_cptr_bilu0_parts", dict(precision="fp32", second_stage="bilu0", first_stage=args.first,
                                               ilu_parts=parts, resid_fp64=1, ilu_accum_fp64=1), False),
                ("fp64_cptr_bilu0_parts", dict(precision="fp64", second_stage="bilu0", ilu_parts=parts), False)):
            sc, su = setup(pr, **opt)
            mc_ = None
            if mdl:
                mc_ = cptr.LearnModel(pr.nv, neumann_params(pr.nv, seed=1))
                mc_.attach(sc)
            dc, ic, _ = run(sc, 1, 1, tag, b)
            compare[tag] = leg(dc, ic, su, pr.n)
            sc.close()
            if mc_ is not None:
                mc_.close()
        if args.context:
            # the same stages behind the CPR first stage (one A_pp V-cycle, also
            # with the True-IMPES decoupling operator, Section 3.1), behind the
            # block-diagonal CPTR-BD(AMG) first stage (Section 4.4), the block
            # triangular variants of eq:Aschur, CPTR-uAMG (Section 3.4; also with
            # True-IMPES on the pressure-temperature system, Section 3.2), and
            # CPTR with the BILU(1) second stage
            for tag, first, opt in (
                    ("fp64_cpr_bilu0", "cpr", dict(precision="fp64", second_stage="bilu0")),
                    ("fp32_cpr_bilu0_mc", "cpr", dict(precision="fp32", second_stage="bilu0_mc")),
                    ("fp64_cptr_lower_bilu0", "cptr_lower", dict(precision="fp64", second_stage="bilu0")),
                    ("fp64_cptr_upper_bilu0", "cptr_upper", dict(precision="fp64", second_stage="bilu0")),
                    ("fp64_cptr_bd_bilu0", "cptr_bd", dict(precision="fp64", second_stage="bilu0")),
                    ("fp32_cptr_bd_bilu0_mc", "cptr_bd", dict(precision="fp32", second_stage="bilu0_mc")),
                    ("fp64_cptr_uamg_bilu0", "cptr_uamg", dict(precision="fp64", second_stage="bilu0")),
                    ("fp32_cptr_uamg_bilu0_mc", "cptr_uamg", dict(precision="fp32", second_stage="bilu0_mc")),
                    ("fp64_cptr_uamg_ti_bilu0", "cptr_uamg", dict(precision="fp64", second_stage="bilu0",
                                                                  decoupling="ti")),
                    ("fp64_cpr_ti_bilu0", "cpr", dict(precision="fp64", second_stage="bilu0", decoupling="ti")),
                    ("fp64_cptr_bilu1", args.first, dict(precision="fp64", second_stage="bilu0", ilu_level=1)),
                    ("fp32_cptr_bilu1_mc", args.first, dict(precision="fp32", second_stage="bilu0_mc",
                                                            ilu_level=1))):
                sc, su = setup(pr, first_stage=first, **opt)
                dc, ic, _ = run(sc, 1, 1, tag, b)
                compare[tag] = leg(dc, ic, su, pr.n)
                sc.close()
        compare["speedup_vs_fp64"] = round(d64 / dt, 3)
        compare["solution_rel_diff_vs_fp64"] = float(torch.linalg.vector_norm(x_l - x64) /
                                                     torch.linalg.vector_norm(x64))

    large = None
    if not args.no_large:
        # the three-phase 1M-cell case: plain FP64 CPTR against FP32 CPTR
        t0 = time.perf_counter()
        pl = make_problem(config="large")
        log(f"generated large {CONFIGS['large']['shape']} nv={pl.nv} in {time.perf_counter() - t0:.1f} s")
        bl = torch.as_tensor(pl.b, device="cuda")
        large = {"workload": f"large: {'x'.join(map(str, CONFIGS['large']['shape']))} cells, three-phase, "
                             f"nv={pl.nv}, FGMRES({CONFIGS['large']['restart']}) rtol 1e-6", "cells": pl.n}
        # the FP32 legs form b1 and the rows of the ILU solves with FP64 sums
        # (FP32 sums: 81 iterations whole, 59 with b1 in FP64)
        for tag, opt, reps in (
                ("fp64_cptr_bilu0", dict(precision="fp64", second_stage="bilu0"), 1),
                ("fp32_cptr_bilu0_parts", dict(precision="fp32", second_stage="bilu0", ilu_parts=parts,
                                               resid_fp64=1, ilu_accum_fp64=1), 3),
                ("fp64_cptr_bilu0_parts", dict(precision="fp64", second_stage="bilu0", ilu_parts=parts), 1),
                ("fp32_cptr_bilu0", dict(precision="fp32", second_stage="bilu0", resid_fp64=1, ilu_accum_fp64=1), 1)):
            sc, su = setup(pl, **opt)
            dc, ic, _ = run(sc, reps, 1, f"large {tag}", bl)
            large[tag] = leg(dc, ic, su, pl.n)
            sc.close()
        large["speedup_fp32_parts_vs_fp64"] = round(large["fp64_cptr_bilu0"]["time_to_tol_s"] /
                                                    large["fp32_cptr_bilu0_parts"]["time_to_tol_s"], 3)
        large["parts"] = "x".join(map(str, parts))
        del pl, bl

    newton = None
    if not args.no_newton:
        newton = newton_leg(args.config, log)
        newton["resetup"] = resetup

    held = None
    if args.held_out:
        held = held_out_eval(cfg, model, restart, args.first, log)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(pr, args.cpu_iters or None)
        log(f"cpu baseline: {cpu}")
    # the roofline of the dominant kernel of the timed solve: each learned
    # layer and the Krylov product run once per FGMRES iteration
    cands = list(kernels)
    dom = max(cands, key=lambda r: r["avg_us"])
    roof = dict(bound="hbm", achieved=dom["achieved"], peak=HBM_PEAK_GBS, unit="GB/s", frac=dom["frac"],
                traffic=dom.get("traffic"), kernel=dom["kernel"], bytes_per_launch=dom["bytes_per_launch"],
                avg_us=dom["avg_us"], launches=dom.get("launches", 50),
                measured="inside two solves of the workload, HIP events around every launch (cptr_kernel_timing)",
                others=[{k: r[k] for k in ("kernel", "avg_us", "achieved", "frac", "bytes_per_launch", "traffic")}
                        for r in cands if r is not dom])
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
                   "first_stage": args.first, "amg_coarse_size": args.amg_coarse_size,
                   "amg_sweeps": args.amg_sweeps, "amg_sweeps_T": args.amg_sweeps_T,
                   "cells": pr.n, "nnzb": pr.nnzb, "restart": restart},
        "iters": info["iters"],
        "cell_iters_per_s": round(pr.n * info["iters"] / dt, 1),
        "relres_true": info["relres_true"],
        "fell_back": info["fell_back"],
        "setup_s": round(setup_l, 3),
        "training": train_info,
        "compare": compare,
        "large": large,
        "held_out": held,
        "newton": newton,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    sl.close()
    model.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

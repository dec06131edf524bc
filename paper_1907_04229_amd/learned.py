"""Training driver of the learned second stage (cptr_learn.h).

Training pairs are the inputs the second stage sees: b1 = v - A x1 with
x1 = M1^{-1} v the first-stage output, for the Arnoldi vectors v of FGMRES
solves.  Training starts from the truncated Neumann series of block Jacobi
(learned_init.neumann_params).  Every step of training (forward, loss, A^T
product, backward, Adam) runs in libcptr.
"""
import numpy as np

from . import cptr
from .learned_init import neumann_params

_SCALE = {"p": 1.0e4, "s": 1.0e-2, "T": 1.0}


def training_pairs(solver, count, seed, restart=30, rtol=1e-6):
    """(count, n*nv) FP64 device tensor of second-stage inputs for one system.

    The vectors the preconditioner sees inside FGMRES are the Arnoldi basis
    vectors v_j; each gives the pair input b1 = v_j - A M1^{-1} v_j, formed by
    the library's two-stage residual (cptr_stage_residual).  They are
    collected from FGMRES solves (with the solver's own second stage) of the
    Newton right-hand side and of products A x of random increments."""
    import torch
    pr = solver.problem
    n, nv = pr.n, pr.nv
    N = n * nv
    dev = solver.vals.device
    rng = np.random.Generator(np.random.PCG64(seed))
    scale = np.array([_SCALE["p"]] + [_SCALE["s"]] * (nv - 2) + [_SCALE["T"]])
    out = torch.empty((count, N), dtype=torch.float64, device=dev)
    v = torch.empty(N, dtype=torch.float64, device=dev)
    k, solves = 0, 0
    while k < count:
        if solves == 0:
            rhs = torch.as_tensor(pr.b, device=dev)
        else:
            x = torch.as_tensor((rng.standard_normal((n, nv)) * scale).reshape(-1), device=dev)
            rhs = torch.empty_like(x)
            cptr.cptr_bsr_spmv(n, nv, solver.rp, solver.ci, solver.vals, x, rhs)
        solves += 1
        _, info = solver.solve(rhs, restart=restart, rtol=rtol)
        last = info["iters"] - restart * info["restarts"]
        for j in range(min(last, restart)):
            if k == count:
                break
            cptr.cptr_krylov_vector(solver.h, j, v)
            # b1 = v - A M1^{-1} v as the second stage receives it (the
            # library's two-stage residual, in the solver's precision)
            cptr.cptr_stage_residual(solver.h, v, out[k])
            k += 1
        if solves > 4 * count:
            raise RuntimeError("FGMRES produced too few basis vectors for the training set")
    return out


def train(problems, nv, steps=200, batch=4, pairs=16, lr=1e-5, seed=0, log=None,
          theta0=None, val_frac=0.25, eval_every=25, val_problems=None, val_restart=30,
          rollback=None, lr_final=None, **solver_opts):
    """Train one model on the given systems.

    The pairs of every system are split into a training and a validation part
    (the last `val_frac` of them).  Model selection: with `val_problems`, the
    parameters (checked every `eval_every` steps, the initial ones included)
    whose FP32 learned-stage FGMRES(val_restart) solves of those systems to
    1e-6 take the fewest iterations in total are kept, ties broken by the
    validation loss; without them, the lowest validation loss.  Returns
    (model, history) with history = {"train": loss per step, "val":
    [(step, validation loss, iterations or None)], "best_step": step of the
    kept parameters, "rollbacks": steps at which training was rolled back}.

    rollback: when a validation loss is not finite or exceeds `rollback` times
    the lowest one so far, training continues from the kept parameters with a
    fresh Adam state (a divergence guard).  lr_final: the step size decays
    from `lr` to `lr_final` on a half cosine over the steps (constant when
    None).
    """
    import torch
    theta = neumann_params(nv, seed=seed) if theta0 is None else theta0
    model = cptr.LearnModel(nv, theta)
    sets = []
    for q, pr in enumerate(problems):
        s = cptr.Solver(pr, **solver_opts)
        model.attach(s)
        data = training_pairs(s, pairs, seed + 1000 + q)
        nval = int(round(val_frac * pairs))
        sets.append((s, data[:pairs - nval], data[pairs - nval:]))
    vsolv = []
    for pr in val_problems or ():
        opts = dict(solver_opts, precision="fp32", second_stage="learned")
        vs = cptr.Solver(pr, **opts)
        model.attach(vs)
        vsolv.append((vs, torch.as_tensor(pr.b, device=vs.vals.device)))

    def val_loss():
        tot, cnt = 0.0, 0
        for s, _, val in sets:
            if val.shape[0]:
                model.attach(s)
                tot += cptr.cptr_learn_grad(s, val, want_grad=False)[0] * val.shape[0]
                cnt += val.shape[0]
        return tot / cnt if cnt else float("nan")

    def val_iters():
        if not vsolv:
            return None
        total = 0
        for vs, b in vsolv:
            model.attach(vs)
            _, info = vs.solve(b, restart=val_restart, rtol=1e-6, maxit=10 * val_restart)
            # a fallback or no convergence counts as the iteration cap
            total += info["iters"] if info["converged"] and not info["fell_back"] else 10 * val_restart
        return total

    def key(v, it):
        return (it if it is not None else 0, v)

    rng = np.random.Generator(np.random.PCG64(seed + 7))
    hist = {"train": [], "val": [], "best_step": 0, "rollbacks": []}
    v0, i0 = val_loss(), val_iters()
    best = (key(v0, i0), model.params())
    lowest = v0
    hist["val"].append((0, v0, i0))

    def step_size(step):
        if lr_final is None or steps <= 1:
            return lr
        return lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * step / (steps - 1)))

    for step in range(steps):
        s, data, _ = sets[step % len(sets)]
        model.attach(s)
        idx = rng.choice(data.shape[0], size=min(batch, data.shape[0]), replace=False)
        loss = cptr.cptr_learn_train_step(s, data[idx], step_size(step))
        hist["train"].append(loss)
        if (step + 1) % eval_every == 0 or step == steps - 1:
            v, it = val_loss(), val_iters()
            hist["val"].append((step + 1, v, it))
            if key(v, it) < best[0]:
                best = (key(v, it), model.params())
                hist["best_step"] = step + 1
            if rollback is not None and (not np.isfinite(v) or v > rollback * lowest):
                model.set_params(best[1])  # and a fresh Adam state
                hist["rollbacks"].append(step + 1)
            elif np.isfinite(v):
                lowest = min(lowest, v)
            if log:
                log(f"step {step + 1}: train loss {loss:.4f}, validation loss {v:.4f}"
                    + (f", validation iterations {it}" if it is not None else ""))
    model.set_params(best[1])
    for s, _, _ in sets:
        s.close()
    for vs, _ in vsolv:
        vs.close()
    return model, hist

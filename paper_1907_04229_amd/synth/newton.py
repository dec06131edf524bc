"""Newton's method with a backtracking line search for one implicit step of
the thermal model, on the CPU (numpy residual, complex-step Jacobian, direct
sparse solves): the host counterpart of the library's cptr_newton_solve, used
to check it.  Section 3 solves each implicit step by Newton's method with a
line search, to relative function and step tolerances of 1e-8.

Per iterate: dx = -J(x)^{-1} F*(x); lambda = 1, 1/2, ... until
||F*(x + lambda dx)|| <= (1 - 1e-4 lambda) ||F*(x)||; stop when
||F*(x)|| <= rtol ||F*(x0)|| or ||lambda dx|| <= stol ||x||.
"""
import numpy as np


def jacobian_csr(model, x, xn):
    """The Jacobian at x as a scipy CSR matrix of the n nv unknowns."""
    import scipy.sparse as sp
    rp, col, vals = model.jacobian(x, xn)
    nv = model.nv
    return sp.bsr_matrix((vals, col, rp), shape=(model.g.n * nv, model.g.n * nv)).tocsr()


def newton_step(model, x0, xn, rtol=1e-8, stol=1e-8, max_it=50, max_backtrack=10):
    """Returns (x, info) for one implicit step from the guess x0 ((n, nv) array)."""
    from scipy.sparse.linalg import spsolve
    x = np.array(x0, dtype=float)
    F = model.residual(x, xn).reshape(-1)
    f0 = f = float(np.linalg.norm(F))
    info = dict(iters=0, backtracks=0, converged=f == 0.0, fnorm0=f0)
    while not info["converged"] and info["iters"] < max_it:
        dx = spsolve(jacobian_csr(model, x, xn), -F).reshape(x.shape)
        lam, ok = 1.0, False
        for _ in range(max_backtrack + 1):
            xt = x + lam * dx
            Ft = model.residual(xt, xn).reshape(-1)
            ft = float(np.linalg.norm(Ft))
            if np.isfinite(ft) and ft <= (1.0 - 1e-4 * lam) * f:
                ok = True
                break
            lam *= 0.5
            info["backtracks"] += 1
        info["iters"] += 1
        if not ok:
            break
        step = lam * float(np.linalg.norm(dx))
        x, F, f = xt, Ft, ft
        info["converged"] = f <= rtol * f0 or step <= stol * float(np.linalg.norm(x))
    info["fnorm"] = f
    return x, info

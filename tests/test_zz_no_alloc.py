"""fgmres_solve_static (the entry point that allocates nothing) against
fgmres_solve, through the C ABI: two calls in a row on one GPU, the second on
a smaller system, and a request beyond the static workspace.

Bar: the same kernels in the same order on the same inputs, so the same
iteration count and a solution within 1e-12 (relative 2-norm) of the
fgmres_solve one, in FP64 and with the FP32 preconditioner; for FP64 also
the oracle's bar (iterations within +-1, solution within 1e-8).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1907_04229_amd import cptr  # noqa: E402
from paper_1907_04229_amd.synth import make_problem  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _check(pr, precision, second, rhs):
    print(f"\n[no-alloc] {pr.shape} nv={pr.nv} {precision} {second}", flush=True)
    s = cptr.Solver(pr, device=DEV, precision=precision, second_stage=second)
    b = _dev(rhs)
    x_ref, i_ref = s.solve(b, restart=30, rtol=1e-6)
    x = torch.full_like(b, 7.0)   # overwritten: zero initial guess
    info = cptr.fgmres_solve_static(s.h, b, x, restart=30, rtol=1e-6)
    torch.cuda.synchronize()
    d = float(torch.linalg.vector_norm(x - x_ref) / torch.linalg.vector_norm(x_ref))
    print(f"iters static {info['iters']} handle {i_ref['iters']}, rel diff {d:.2e}", flush=True)
    assert info["converged"] and info["relres_true"] <= 1e-6
    assert info["iters"] == i_ref["iters"] and d <= 1e-12
    if precision == "fp64":
        o = O.Oracle.from_problem(pr, first="cptr", second=second)
        xo, io = o.fgmres(rhs, m=30, rtol=1e-6)
        err = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
        assert abs(info["iters"] - io["iters"]) <= 1 and err <= 1e-8
        o.close()
    s.close()


@pytest.mark.parametrize("precision,second", [("fp64", "bilu0"), ("fp32", "bilu0_mc")])
def test_static_workspace_two_calls_second_smaller(precision, second):
    big = make_problem(shape=(24, 20, 10), kind="gaussian", sigma=2.0, corr_len=4.0, seed=61)
    small = make_problem(shape=(7, 5, 3), kind="iid", seed=62, heater=True)
    assert small.n < big.n
    _check(big, precision, second, big.b)
    _check(small, precision, second, small.b_star)


def test_static_workspace_rejects_a_system_beyond_it():
    print("\n[no-alloc] beyond the static workspace", flush=True)
    pr = make_problem(shape=(7, 5, 3), kind="iid", seed=62)
    s = cptr.Solver(pr, device=DEV, precision="fp64", second_stage="bilu0")
    b = _dev(pr.b)
    x = torch.zeros_like(b)
    # restart 64 on this grid fits; the limit is reached through the byte count
    info = cptr.fgmres_solve_static(s.h, b, x, restart=64, rtol=1e-6)
    assert info["converged"]
    s.close()
    big = make_problem(shape=(64, 64, 32), kind="iid", seed=63)     # 393,216 unknowns, FP64
    s = cptr.Solver(big, device=DEV, precision="fp64", second_stage="bilu0")
    b = _dev(big.b)
    x = torch.zeros_like(b)
    with pytest.raises(cptr.CptrError) as e:
        cptr.fgmres_solve_static(s.h, b, x, restart=64)           # 65 x 393,216 x 8 B > 256 MiB
    assert e.value.code == -1
    info = cptr.fgmres_solve_static(s.h, b, x, restart=30, rtol=1e-6)
    assert info["converged"] and info["relres_true"] <= 1e-6
    s.close()

"""The thermal model on the GPU (cptr_model.h) against the CPU generator
(paper_1907_04229_amd.synth): residual F*, Jacobian and S~_T assembly, and
implicit time steps of the device Newton loop (cptr_newton_solve: assembly,
GPU re-setup, CPTR-FGMRES, line search) against the CPU Newton loop with
direct solves.

Tolerances.  Both assemblies evaluate the same formulas in FP64; the CPU
differentiates by complex step, the GPU in forward mode, both exact up to
rounding, and the two sum a row's contributions in the same order.  Their
differences are rounding differences of a few units in the last place of
the larger contributions, so each row kind (and each block position of the
Jacobian) is compared against 1e-10 of its largest magnitude over the grid.
Two Newton loops that both stop at ||F*|| <= 1e-8 ||F*(x0)|| (or at a step
below 1e-8 ||x||) differ by at most the sum of the Newton corrections left at
their end points, J^-1 F* at each (first order in F*); that sum, per kind of
unknown, is the bound on their distance."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1907_04229_amd import cptr  # noqa: E402
from paper_1907_04229_amd.synth.newton import jacobian_csr, newton_step  # noqa: E402
from paper_1907_04229_amd.synth.problem import build_model  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"

CASES = {
    # two-phase, injector, producer and a heated corner column block
    "two": dict(shape=(12, 10, 6), kind="gaussian", sigma=2.0, corr_len=3.0, seed=53, heater=True),
    # three-phase (nv = 4); a short step keeps Newton without saturation chopping convergent
    "three": dict(shape=(6, 6, 4), kind="gaussian", sigma=2.0, corr_len=3.0, seed=52, three_phase=True,
                  dt_days=0.1),
    # ragged odd sizes
    "ragged": dict(shape=(7, 5, 3), kind="iid", seed=54, heater=True),
    # a single column: z faces only, injector and producer in the same cells
    "column": dict(shape=(1, 1, 9), kind="iid", seed=55),
}


def banner(msg):
    print(f"\n[gpu-model] {msg}", flush=True)


def dev_model(m):
    g, w = m.g, m.wells
    return cptr.Model((g.nx, g.ny, g.nz), m.perm, m.poro, three_phase=m.three_phase, dt=m.dt, inj=w.inj,
                      prod=w.prod, heat=w.heat, dx=g.dx, device=DEV)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device=DEV)


def state(m, kind, seed=61):
    x = m.initial_state()
    if kind == "perturbed":
        rng = np.random.default_rng(seed)
        scale = np.array([1.0e5] + [0.02] * (m.nv - 2) + [2.0])
        x = x + rng.uniform(-1.0, 1.0, x.shape) * scale
    return x


def worst(a, b, axis_scale):
    """max |a - b| / (max |b| of its kind) over the kinds along the last axis."""
    d = np.abs(a - b).reshape(-1, axis_scale)
    s = np.abs(b).reshape(-1, axis_scale).max(axis=0)
    return float((d.max(axis=0) / np.maximum(s, 1e-300)).max())


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("kind", ["initial", "perturbed"])
def test_assembly_matches_the_generator(name, kind):
    banner(f"assembly {name} {kind}")
    m = build_model(**CASES[name])
    d = dev_model(m)
    xn = m.initial_state()
    x = state(m, kind)
    rp, col, slot = m.g.bsr_pattern()
    assert np.array_equal(d.row_ptr, rp) and np.array_equal(d.col_idx, col)
    F, A, S = d.assemble(dev(x), dev(xn))
    Fc = m.residual(x, xn).reshape(-1)
    _, _, Jc = m.jacobian(x, xn)
    _, _, Sc = m.schur_approx(x)
    torch.cuda.synchronize()
    nv = m.nv
    ef = worst(F.cpu().numpy(), Fc, nv)
    ej = worst(A.cpu().numpy(), Jc.reshape(-1), nv * nv)
    es = worst(S.cpu().numpy(), Sc, 1)
    print(f"residual {ef:.1e}  Jacobian {ej:.1e}  S~_T {es:.1e}")
    assert ef <= 1e-10 and ej <= 1e-10 and es <= 1e-10
    d.close()


@pytest.mark.parametrize("name,precision", [("two", "fp64"), ("two", "fp32"), ("three", "fp64")])
def test_newton_steps_match_the_cpu_newton(name, precision):
    """Two implicit steps on the device (the handle set up once at the initial
    state, re-set up on the GPU at every Newton iterate) against the CPU loop,
    each step from the same previous state."""
    from scipy.sparse.linalg import spsolve
    banner(f"newton {name} {precision}")
    m = build_model(**CASES[name])
    d = dev_model(m)
    xn = m.initial_state()
    xg, xng = dev(xn), dev(xn)
    opts = dict(precision=precision, second_stage="bilu0")
    if precision == "fp32":
        opts.update(resid_fp64=1)
    s = d.solver(xg, xng, **opts)
    xc_prev = xn
    for step in range(2):
        info = d.newton(s, xg, xng)
        xc, ic = newton_step(m, xc_prev, xc_prev)
        xgh = xg.cpu().numpy().reshape(xn.shape)
        print(f"step {step}: gpu {info['iters']} its ({info['lin_iters']} linear, {info['backtracks']} halvings, "
              f"{info['solve_ms']:.0f} ms), cpu {ic['iters']} its; |F| {info['fnorm0']:.3e} -> {info['fnorm']:.3e}")
        assert info["converged"] and ic["converged"]
        assert abs(info["iters"] - ic["iters"]) <= 2
        xprev_g = xng.cpu().numpy().reshape(xn.shape)
        Fg = m.residual(xgh, xprev_g).reshape(-1)
        Fc = m.residual(xc, xc_prev).reshape(-1)
        cg = np.abs(spsolve(jacobian_csr(m, xgh, xprev_g), Fg)).reshape(xn.shape).max(axis=0)
        cc = np.abs(spsolve(jacobian_csr(m, xc, xc_prev), Fc)).reshape(xn.shape).max(axis=0)
        inc = np.abs(xc - xc_prev).max(axis=0)
        dist = np.abs(xgh - xc).max(axis=0)
        bound = 2.0 * (cg + cc) + 1e-9 * inc
        print(f"  distance {dist} bound {bound}")
        assert np.all(dist <= bound)
        # the next step: both sides from the GPU's state (the same nonlinear
        # system, so that the bound above covers the step alone)
        xng.copy_(xg)
        xc_prev = xgh
    s.close()
    d.close()


def test_newton_rejects_a_handle_of_another_pattern():
    banner("newton, wrong handle")
    m = build_model(**CASES["ragged"])
    other = build_model(**CASES["two"])
    d, e = dev_model(m), dev_model(other)
    x = dev(m.initial_state())
    xo = dev(other.initial_state())
    s = e.solver(xo, xo, precision="fp64", second_stage="bilu0")
    with pytest.raises(cptr.CptrError) as err:
        d.newton(s, x, x.clone())
    assert err.value.code == -1
    s.close()
    d.close()
    e.close()

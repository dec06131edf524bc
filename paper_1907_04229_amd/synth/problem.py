"""Seeded synthetic linear systems of the thermal Newton step.

`make_problem` builds the Jacobian A (BSR), b = -F*(x0), the assembled Schur
approximation S~_T (CSR) and a manufactured right-hand side b* = A x_true, for
the first Newton iterate of the first implicit Euler step from the uniform
initial state (p0 = 4.1369e7 Pa, T0 = 288.706 K, S_o = 0.9 two-phase or
(S_w, S_g) = (0.1, 0.05) three-phase, dt = 10 days, 0.5 m cubic cells, gravity
along -z).  Wells: a hot-water injector completed over all layers of cell
column (0, 0) and a Peaceman producer over column (nx-1, ny-1); optionally a
heated 3x3 column block at the injector corner.

Named workloads (sizes and fields; see `CONFIGS`):
  small   10x10x5,   two-phase, nv=3, iid ln k (sigma 1.0)
  medium  64x64x32,  two-phase, nv=3, Gaussian field l=8 sigma 2.0, heaters
  large   128x128x64, three-phase, nv=4, Gaussian field l=8 sigma 2.5
  learned 128x128x64, two-phase, nv=3, Gaussian field l=8 sigma 2.0
  stress  256x256x64, three-phase, nv=4, channelised facies (1e4 contrast)
"""
from dataclasses import dataclass, field
import numpy as np

from .fields import make_fields
from .model import DAY, Grid, ThermalModel, Wells
from . import props as P

CONFIGS = {
    "small": dict(shape=(10, 10, 5), three_phase=False, kind="iid", sigma=1.0,
                  corr_len=8.0, seed=1, heater=False, restart=30),
    "medium": dict(shape=(64, 64, 32), three_phase=False, kind="gaussian", sigma=2.0,
                   corr_len=8.0, seed=2, heater=True, restart=30),
    "large": dict(shape=(128, 128, 64), three_phase=True, kind="gaussian", sigma=2.5,
                  corr_len=8.0, seed=3, heater=False, restart=30),
    "learned": dict(shape=(128, 128, 64), three_phase=False, kind="gaussian", sigma=2.0,
                    corr_len=8.0, seed=200, heater=False, restart=30),
    "stress": dict(shape=(256, 256, 64), three_phase=True, kind="channelised", sigma=1.0,
                   corr_len=(32.0, 4.0, 2.0), seed=5, heater=False, restart=50),
}

# typical increment magnitude of each unknown kind, used for x_true
_SCALE_P, _SCALE_S, _SCALE_T = 1.0e4, 1.0e-2, 1.0


@dataclass
class Problem:
    shape: tuple
    nv: int
    row_ptr: np.ndarray      # int32 [n+1]
    col_idx: np.ndarray      # int32 [nnzb]
    vals: np.ndarray         # float64 [nnzb*nv*nv], row-major blocks
    st_row_ptr: np.ndarray   # int32 [n+1]
    st_col_idx: np.ndarray   # int32 [nnz]
    st_vals: np.ndarray      # float64 [nnz]
    b: np.ndarray            # float64 [n*nv], -F*(x0), interleaved
    b_star: np.ndarray       # float64 [n*nv], A @ x_true
    x_true: np.ndarray       # float64 [n*nv]
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.row_ptr.size - 1

    @property
    def nnzb(self):
        return self.col_idx.size


def bsr_matvec(row_ptr, col, vals, nv, x):
    """y = A x for a BSR matrix (used only to manufacture b*)."""
    n = row_ptr.size - 1
    blocks = vals.reshape(-1, nv, nv)
    xb = x.reshape(-1, nv)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    contrib = np.einsum("kij,kj->ki", blocks, xb[col])
    y = np.zeros((n, nv))
    for r in range(nv):
        y[:, r] = np.bincount(rows, weights=contrib[:, r], minlength=n)
    return y.reshape(-1)


def build_model(shape, three_phase=False, kind="iid", sigma=1.0, corr_len=8.0,
                seed=1, heater=False, frozen_props=False, wells=True, dt_days=10.0, **_):
    nx, ny, nz = shape
    grid = Grid(nx, ny, nz)
    perm, poro = make_fields(shape, kind, seed, sigma=sigma, corr_len=corr_len)
    if wells:
        inj = [grid.cell(0, 0, k) for k in range(nz)]
        prod = [grid.cell(nx - 1, ny - 1, k) for k in range(nz)] if grid.n > 1 else []
    else:
        inj, prod = [], []
    heat = []
    if heater:
        heat = [grid.cell(i, j, k) for k in range(nz)
                for j in range(min(3, ny)) for i in range(min(3, nx))]
    phases = None
    if frozen_props:
        base = [P.WATER, P.GAS, P.OIL] if three_phase else [P.WATER, P.OIL]
        phases = [P.frozen_T(ph) for ph in base]
    return ThermalModel(grid, perm, poro, three_phase=three_phase,
                        wells=Wells(inj, prod, heat), phases=phases, dt=dt_days * DAY)


def make_problem(shape=None, config=None, xtrue_seed=None, state=None, **kw):
    """Build the linear system of one Newton iterate.

    Either a named config (see CONFIGS) or explicit model keywords."""
    if config is not None:
        kw = {**CONFIGS[config], **kw}
        shape = kw.pop("shape")
    model = build_model(shape, **kw)
    x0 = model.initial_state() if state is None else state
    xn = model.initial_state()
    row_ptr, col, vals = model.jacobian(x0, xn)
    b = -model.residual(x0, xn).reshape(-1)
    srp, scol, svals = model.schur_approx(x0)
    nv = model.nv
    rng = np.random.Generator(np.random.PCG64(
        (kw.get("seed", 0) * 7919 + 13) if xtrue_seed is None else xtrue_seed))
    scale = np.array([_SCALE_P] + [_SCALE_S] * (nv - 2) + [_SCALE_T])
    x_true = (rng.standard_normal((model.g.n, nv)) * scale).reshape(-1)
    flat = vals.reshape(-1)
    b_star = bsr_matvec(row_ptr, col, flat, nv, x_true)
    return Problem(shape=tuple(shape), nv=nv,
                   row_ptr=row_ptr.astype(np.int32), col_idx=col.astype(np.int32),
                   vals=np.ascontiguousarray(flat),
                   st_row_ptr=srp.astype(np.int32), st_col_idx=scol.astype(np.int32),
                   st_vals=svals, b=b, b_star=b_star, x_true=x_true,
                   meta=dict(kw, nv=nv))

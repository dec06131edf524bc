"""Pins of the synthetic-input generator (physics, Jacobian, Schur approximation)."""
import json
import os

import numpy as np
import pytest

from paper_1907_04229_amd.synth import make_problem, build_model
from paper_1907_04229_amd.synth import props as P
from paper_1907_04229_amd.synth.model import DAY

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "property_spot_values.json")


def _dense(rp, col, vals, nv):
    n = rp.size - 1
    A = np.zeros((n * nv, n * nv))
    blocks = vals.reshape(-1, nv, nv)
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            A[i * nv:(i + 1) * nv, col[k] * nv:(col[k] + 1) * nv] = blocks[k]
    return A


def _perturbed(m, seed=0):
    x0 = m.initial_state()
    rng = np.random.default_rng(seed)
    x = x0.copy()
    x[:, 0] += rng.normal(0, 1e5, m.g.n)
    x[:, 1] += rng.uniform(0, 0.05, m.g.n)
    x[:, -1] += rng.uniform(0, 30, m.g.n)
    return x, x0


def test_property_spot_values():
    g = json.load(open(GOLDEN))
    for T, mu in g["mu_water_cP"]:
        assert P.mu_water(T) * 1e3 == pytest.approx(mu, abs=1e-4)
    for p, T, rho in g["rho_water_kg_m3"]:
        assert P.rho_water(p, T) == pytest.approx(rho, abs=1e-2)


@pytest.mark.parametrize("three_phase,shape", [(False, (4, 3, 3)), (True, (4, 3, 3)),
                                               (False, (1, 1, 9)), (False, (1, 4, 3)), (True, (5, 1, 3))])
def test_jacobian_matches_finite_differences(three_phase, shape):
    """Also on grids with nx = 1 or ny = 1, where stencil offsets of two axes
    coincide (-nx = -1, nx ny = nx)."""
    m = build_model(shape, three_phase=three_phase, kind="iid", seed=3, heater=True)
    x, x0 = _perturbed(m)
    rp, col, vals = m.jacobian(x, x0)
    n, nv = m.g.n, m.nv
    A = _dense(rp, col, vals.reshape(-1), nv)
    scale = np.array([1e3] + [1e-4] * (nv - 2) + [1e-2])
    J = np.zeros_like(A)
    for c in range(n * nv):
        h = scale[c % nv]
        xp = x.reshape(-1).copy()
        xp[c] += h
        xm = x.reshape(-1).copy()
        xm[c] -= h
        J[:, c] = (m.residual(xp.reshape(n, nv), x0).reshape(-1)
                   - m.residual(xm.reshape(n, nv), x0).reshape(-1)) / (2 * h)
    assert np.abs(J - A).max() <= 1e-7 * np.abs(A).max()


@pytest.mark.parametrize("three_phase", [False, True])
def test_schur_approx_equals_att_for_temperature_independent_fluids(three_phase):
    # With rho_a, mu_a independent of T, the derivative of the energy equation
    # w.r.t. T is exactly the operator of eq:Se (compare A_TT in Section 3).
    m = build_model((5, 4, 3), three_phase=three_phase, kind="iid", seed=4, heater=True,
                    frozen_props=True)
    x, x0 = _perturbed(m, 1)
    rp, col, vals = m.jacobian(x, x0)
    srp, scol, sv = m.schur_approx(x)
    assert (srp == rp).all() and (scol == col).all()
    att = vals[:, -1, -1]
    assert np.abs(att - sv).max() <= 1e-13 * np.abs(sv).max()
    # ... and it differs once the viscosities depend on temperature
    m2 = build_model((5, 4, 3), three_phase=three_phase, kind="iid", seed=4, heater=True)
    _, _, vals2 = m2.jacobian(x, x0)
    _, _, sv2 = m2.schur_approx(x)
    assert np.abs(vals2[:, -1, -1] - sv2).max() > 1e-3 * np.abs(sv2).max()


def test_flux_conservation_column_sums_vanish():
    # Closed (homogeneous Neumann) boundary, no sources, accumulation switched
    # off by an infinite time step: every facet flux leaves one cell and enters
    # the other, so each column of the Jacobian sums to zero per equation.
    m = build_model((4, 4, 3), kind="iid", seed=5, wells=False)
    m.dt = 1e30 * DAY
    x, x0 = _perturbed(m, 2)
    rp, col, vals = m.jacobian(x, x0)
    A = _dense(rp, col, vals.reshape(-1), m.nv)
    nv = m.nv
    for r in range(nv):
        colsum = A[r::nv, :].sum(axis=0)
        assert np.abs(colsum).max() <= 1e-12 * np.abs(A).max()


def test_problem_shapes_and_pattern():
    pr = make_problem(config="small")
    assert pr.n == 500 and pr.nv == 3
    assert pr.nnzb == 3100                      # 7 n - 2 (nx ny + nx nz + ny nz)
    rp, ci = pr.row_ptr, pr.col_idx
    for i in range(pr.n):
        row = ci[rp[i]:rp[i + 1]]
        assert (np.diff(row) > 0).all() and i in row
    A = _dense(rp, ci, pr.vals, pr.nv)
    assert np.allclose(A @ pr.x_true, pr.b_star, rtol=1e-12, atol=1e-12 * np.abs(pr.b_star).max())
    # pressure row is T_ref * sum_a c_va F_a and row 1 is c_ref T_ref F_w (eq:weighted, eq:scaling)
    assert np.isfinite(pr.b).all() and np.abs(pr.b).max() > 0


def test_seeded_inputs_are_reproducible():
    a = make_problem(config="small")
    b = make_problem(config="small")
    assert np.array_equal(a.vals, b.vals) and np.array_equal(a.b, b.b)
    assert np.array_equal(a.st_vals, b.st_vals)

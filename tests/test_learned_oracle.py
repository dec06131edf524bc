"""Pins of the FP64 learned-stage oracle: central-difference gradient check,
block-Jacobi reduction at W_out = 0, positive homogeneity."""
import numpy as np
import pytest

from oracle import learned as L
from paper_1907_04229_amd.learned_init import init_params, n_params
from paper_1907_04229_amd.synth import make_problem


@pytest.fixture(scope="module", params=[3, 4])
def setup(request):
    three = request.param == 4
    pr = make_problem(shape=(4, 3, 2), kind="iid", seed=31, three_phase=three)
    # a change of units keeps the blocks well scaled for finite differences
    nv = pr.nv
    cs = np.array([1e4] + [1e-2] * (nv - 2) + [1.0])
    vals = (pr.vals.reshape(-1, nv, nv) * cs[None, None, :]).reshape(-1)
    nbr = L.neighbors(pr.row_ptr, pr.col_idx, pr.n)
    dinv, E = L.edge_features(pr.row_ptr, pr.col_idx, vals, nv, nbr)
    A = L.bsr_dense(pr.row_ptr, pr.col_idx, vals, nv)
    return pr, nv, vals, nbr, dinv, E, A


def test_neighbour_directions():
    pr = make_problem(shape=(4, 3, 2), kind="iid", seed=1)
    nbr = L.neighbors(pr.row_ptr, pr.col_idx, pr.n)
    i = 1 + 4 * (1 + 3 * 0)           # cell (1, 1, 0)
    assert list(nbr[i]) == [i - 1, i + 1, i - 4, i + 4, -1, i + 12]


def test_n_params_layout():
    for nv in (3, 4):
        assert n_params(nv) == L.n_params(nv)
        th = init_params(nv, seed=1)
        p = L.unflatten(th.astype(np.float64), nv)
        assert (p["W_out"] == 0).all() and (p["b0"] == 0).all()


def test_zero_output_layer_is_block_jacobi(setup):
    pr, nv, vals, nbr, dinv, E, A = setup
    th = init_params(nv, seed=2)
    b1 = np.random.default_rng(0).standard_normal(pr.n * nv)
    z, _ = L.forward(th, b1, dinv, E, nbr, nv)
    want = np.einsum("irc,ic->ir", dinv, b1.reshape(-1, nv)).reshape(-1)
    assert np.allclose(z, want, rtol=1e-13, atol=0)


def test_positive_homogeneity(setup):
    pr, nv, vals, nbr, dinv, E, A = setup
    th = init_params(nv, seed=3, out_scale=0.3)
    b1 = np.random.default_rng(1).standard_normal(pr.n * nv)
    z1, _ = L.forward(th, b1, dinv, E, nbr, nv)
    z2, _ = L.forward(th, 7.5 * b1, dinv, E, nbr, nv)
    assert np.allclose(z2, 7.5 * z1, rtol=1e-12, atol=1e-14 * np.abs(z2).max())


def test_gradient_central_differences(setup):
    pr, nv, vals, nbr, dinv, E, A = setup
    th = init_params(nv, seed=4, out_scale=0.2).astype(np.float64)
    th[th.size // 3] += 0.1                      # make some biases nonzero
    b1 = np.random.default_rng(2).standard_normal(pr.n * nv)
    f, g = L.loss_and_grad(th, b1, A, dinv, E, nbr, nv)
    rng = np.random.default_rng(3)
    idx = rng.choice(th.size, 60, replace=False)
    idx = np.concatenate([idx, [0, th.size - 1]])
    for k in idx:
        h = 1e-6 * max(1.0, abs(th[k]))
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (L.loss_and_grad(tp, b1, A, dinv, E, nbr, nv)[0]
              - L.loss_and_grad(tm, b1, A, dinv, E, nbr, nv)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g).max()), (k, fd, g[k])


def test_neumann_initialisation_is_the_series():
    """neumann_params makes the network compute sum_k (-D^{-1} O)^k D^{-1} b1
    (K = 3 for nv = 3, K = 2 for nv = 4), checked against the series formed
    from the dense matrix."""
    from paper_1907_04229_amd.learned_init import neumann_params, neumann_order
    for kw in [dict(shape=(6, 5, 4), seed=3), dict(shape=(5, 4, 3), seed=4, three_phase=True)]:
        pr = make_problem(kind="gaussian", sigma=1.5, corr_len=3.0, **kw)
        n, nv = pr.n, pr.nv
        nbr = L.neighbors(pr.row_ptr, pr.col_idx, n)
        dinv, E = L.edge_features(pr.row_ptr, pr.col_idx, pr.vals, nv, nbr)
        A = L.bsr_dense(pr.row_ptr, pr.col_idx, pr.vals, nv)
        Dinv = np.zeros_like(A)
        for i in range(n):
            Dinv[i * nv:(i + 1) * nv, i * nv:(i + 1) * nv] = dinv[i]
        J = Dinv @ A - np.eye(n * nv)
        b1 = np.random.default_rng(1).standard_normal(n * nv)
        t = Dinv @ b1
        want = t.copy()
        for _ in range(neumann_order(nv)):
            t = -J @ t
            want += t
        z, _ = L.forward(neumann_params(nv, seed=2).astype(np.float64), b1, dinv, E, nbr, nv)
        assert np.linalg.norm(z - want) <= 1e-11 * np.linalg.norm(want)

"""Seeded initial parameters of the learned second stage (flat FP32 vector).

Layout: W_in (64 x nv); for each of the 3 layers W_e (64 x nv^2), W_s (64 x 64),
W_m (64 x 64), b (64); W_out (nv x 64); all row-major.  W_out starts at zero,
so the untrained stage is block Jacobi."""
import numpy as np

HIDDEN, LAYERS = 64, 3


def n_params(nv):
    return HIDDEN * nv + LAYERS * (HIDDEN * nv * nv + 2 * HIDDEN * HIDDEN + HIDDEN) + nv * HIDDEN


def init_params(nv, seed=0, out_scale=0.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [rng.standard_normal(HIDDEN * nv) / np.sqrt(nv)]
    for _ in range(LAYERS):
        parts.append(rng.standard_normal(HIDDEN * nv * nv) / nv)
        parts.append(rng.standard_normal(HIDDEN * HIDDEN) * (0.5 / np.sqrt(HIDDEN)))
        parts.append(rng.standard_normal(HIDDEN * HIDDEN) * (0.5 / np.sqrt(HIDDEN)))
        parts.append(np.zeros(HIDDEN))
    parts.append(rng.standard_normal(nv * HIDDEN) * out_scale)
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == n_params(nv)
    return theta

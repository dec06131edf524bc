"""Seeded initial parameters of the learned second stage (flat FP32 vector).

Layout: W_in (64 x nv); for each of the 3 layers W_e (64 x nv^2), W_s (64 x 64),
W_m (64 x 64), b (64); W_out (nv x 64); all row-major.

Two initialisations:

* ``init_params``: random hidden layers and W_out = 0, so the untrained stage
  is block Jacobi, z2 = D^{-1} b1.
* ``neumann_params``: weights that make the network compute the truncated
  Neumann series of block Jacobi, z2 = sum_{k=0..K} (-D^{-1} O)^k D^{-1} b1
  (O the off-diagonal blocks of A), with K = 3 for nv = 3 and K = 2 for
  nv = 4 (the channel budget of 64).  In the scaled unknowns u = S^{-1} D^{-1} b1
  the series is sum_k (-e)^k u with e the scaled edge blocks.  One message
  product g * h_nbr forms e[r][c] t_c(nbr) in a channel that holds t_c, so a
  term t is kept in nv^2 channels (one copy of t_c per row r); the ReLU of the
  residual update carries a signed term as a pair of channels (relu(t),
  relu(-t)).  Channel map:
      U  (nv^2):    h0 = u_c copies (W_in), never updated afterwards
      T1 (2 nv^2):  layer 1 writes relu(+-t1_c) copies, t1 = -e u
      T2 (2 nv^2):  layer 2 writes relu(+-t2_c) copies, t2 = -e t1   (K = 3)
      TK (2 nv):    the last layer writes relu(+-tK_c) once
  Remaining channels get small random weights and a zero read-out, so
  training can put them to use.
"""
import numpy as np

HIDDEN, LAYERS = 64, 3


def n_params(nv):
    return HIDDEN * nv + LAYERS * (HIDDEN * nv * nv + 2 * HIDDEN * HIDDEN + HIDDEN) + nv * HIDDEN


def _split(theta, nv):
    p, o = {}, 0
    shapes = [("W_in", (HIDDEN, nv))]
    for l in range(LAYERS):
        shapes += [(f"W_e{l}", (HIDDEN, nv * nv)), (f"W_s{l}", (HIDDEN, HIDDEN)),
                   (f"W_m{l}", (HIDDEN, HIDDEN)), (f"b{l}", (HIDDEN,))]
    shapes.append(("W_out", (nv, HIDDEN)))
    for name, shape in shapes:
        size = int(np.prod(shape))
        p[name] = theta[o:o + size].reshape(shape)   # views into theta
        o += size
    return p


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


def neumann_order(nv):
    return 3 if nv <= 3 else 2


def neumann_params(nv, seed=0, free_scale=1e-2):
    """Parameters whose forward pass is the order-K Neumann series (see above)."""
    K = neumann_order(nv)
    Q = nv * nv
    theta = np.zeros(n_params(nv), np.float64)
    p = _split(theta, nv)
    U = np.arange(Q).reshape(nv, nv)                      # U[r, c]
    nxt = Q
    terms = []                                            # channel maps of T1 .. T(K-1)
    for _ in range(K - 1):
        terms.append(np.arange(nxt, nxt + 2 * Q).reshape(2, nv, nv))   # [sign, r, c]
        nxt += 2 * Q
    last = np.arange(nxt, nxt + 2 * nv).reshape(2, nv)    # [sign, c]
    nxt += 2 * nv
    assert nxt <= HIDDEN
    for r in range(nv):
        for c in range(nv):
            p["W_in"][U[r, c], c] = 1.0
    src = [(U, None)] + [(t, True) for t in terms]        # layer l reads src[l]
    for l in range(K):
        chan, signed = src[l]
        We, Wm = p[f"W_e{l}"], p[f"W_m{l}"]
        # message channels: e[r][c] * t_c(nbr) in the channel holding t_c for row r
        if signed:
            for sg in range(2):
                for r in range(nv):
                    for c in range(nv):
                        We[chan[sg, r, c], r * nv + c] = 1.0
        else:
            for r in range(nv):
                for c in range(nv):
                    We[chan[r, c], r * nv + c] = 1.0

        # (e t)_c = sum_c' m[row c, col c'] (minus the negative copy when signed)
        def et_weights(c):
            w = {}
            if signed:
                for c2 in range(nv):
                    w[chan[0, c, c2]] = 1.0
                    w[chan[1, c, c2]] = -1.0
            else:
                for c2 in range(nv):
                    w[chan[c, c2]] = 1.0
            return w

        dst = terms[l] if l < K - 1 else None
        for c in range(nv):
            for k, wt in et_weights(c).items():
                # new term t' = -(e t): + copy gets -wt, - copy gets +wt
                if dst is not None:
                    for r2 in range(nv):
                        Wm[dst[0, r2, c], k] = -wt
                        Wm[dst[1, r2, c], k] = wt
                else:
                    Wm[last[0, c], k] = -wt
                    Wm[last[1, c], k] = wt
    # read-out: sum of the terms, one copy each
    for c in range(nv):
        for t in terms:
            p["W_out"][c, t[0, 0, c]] = 1.0
            p["W_out"][c, t[1, 0, c]] = -1.0
        p["W_out"][c, last[0, c]] = 1.0
        p["W_out"][c, last[1, c]] = -1.0
    # free channels: small random weights, zero read-out
    rng = np.random.Generator(np.random.PCG64(seed))
    free = np.arange(nxt, HIDDEN)
    if free.size and free_scale > 0:
        p["W_in"][free] = rng.standard_normal((free.size, nv)) * free_scale
        for l in range(LAYERS):
            p[f"W_e{l}"][free] = rng.standard_normal((free.size, Q)) * free_scale
            p[f"W_s{l}"][free[:, None], free[None, :]] = (
                rng.standard_normal((free.size, free.size)) * free_scale)
            p[f"W_m{l}"][free[:, None], free[None, :]] = (
                rng.standard_normal((free.size, free.size)) * free_scale)
    return theta.astype(np.float32)

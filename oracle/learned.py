"""FP64 oracle of the learned second stage: forward pass, loss and a
hand-derived backward pass, in plain numpy.

TEST INFRASTRUCTURE ONLY (same status as the rest of oracle/): it is the
reference the GPU kernels are checked against.  Nothing in the product imports
it.

The learned second stage is not in the paper; it replaces the ILU(0) second
stage of the two-stage preconditioner (Section 3, "Two-stage
preconditioners": x = M2^{-1} b1 + x1) by a small message-passing network on
the 7-point cell graph.  Definition (both sides implement exactly this):

  inputs      r_i = D_i^{-1} b1_i  (D_i the diagonal nv x nv block of A)
              s_k = sqrt(mean over cells of r_ik^2), one scale per unknown k (the
                    unknowns have different units); u_ik = r_ik / s_k (0 if s_k = 0)
              e_{i,d} = S^{-1} D_i^{-1} A_{i, nbr(i,d)} S (flattened row-major),
              S = diag(s), i.e. the block in the scaled unknowns; zero when
              cell i has no neighbour in direction d; d = 0..5 orders the
              neighbours as (-axis0, +axis0, -axis1, +axis1, -axis2, +axis2),
              axes ordered by increasing |column - row| offset
  h0_i        = W_in u_i
  layer l=1..3
    g_{i,d}   = W_e^l e_{i,d}
    m_i       = sum_d g_{i,d} * h^{l-1}_{nbr(i,d)}          (elementwise)
    a_i       = W_s^l h^{l-1}_i + W_m^l m_i + b^l
    h^l_i     = h^{l-1}_i + relu(a_i)
  output      z2_ik = s_k (u_ik + (W_out h3_i)_k)
With W_out = 0 the stage is block Jacobi: z2 = D^{-1} b1.
Loss of one pair (A, b1): ||b1 - A z2||^2 / ||b1||^2.
"""
import numpy as np

HIDDEN = 64
LAYERS = 3
NDIR = 6


def neighbors(row_ptr, col, n):
    """nbr[i, d] (or -1) from a 7-point cell-graph pattern."""
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    off = col.astype(np.int64) - rows
    mags = np.unique(np.abs(off[off != 0]))
    if mags.size > 3:
        raise ValueError("not a 7-point pattern")
    nbr = -np.ones((n, NDIR), np.int64)
    for k in np.where(off != 0)[0]:
        axis = int(np.searchsorted(mags, abs(off[k])))
        d = 2 * axis + (1 if off[k] > 0 else 0)
        nbr[rows[k], d] = col[k]
    return nbr


def edge_features(row_ptr, col, vals, nv, nbr):
    n = row_ptr.size - 1
    blocks = vals.reshape(-1, nv, nv)
    dinv = np.empty((n, nv, nv))
    E = np.zeros((n, NDIR, nv * nv))
    pos = {}
    for i in range(n):
        for k in range(row_ptr[i], row_ptr[i + 1]):
            pos[(i, col[k])] = k
        dinv[i] = np.linalg.inv(blocks[pos[(i, i)]])
    for i in range(n):
        for d in range(NDIR):
            j = nbr[i, d]
            if j >= 0:
                E[i, d] = (dinv[i] @ blocks[pos[(i, j)]]).reshape(-1)
    return dinv, E


def bsr_dense(row_ptr, col, vals, nv):
    n = row_ptr.size - 1
    A = np.zeros((n * nv, n * nv))
    bl = vals.reshape(-1, nv, nv)
    for i in range(n):
        for k in range(row_ptr[i], row_ptr[i + 1]):
            A[i * nv:(i + 1) * nv, col[k] * nv:(col[k] + 1) * nv] = bl[k]
    return A


def unflatten(theta, nv):
    """Parameter dict from the flat vector (layout shared with the GPU code)."""
    p, o = {}, 0

    def take(name, shape):
        nonlocal o
        size = int(np.prod(shape))
        p[name] = theta[o:o + size].reshape(shape)
        o += size

    take("W_in", (HIDDEN, nv))
    for l in range(LAYERS):
        take(f"W_e{l}", (HIDDEN, nv * nv))
        take(f"W_s{l}", (HIDDEN, HIDDEN))
        take(f"W_m{l}", (HIDDEN, HIDDEN))
        take(f"b{l}", (HIDDEN,))
    take("W_out", (nv, HIDDEN))
    assert o == theta.size
    return p


def n_params(nv):
    return HIDDEN * nv + LAYERS * (HIDDEN * nv * nv + 2 * HIDDEN * HIDDEN + HIDDEN) + nv * HIDDEN


def forward(theta, b1, dinv, E, nbr, nv, s=None):
    """z2 and the intermediate values of the backward pass.  `s` (optional)
    gives the per-unknown scales instead of the RMS over these cells, so that
    a neighbourhood cut out of a larger system uses that system's scales."""
    p = unflatten(np.asarray(theta, np.float64), nv)
    n = dinv.shape[0]
    r = np.einsum("irc,ic->ir", dinv, b1.reshape(n, nv))
    if s is None:
        s = np.sqrt(np.mean(r * r, axis=0))
    inv = np.where(s > 0.0, 1.0 / np.where(s > 0.0, s, 1.0), 0.0)
    cache = dict(s=s, r=r)
    u = r * inv
    # edge blocks in the scaled unknowns: e[r][c] * s_c / s_r
    fac = (inv[:, None] * s[None, :]).reshape(-1)
    Es = E * fac[None, None, :]
    h = u @ p["W_in"].T
    hs, ms, as_, gs = [h], [], [], []
    mask = (nbr >= 0)
    for l in range(LAYERS):
        g = Es @ p[f"W_e{l}"].T                      # (n, 6, 64)
        hn = np.where(mask[:, :, None], h[np.maximum(nbr, 0)], 0.0)
        m = np.sum(g * hn, axis=1)
        a = h @ p[f"W_s{l}"].T + m @ p[f"W_m{l}"].T + p[f"b{l}"]
        h = h + np.maximum(a, 0.0)
        hs.append(h)
        ms.append(m)
        as_.append(a)
        gs.append(g)
    out = h @ p["W_out"].T
    z2 = s * (u + out)   # s broadcasts over the unknowns
    cache.update(u=u, hs=hs, ms=ms, as_=as_, gs=gs, Es=Es)
    return z2.reshape(-1), cache


def loss_and_grad(theta, b1, A_dense, dinv, E, nbr, nv):
    """Loss ||b1 - A z2||^2 / ||b1||^2 of one pair and its gradient (flat)."""
    theta = np.asarray(theta, np.float64)
    p = unflatten(theta, nv)
    n = dinv.shape[0]
    z2, c = forward(theta, b1, dinv, E, nbr, nv)
    bb = float(b1 @ b1)
    res = b1 - A_dense @ z2
    L = float(res @ res) / bb
    grads = {k: np.zeros_like(v) for k, v in p.items()}
    dz = (-2.0 / bb) * (A_dense.T @ res)             # dL/dz2
    dout = c["s"][None, :] * dz.reshape(n, nv)
    h3 = c["hs"][-1]
    grads["W_out"] = dout.T @ h3
    dh = dout @ p["W_out"]
    mask = (nbr >= 0)
    for l in reversed(range(LAYERS)):
        hprev = c["hs"][l]
        a, m, g = c["as_"][l], c["ms"][l], c["gs"][l]
        da = dh * (a > 0.0)
        grads[f"W_s{l}"] = da.T @ hprev
        grads[f"W_m{l}"] = da.T @ m
        grads[f"b{l}"] = da.sum(axis=0)
        dm = da @ p[f"W_m{l}"]
        hn = np.where(mask[:, :, None], hprev[np.maximum(nbr, 0)], 0.0)
        dg = dm[:, None, :] * hn                     # (n, 6, 64)
        grads[f"W_e{l}"] = np.einsum("idk,idq->kq", dg, c["Es"])
        dh_new = dh + da @ p[f"W_s{l}"]
        contrib = dm[:, None, :] * g                 # d loss / d h_nbr(i,d)
        for d in range(NDIR):
            ok = mask[:, d]
            np.add.at(dh_new, nbr[ok, d], contrib[ok, d])
        dh = dh_new
    grads["W_in"] = dh.T @ c["u"]
    return L, _flatten(grads, nv)


def _flatten(g, nv):
    parts = [g["W_in"].reshape(-1)]
    for l in range(LAYERS):
        parts += [g[f"W_e{l}"].reshape(-1), g[f"W_s{l}"].reshape(-1), g[f"W_m{l}"].reshape(-1),
                  g[f"b{l}"].reshape(-1)]
    parts.append(g["W_out"].reshape(-1))
    return np.concatenate(parts)

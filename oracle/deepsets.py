"""FP64 reference of the learned warm-start network (test infrastructure).

The network is not part of the paper: it proposes a cluster's initial
centroid (support points and weights) from the cluster's members, to
warm-start the B-ADMM centroid update.  This module is the plain numpy
statement of its forward pass, loss and gradient, used to check the GPU
kernels; its own gradient is pinned by central finite differences.

Architecture (hidden width H, support size m, dimension d):
  per point (member k, support j) of cluster c:
      f = [ (y_j - mu_c) / s_c ,  m_k w_j ]          (d + 1, zero padded to DIN)
      h1 = relu(f W1 + b1);  h2 = relu(h1 W2 + b2)    (H)
  pool  g_c = sum_points (w_j / N_c) h2               (weighted mean)
  head  u1 = relu(g V1 + e1); u2 = relu(u1 V2 + e2); o = u2 V3 + e3
  output Delta_i = o[i d : i d + d], logits_i = o[m d + i]
         x_i = mu_c + s_c Delta_i,  w = softmax(logits)
mu_c, s_c: weighted mean and RMS radius of the cluster's points.
Loss per cluster, in standardised coordinates t_j = (x*_j - mu_c)/s_c:
  Chamfer  sum_j w*_j |Delta_nn(j) - t_j|^2 + sum_i w_i |Delta_i - t_nn(i)|^2
  plus the cross-entropy -sum_i q_i log w_i, q_i = target mass whose
  nearest predicted point is i.  The batch loss is the mean over clusters.
Parameters are one flat vector in the order W1, b1, W2, b2, V1, e1, V2, e2,
V3, e3 (row-major, input index first).
"""
from __future__ import annotations

import numpy as np

from synth.generators import deepsets_init_params


def dims(m, d, H):
    din = (d + 1 + 15) // 16 * 16
    out = m * (d + 1)
    outp = (out + 31) // 32 * 32
    return din, out, outp


def param_shapes(m, d, H):
    din, _, outp = dims(m, d, H)
    return [("W1", (din, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
            ("V1", (H, H)), ("e1", (H,)), ("V2", (H, H)), ("e2", (H,)),
            ("V3", (H, outp)), ("e3", (outp,))]


def param_count(m, d, H):
    return sum(int(np.prod(s)) for _, s in param_shapes(m, d, H))


def unpack(theta, m, d, H):
    out, o = {}, 0
    for name, shp in param_shapes(m, d, H):
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def pack(parts, m, d, H):
    return np.concatenate([parts[n].reshape(-1)
                           for n, _ in param_shapes(m, d, H)])


def init_params(m, d, H, seed):
    """Seeded initial parameters (drawn by the shared input generator)."""
    return deepsets_init_params(m, d, H, seed)


def round_bf16(a):
    """Round to the nearest bfloat16 value (ties to even), as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16) << np.uint64(16)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def cluster_points(wl, members):
    """Points, their weights w_j, the m_k w_j feature and the pooling
    weights w_j / N_c of one cluster."""
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    ys, ws, mw = [], [], []
    for k in members:
        a, b = off[k], off[k + 1]
        ys.append(X[a:b])
        ws.append(W[a:b])
        mw.append((b - a) * W[a:b])
    y = np.concatenate(ys)
    w = np.concatenate(ws)
    return y, w, np.concatenate(mw), w / len(members)


def forward_backward(theta, clusters, m, d, H, bf16=False):
    """Loss and gradient for a batch.

    clusters: list of dicts with y (P x d), w (P), mw (P), pw (P),
    xt (m x d targets), wt (m target weights).  bf16=True rounds the
    parameters and the stored activations to bfloat16 where the GPU path
    stores them (inputs to each matrix product), for like-for-like checks.
    Returns (mean loss, gradient vector)."""
    din, out, outp = dims(m, d, H)
    rb = round_bf16 if bf16 else (lambda a: a)
    P = unpack(theta, m, d, H)
    Pq = {k: rb(v) if k[0] in "WV" else v for k, v in P.items()}
    grads = {k: np.zeros_like(v) for k, v in P.items()}
    total = 0.0
    B = len(clusters)
    for cl in clusters:
        y, pw, mw = cl["y"], cl["pw"], cl["mw"]
        w = cl["w"]
        mu = (w @ y) / w.sum()
        s = np.sqrt((w * ((y - mu) ** 2).sum(1)).sum() / w.sum())
        s = max(s, 1e-12)
        f = np.zeros((len(y), din))
        f[:, :d] = (y - mu) / s
        f[:, d] = mw
        f = rb(f)
        z1 = f @ Pq["W1"] + P["b1"]
        h1 = rb(np.maximum(z1, 0))
        z2 = h1 @ Pq["W2"] + P["b2"]
        h2 = rb(np.maximum(z2, 0))
        g = pw @ h2
        gq = rb(g)
        a1 = gq @ Pq["V1"] + P["e1"]
        u1 = rb(np.maximum(a1, 0))
        a2 = u1 @ Pq["V2"] + P["e2"]
        u2 = rb(np.maximum(a2, 0))
        o = u2 @ Pq["V3"] + P["e3"]
        delta = o[:m * d].reshape(m, d)
        logit = o[m * d:m * d + m]
        ex = np.exp(logit - logit.max())
        wh = ex / ex.sum()
        t = (cl["xt"] - mu) / s
        D = ((delta[:, None, :] - t[None, :, :]) ** 2).sum(2)   # m x m*
        nn_t = D.argmin(0)                                       # per target
        nn_p = D.argmin(1)                                       # per pred
        wt = cl["wt"]
        a = D[np.arange(m), nn_p]
        lx = float(wt @ D[nn_t, np.arange(len(wt))]) + float(wh @ a)
        q = np.zeros(m)
        np.add.at(q, nn_t, wt)
        lw = -float(q @ np.log(np.maximum(wh, 1e-300)))
        total += lx + lw
        # gradient of this cluster's loss
        dd = np.zeros((m, d))
        for j in range(len(wt)):
            dd[nn_t[j]] += 2.0 * wt[j] * (delta[nn_t[j]] - t[j])
        dd += 2.0 * wh[:, None] * (delta - t[nn_p])
        dlogit = wh * q.sum() - q + wh * (a - wh @ a)
        do = np.zeros(outp)
        do[:m * d] = dd.reshape(-1)
        do[m * d:m * d + m] = dlogit
        do /= B
        doq = rb(do)
        grads["V3"] += np.outer(u2, doq)
        grads["e3"] += do
        du2 = Pq["V3"] @ doq
        da2 = rb(du2 * (a2 > 0))
        grads["V2"] += np.outer(u1, da2)
        grads["e2"] += da2
        du1 = Pq["V2"] @ da2
        da1 = rb(du1 * (a1 > 0))
        grads["V1"] += np.outer(gq, da1)
        grads["e1"] += da1
        dg = Pq["V1"] @ da1
        dz2 = rb(np.outer(pw, dg) * (z2 > 0))
        grads["W2"] += h1.T @ dz2
        grads["b2"] += dz2.sum(0)
        dh1 = dz2 @ Pq["W2"].T
        dz1 = rb(dh1 * (z1 > 0))
        grads["W1"] += f.T @ dz1
        grads["b1"] += dz1.sum(0)
    return total / B, pack(grads, m, d, H)


def propose(theta, cl, m, d, H, bf16=False):
    """Proposed (x, w) for one cluster.  bf16=True rounds parameters and
    stored activations where the GPU path stores them as BF16."""
    din, out, outp = dims(m, d, H)
    rb = round_bf16 if bf16 else (lambda a: a)
    P = unpack(theta, m, d, H)
    Pq = {k: rb(v) if k[0] in "WV" else v for k, v in P.items()}
    y, w, pw, mw = cl["y"], cl["w"], cl["pw"], cl["mw"]
    mu = (w @ y) / w.sum()
    s = max(np.sqrt((w * ((y - mu) ** 2).sum(1)).sum() / w.sum()), 1e-12)
    f = np.zeros((len(y), din))
    f[:, :d] = (y - mu) / s
    f[:, d] = mw
    f = rb(f)
    h1 = rb(np.maximum(f @ Pq["W1"] + P["b1"], 0))
    h2 = rb(np.maximum(h1 @ Pq["W2"] + P["b2"], 0))
    g = rb(pw @ h2)
    u1 = rb(np.maximum(g @ Pq["V1"] + P["e1"], 0))
    u2 = rb(np.maximum(u1 @ Pq["V2"] + P["e2"], 0))
    o = u2 @ Pq["V3"] + P["e3"]
    x = mu + s * o[:m * d].reshape(m, d)
    lg = o[m * d:m * d + m]
    ex = np.exp(lg - lg.max())
    return x, ex / ex.sum()


def product_bound(cl, x, w):
    """sum over members k, support i, points j of w_i w_j^(k) |x_i - y_j|^2
    (the cost of the product coupling, an upper bound on the barycenter
    objective at (x, w)), by brute force."""
    y, wy = cl["y"], cl["w"]
    C = ((x[:, None, :] - y[None, :, :]) ** 2).sum(2)
    return float(w @ C @ wy)

"""Shared test helpers: run the oracle cluster-by-cluster, compare plans."""
import numpy as np

import oracle


def oracle_barycenters(wl, labels, Xc, Wc, plans=None, warm=None,
                       residuals=None, **kw):
    """Oracle B-ADMM for every non-empty cluster of `labels`.

    Returns (Xc', Wc', traces[K] (T each, None when empty), rhos, plans);
    if `residuals` is a list it receives the residual traces (per cluster,
    None when empty)."""
    K, m, d = Xc.shape
    n = int(wl["offsets"][-1])
    if plans is None:
        plans = oracle.Plans(m, n)
    Xo, Wo = Xc.copy(), Wc.copy()
    traces, rhos = [None] * K, np.zeros(K)
    if residuals is not None:
        residuals.extend([None] * K)
    for c in range(K):
        mem = np.nonzero(labels == c)[0]
        if len(mem) == 0:
            continue
        wm = None if warm is None else warm[mem].astype(np.uint8)
        out = oracle.barycenter(wl, mem, Xc[c], Wc[c], plans=plans, warm=wm,
                                **kw)
        Xo[c], Wo[c] = out["x"], out["w"]
        traces[c], rhos[c] = out["ftrace"], out["rho"]
        if residuals is not None:
            residuals[c] = out["rtrace"]
    return Xo, Wo, traces, rhos, plans


def sub_workload(wl, idx):
    """The instances `idx` of a workload as a workload of their own (same
    points and weights, renumbered 0..len(idx)-1 in the order given)."""
    off = wl["offsets"]
    idx = np.asarray(idx, dtype=np.int64)
    sizes = off[idx + 1] - off[idx]
    o = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    rows = np.concatenate([np.arange(off[k], off[k + 1]) for k in idx])
    return {"offsets": o, "X": np.ascontiguousarray(wl["X"][rows]),
            "W": np.ascontiguousarray(wl["W"][rows])}


def marginal_errors(ctx, wl, plans_o, ks):
    """Max abs difference of row/column sums of Pi1 and Pi2, GPU vs oracle,
    over instances ks."""
    off = wl["offsets"]
    err = 0.0
    for k in ks:
        g1, g2, _ = ctx.plans_get(int(k))
        o1, o2, _ = plans_o.block(off, int(k))
        for g, o in ((g1, o1), (g2, o2)):
            err = max(err, np.abs(g.sum(0) - o.sum(0)).max(),
                      np.abs(g.sum(1) - o.sum(1)).max())
    return err


def plan_errors(ctx, wl, plans_o, ks, rho_of, local=None):
    """Element-by-element comparison of the plans of instances ks, GPU vs
    oracle: (max |Pi1 - Pi1_o|, max |Pi2 - Pi2_o|, max |Lambda -
    Lambda_o| / rho, max marginal difference).  rho_of(k) gives the rho of
    instance k's cluster (Lambda carries rho's scale, Eq. (badmm2)).
    local maps a GPU instance index to the oracle's (for oracle runs on a
    sub-workload; default: the same index)."""
    off_o = wl["offsets"]
    e1 = e2 = el = em = 0.0
    for k in ks:
        g1, g2, gl = ctx.plans_get(int(k))
        ko = int(k) if local is None else int(local[int(k)])
        o1, o2, ol = plans_o.block(off_o, ko)
        assert g1.shape == o1.shape
        e1 = max(e1, float(np.abs(g1 - o1).max()))
        e2 = max(e2, float(np.abs(g2 - o2).max()))
        el = max(el, float(np.abs(gl - ol).max()) / rho_of(int(k)))
        for g, o in ((g1, o1), (g2, o2)):
            em = max(em, float(np.abs(g.sum(0) - o.sum(0)).max()),
                     float(np.abs(g.sum(1) - o.sum(1)).max()))
    return e1, e2, el, em

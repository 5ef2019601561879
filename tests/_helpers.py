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

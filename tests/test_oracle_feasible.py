"""Pins of the oracle's rounded-plan objective and product-coupling bound.

round_feasible is pinned by exact marginals, by leaving couplings unchanged
and by LP optimality (its cost can never be below the transport LP's);
feasible_objective by converging onto the LP objective for a converged
B-ADMM run; product_bound by its closed form through the weighted mean."""
import numpy as np

import oracle
from oracle import deepsets as ds
from synth.generators import make_workload, warmstart_clusters


def test_round_feasible_marginals_and_identity():
    rng = np.random.Generator(np.random.PCG64(3))
    for m, mk in ((5, 7), (16, 4), (1, 9), (8, 1)):
        P = rng.random((m, mk)) * rng.random((m, 1))
        a = rng.random(m) + 0.1
        a /= a.sum()
        b = rng.random(mk) + 0.1
        b /= b.sum()
        R = oracle.round_feasible(P, a, b)
        assert np.all(R >= 0)
        np.testing.assert_allclose(R.sum(1), a, atol=1e-15)
        np.testing.assert_allclose(R.sum(0), b, atol=1e-15)
        # a coupling is returned unchanged
        np.testing.assert_allclose(oracle.round_feasible(R, a, b), R,
                                   atol=1e-16)
    # product coupling stays
    a = np.array([0.2, 0.8])
    b = np.array([0.5, 0.25, 0.25])
    np.testing.assert_array_equal(oracle.round_feasible(np.outer(a, b), a, b),
                                  np.outer(a, b))


def test_rounded_cost_bounds_lp_and_matches_lp_plan():
    wl = make_workload("gmm_d3_n256", N=6)
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    rng = np.random.Generator(np.random.PCG64(5))
    x = rng.random((4, 3))
    w = np.array([0.1, 0.2, 0.3, 0.4])
    for k in range(6):
        y, wy = X[off[k]:off[k + 1]], W[off[k]:off[k + 1]]
        lp, plan = oracle.exact_w2(x, w, y, wy)
        C = oracle.cost_block(x, y)
        R = oracle.round_feasible(plan, w, wy)
        assert abs((R * C).sum() - lp) < 1e-9 * max(1, lp)
        noisy = plan * rng.uniform(0.5, 1.5, size=plan.shape)
        Rn = oracle.round_feasible(noisy, w, wy)
        assert (Rn * C).sum() >= lp - 1e-12


def test_feasible_objective_converges_to_lp():
    wl = make_workload("gmm_d3_n256", N=12)
    members = np.arange(12)
    x0, w0 = oracle.init_centroids(wl, [0], 8)
    out = oracle.barycenter(wl, members, x0[0], w0[0], T=3000, tau=10)
    fo = oracle.feasible_objective(wl, members, out["x"], out["w"],
                                   out["plans"])
    ft = oracle.f_true(wl, members, out["x"], out["w"])
    assert fo >= ft - 1e-12
    assert fo <= ft * (1 + 2e-3)
    # early iterate: still an upper bound, and larger
    early = oracle.barycenter(wl, members, x0[0], w0[0], T=5, tau=10)
    fe = oracle.feasible_objective(wl, members, early["x"], early["w"],
                                   early["plans"])
    assert fe >= oracle.f_true(wl, members, early["x"], early["w"]) - 1e-12


def test_product_bound_closed_form():
    wl = warmstart_clusters("gmm3", 3, seed=11, nc_lo=8, nc_hi=20)
    rng = np.random.Generator(np.random.PCG64(2))
    for c in range(3):
        mem = np.nonzero(wl["labels"] == c)[0]
        y, w, mw, pw = ds.cluster_points(wl, mem)
        cl = dict(y=y, w=w)
        x = rng.random((5, 3))
        wx = rng.random(5)
        wx /= wx.sum()
        bf = ds.product_bound(cl, x, wx)
        Wt = w.sum()
        mu = w @ y / Wt
        S = (w * ((y - mu) ** 2).sum(1)).sum()
        xb = wx @ x
        closed = Wt * ((wx * ((x - xb) ** 2).sum(1)).sum()
                       + ((xb - mu) ** 2).sum()) + S
        assert abs(bf - closed) < 1e-10 * bf
        # the bound is the product plan's transport cost: above each W^2
        tot = 0.0
        off = wl["offsets"]
        for k in mem:
            tot += oracle.exact_w2(x, wx, wl["X"][off[k]:off[k + 1]],
                                   wl["W"][off[k]:off[k + 1]])[0]
        assert tot <= bf + 1e-12


def test_warmstart_cluster_generator():
    wl = warmstart_clusters("gmm3", 5, seed=1, nc_lo=64, nc_hi=128)
    off = wl["offsets"]
    sizes = np.diff(off)
    assert wl["labels"].shape[0] == len(sizes)
    assert np.all(sizes[wl["first"]] == 16)
    assert np.all((sizes >= 4) & (sizes <= 16))
    sums = np.add.reduceat(wl["W"], off[:-1])
    np.testing.assert_allclose(sums, 1.0, atol=1e-12)
    counts = np.bincount(wl["labels"])
    assert np.all((counts >= 64) & (counts <= 128))
    wt = warmstart_clusters("topic64", 2, seed=1, nc_lo=64, nc_hi=70)
    assert wt["X"].shape[1] == 64
    np.testing.assert_allclose(np.linalg.norm(wt["X"], axis=1), 1.0,
                               atol=1e-2)
    assert np.all(np.diff(wt["offsets"])[wt["first"]] == 64)

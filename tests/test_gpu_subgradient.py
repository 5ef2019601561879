"""Subgradient-descent centroid update on the GPU (Appendix A, Algorithm
"Centroid Update with Subgradient Descent": exact transport LPs by a
device network simplex, Eq. (dualvar), Eq. (stepsize)) against the FP64
reference in oracle/subgradient.py (transport LPs by HiGHS), through the C
ABI.  Inputs are generic (continuous weights), so every LP has a unique
optimal plan and row duals unique up to a shift, which the projection of
Eq. (dualvar) removes.  Bars: FP64 device arithmetic -- objective trace,
weights, support and plan entries within 1e-9; FP32 supports (the LP still
runs in FP64 on the FP32-rounded points) -- 1e-5 relative / absolute."""
import numpy as np
import pytest

import oracle
from oracle import subgradient as osg
from synth.generators import (make_workload, pick_init_members,
                              symbol_init_centroids)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def d2():
    from paper_1510_00012_amd import d2 as mod
    mod.load_library()
    return mod


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def _oracle(wl, lab, Xc, Wc, T, tau, alpha, zeta, fixed):
    off = wl["offsets"]
    K = len(Wc)
    res = [None] * K
    for c in range(K):
        mem = np.nonzero(lab == c)[0]
        if len(mem) == 0:
            continue
        ys = [wl["X"][off[k]:off[k + 1]] for k in mem]
        wys = [wl["W"][off[k]:off[k + 1]] for k in mem]
        res[c] = osg.subgradient_barycenter(
            lambda x: [oracle.cost_block(x, y) for y in ys], ys, wys,
            Xc[c], Wc[c], T=T, tau=tau, alpha=alpha, zeta=zeta,
            fixed_support=fixed)
        res[c]["members"] = mem
    return res


@pytest.mark.parametrize("dtype,name,N,K,m,fixed", [
    ("f64", "gmm_d3_n65536_k16", 500, 3, 8, False),
    ("f64", "gmm_d16_n2000000_k256", 300, 3, 16, True),
    ("f32", "gmm_d3_n65536_k16", 500, 3, 8, False)])
def test_subgradient_matches_reference(d2, dtype, name, N, K, m, fixed):
    print(f"[subgradient {name} {dtype} fixed={fixed}]", flush=True)
    wl = make_workload(name, N=N)
    mem = pick_init_members(wl["offsets"], K, m, 23)
    Xc, Wc = oracle.init_centroids(wl, mem, m)
    # merged weights are sums of the seed member's weights, so the seed's
    # transport problem is degenerate (its duals are not unique); mixing in
    # continuous noise makes every problem generic
    rng = np.random.Generator(np.random.PCG64(31))
    Wc = 0.8 * Wc + 0.2 * rng.dirichlet(np.ones(m), size=K)
    lab, _, _ = oracle.assign(wl, Xc, Wc, T=30)
    T, tau, alpha, zeta = 12, 5, 0.3, 1.0
    ref = _oracle(wl, lab, Xc, Wc, T, tau, alpha, zeta, fixed)
    tol = 1e-9 if dtype == "f64" else 1e-5
    with d2.D2Context(0, dtype) as ctx:
        ctx.load_instances(wl["offsets"], wl["X"], wl["W"])
        ctx.centroids_set(Xc, Wc)
        ctx.labels_set(lab)
        st = ctx.subgradient(iters=T, tau=tau, alpha=alpha, zeta=zeta,
                             fixed_support=fixed)
        assert st["lp_failed"] == 0
        g_tr, _ = ctx.objective(T)
        Xg, Wg = ctx.centroids_get()
        worst = wdev = xdev = pdev = 0.0
        for c in range(K):
            r = ref[c]
            if r is None:
                continue
            worst = max(worst, _rel(g_tr[:, c], r["ftrace"]))
            wdev = max(wdev, float(np.abs(Wg[c] - r["w"]).max()))
            xdev = max(xdev, float(np.abs(Xg[c] - r["x"]).max()))
            for q, k in enumerate(r["members"][::7]):
                _, P2, _ = ctx.plans_get(int(k))
                pdev = max(pdev, float(np.abs(P2 - r["plans"][7 * q]).max()))
        print(f"  pivots {st['pivots']} ({st['pivots'] / (T * N):.1f} per LP), "
              f"{st['ms']:.1f} ms; trace rel {worst:.3g}, weights {wdev:.3g},"
              f" support {xdev:.3g}, plans {pdev:.3g}", flush=True)
        assert worst < tol and wdev < tol and xdev < tol and pdev < tol
        if fixed:
            assert np.array_equal(Xg, Xc)


def test_subgradient_symbolic_and_from_badmm(d2):
    """Tripeptide histograms (symbolic, fixed support): the refinement from
    B-ADMM's weights matches the reference and does not raise the exact
    objective of its start by more than the step allows (the best value on
    the trace is at most the first)."""
    print("[subgradient symbolic]", flush=True)
    wl = make_workload("protein_g3_n10742_k10", N=300)
    K, m = 4, 12
    lab = (wl["classes"] % K).astype(np.int32)
    csym, _ = symbol_init_centroids(wl, lab, K, m)
    rng = np.random.Generator(np.random.PCG64(2))
    Wc = rng.dirichlet(np.ones(m), size=K)
    T = 10
    with d2.D2Context(0, "f64") as ctx:
        ctx.load_instances_symbolic(wl["offsets"], wl["sym"], wl["W"],
                                    wl["D"])
        ctx.centroids_set_symbolic(csym, Wc)
        ctx.labels_set(lab)
        ctx.barycenter(iters=30, init=d2.D2_INIT_PRODUCT)
        _, W0 = ctx.centroids_get()
        st = ctx.subgradient(iters=T, alpha=0.2, zeta=1.0)
        assert st["lp_failed"] == 0
        g_tr, _ = ctx.objective(T)
        _, Wg = ctx.centroids_get()
    off, D = wl["offsets"], wl["D"]
    for c in range(K):
        mem = np.nonzero(lab == c)[0]
        wys = [wl["W"][off[k]:off[k + 1]] for k in mem]
        blocks = [D[csym[c]][:, wl["sym"][off[k]:off[k + 1]]] for k in mem]
        r = osg.subgradient_barycenter(lambda _: blocks, None, wys, None,
                                       W0[c], T=T, alpha=0.2, zeta=1.0,
                                       fixed_support=True)
        assert _rel(g_tr[:, c], r["ftrace"]) < 1e-9
        assert np.abs(Wg[c] - r["w"]).max() < 1e-9
        assert g_tr[:, c].min() <= g_tr[0, c]

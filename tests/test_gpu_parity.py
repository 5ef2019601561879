"""GPU (HIP, through the C ABI) vs the FP64 oracle.

Bars (stated in the tests):
  FP64 device arithmetic: objective trace, centroids rel <= 1e-10; every
  entry of Pi1 and Pi2 within 1e-12 of the oracle's, Lambda / rho within
  1e-10.
  FP32 device arithmetic: objective trace rel <= 1e-5; every entry of Pi1
  and Pi2 (hence their row/column sums) within 1e-6 of the oracle's;
  Lambda / rho within PLAN_TOL["f32"][2]; centroid weights/supports within
  1e-5 (absolute, values are O(1)).
Lambda is compared divided by its cluster's rho: Eq. (badmm2) adds
rho (Pi1 - Pi2) per iteration, so Lambda / rho is the running sum of plan
differences, a quantity on the plans' scale.
Sizes span several workgroup chunks per cluster and ragged support sizes.
"""
import numpy as np
import pytest

import oracle
from synth.generators import make_workload, pick_init_members
from tests._helpers import oracle_barycenters, plan_errors

pytestmark = pytest.mark.gpu

# (Pi1 entries, Pi2 entries, Lambda / rho entries, marginals), absolute.
# FP32: an entry is at most its column's weight, so the 1e-6 bar on the
# marginals bounds the entries too; Lambda / rho sums the per-iteration
# differences Pi1 - Pi2 (T of them), whose FP32 rounding errors, a few ulp of
# values below 1 each, are bounded by 2e-7 * T in the worst case and largely
# cancel: 2e-5 covers T = 100 with margin.
PLAN_TOL = {"f64": (1e-12, 1e-12, 1e-10, 1e-12),
            "f32": (1e-6, 1e-6, 2e-5, 1e-6)}


def check_plans(ctx, wl, plans, ks, rhos, labels, dtype, local=None,
                tag=""):
    """Every entry of Pi1, Pi2 and Lambda / rho of instances ks against the
    oracle's plans (PLAN_TOL)."""
    errs = plan_errors(ctx, wl, plans, ks, lambda k: rhos[labels[k]],
                       local=local)
    print(f"  plan errors {tag} {dtype}: Pi1 {errs[0]:.3g} Pi2 {errs[1]:.3g}"
          f" Lambda/rho {errs[2]:.3g} marginals {errs[3]:.3g}", flush=True)
    for e, t, name in zip(errs, PLAN_TOL[dtype],
                          ("Pi1", "Pi2", "Lambda/rho", "marginals")):
        assert e <= t, (tag, name, e, t)
    return errs


@pytest.fixture(scope="module")
def d2():
    from paper_1510_00012_amd import d2 as mod
    mod.load_library()
    return mod


def _ctx(d2, wl, dtype):
    ctx = d2.D2Context(0, dtype)
    ctx.load_instances(wl["offsets"], wl["X"], wl["W"])
    return ctx


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_single_cluster_barycenter(d2, dtype, tol):
    """One cluster, N=256, m=8, d=3, m_k=8 (pixel-colour shape), 200
    iterations with support updates every 10."""
    print(f"[single_cluster {dtype}]", flush=True)
    wl = make_workload("gmm_d3_n256")
    mem = pick_init_members(wl["offsets"], 1, 8, wl["seed"])
    Xc, Wc = oracle.init_centroids(wl, mem, 8)
    lab = np.zeros(256, dtype=np.int32)
    res_o = []
    Xo, Wo, tr, rhos, plans = oracle_barycenters(wl, lab, Xc, Wc, T=200,
                                                 residuals=res_o)
    with _ctx(d2, wl, dtype) as ctx:
        ctx.centroids_set(Xc, Wc)
        ctx.labels_set(lab)
        st = ctx.barycenter(iters=200, tau=10, init=d2.D2_INIT_PRODUCT)
        g_tr, g_rho = ctx.objective(200)
        g_res = ctx.residual(200)
        # primal residual (1/N) sum |Pi1 - Pi2| after every iteration
        assert np.abs(g_res[:, 0] - res_o[0]).max() < (
            1e-12 if dtype == "f64" else 1e-6)
        Xg, Wg = ctx.centroids_get()
        assert _rel(g_rho, rhos) < (1e-12 if dtype == "f64" else 1e-6)
        assert _rel(g_tr[:, 0], tr[0]) < tol, np.max(np.abs(g_tr[:, 0] / tr[0] - 1))
        assert np.abs(Wg - Wo).max() < tol
        assert np.abs(Xg - Xo).max() < tol
        check_plans(ctx, wl, plans, range(256), rhos, lab, dtype,
                    tag="single")
        assert st["launches"] >= 200


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_multi_cluster_barycenter_ragged(d2, dtype):
    """K=4 clusters of a 6000-instance colour-like set (m_k in [4,16],
    m=16): many chunks per cluster, one empty cluster (label 4 unused)."""
    print(f"[multi_cluster {dtype}]", flush=True)
    wl = make_workload("gmm_d3_n65536_k16", N=6000)
    K = 5
    mem = pick_init_members(wl["offsets"], K, 16, 11)
    Xc, Wc = oracle.init_centroids(wl, mem, 16)
    lab, _, _ = oracle.assign(wl, Xc[:4], Wc[:4], T=50)
    res_o = []
    Xo, Wo, tr, rhos, plans = oracle_barycenters(wl, lab, Xc, Wc, T=60,
                                                 tau=10, residuals=res_o)
    tol = 1e-10 if dtype == "f64" else 1e-5
    with _ctx(d2, wl, dtype) as ctx:
        ctx.centroids_set(Xc, Wc)
        ctx.labels_set(lab)
        st = ctx.barycenter(iters=60, tau=10, init=d2.D2_INIT_PRODUCT)
        assert st["n_empty"] == 1
        g_tr, _ = ctx.objective(60)
        g_res = ctx.residual(60)
        for c in range(4):
            assert np.abs(g_res[:, c] - res_o[c]).max() < (
                1e-12 if dtype == "f64" else 1e-6), c
        assert np.all(g_res[:, 4] == 0)
        Xg, Wg = ctx.centroids_get()
        for c in range(4):
            assert _rel(g_tr[:, c], tr[c]) < tol, (c, _rel(g_tr[:, c], tr[c]))
        assert np.abs(Wg - Wo).max() < tol
        assert np.abs(Xg - Xo).max() < tol
        # the empty cluster keeps its centroid (weights as renormalised by
        # d2_centroids_set)
        assert np.array_equal(Xg[4], Xc[4])
        np.testing.assert_allclose(Wg[4], Wc[4] / Wc[4].sum(), rtol=0,
                                   atol=1e-16)
        ks = np.linspace(0, 5999, 300).astype(int)
        check_plans(ctx, wl, plans, ks, rhos, lab, dtype, tag="multi")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("name,m,rule,fixed", [
    ("gmm_d3_n65536_k16", 16, 2, False),
    ("gmm_d3_n65536_k16", 16, 1, True),
    ("gmm_d3_n65536_k16", 16, 2, True),
    ("gmm_d16_n2000000_k256", 16, 2, False),
    ("gmm_d16_n2000000_k256", 16, 1, True),
    ("topic_d64_n200000_k64", 32, 2, False)])
def test_rule2_and_fixed_support(d2, dtype, name, m, rule, fixed):
    """The R2 weight rule (Eq. (badmmw2): w proportional to the squared mean
    of sqrt(w~^(k))) and the fixed-support barycenter (no Eq. (updatex)
    step: the oracle runs with a support-update period beyond T) on the
    on-the-fly (d = 3) and cached-cost (d = 16, 64) paths: objective trace,
    centroids and every plan entry against the oracle."""
    print(f"[rule={rule} fixed={fixed} {name} {dtype}]", flush=True)
    N = 3000
    wl = make_workload(name, N=N)
    K = 3
    mem = pick_init_members(wl["offsets"], K, m, 19)
    Xc, Wc = oracle.init_centroids(wl, mem, m)
    lab, _, _ = oracle.assign(wl, Xc, Wc, T=30)
    T = 40
    Xo, Wo, tr, rhos, plans = oracle_barycenters(
        wl, lab, Xc, Wc, T=T, tau=(10 ** 9 if fixed else 10), rule=rule)
    tol = 1e-10 if dtype == "f64" else 1e-5
    with _ctx(d2, wl, dtype) as ctx:
        ctx.centroids_set(Xc, Wc)
        ctx.labels_set(lab)
        ctx.barycenter(iters=T, tau=10, rule=rule, fixed_support=fixed,
                       init=d2.D2_INIT_PRODUCT)
        g_tr, _ = ctx.objective(T)
        Xg, Wg = ctx.centroids_get()
        for c in range(K):
            if tr[c] is not None:
                assert _rel(g_tr[:, c], tr[c]) < tol, (c, _rel(g_tr[:, c],
                                                           tr[c]))
        assert np.abs(Wg - Wo).max() < tol
        if fixed:
            assert np.array_equal(Xg, Xc)
        else:
            assert np.abs(Xg - Xo).max() < tol
        check_plans(ctx, wl, plans, range(0, N, 3), rhos, lab, dtype,
                    tag=f"rule={rule} fixed={fixed} {name}")


def test_edge_shapes(d2):
    """m not a power of two (m=6), single-point instances, zero weights,
    the largest supported tile (m=32, m_k=64) and d=1."""
    print("[edge_shapes]", flush=True)
    rng = np.random.default_rng(5)
    sizes = np.concatenate([[1, 1, 64, 2, 63], rng.integers(1, 40, 200)])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    for d, m in ((1, 6), (3, 32)):
        X = rng.random((n, d))
        W = np.concatenate([rng.dirichlet(np.ones(s)) for s in sizes])
        W[off[2] + 5] = 0.0          # zero-weight support point
        W[off[2]:off[3]] /= W[off[2]:off[3]].sum()
        wl = {"offsets": off, "X": X, "W": W}
        Xc = rng.random((2, m, d))
        Wc = rng.dirichlet(np.ones(m), size=2)
        lab = (np.arange(len(sizes)) % 2).astype(np.int32)
        Xo, Wo, tr, rhos, plans = oracle_barycenters(wl, lab, Xc, Wc, T=25,
                                                     tau=5)
        with _ctx(d2, wl, "f32") as ctx:
            ctx.centroids_set(Xc, Wc)
            ctx.labels_set(lab)
            ctx.barycenter(iters=25, tau=5, init=d2.D2_INIT_PRODUCT)
            g_tr, _ = ctx.objective(25)
            Xg, Wg = ctx.centroids_get()
            for c in range(2):
                assert _rel(g_tr[:, c], tr[c]) < 1e-5
            assert np.abs(Wg - Wo).max() < 1e-5
            assert np.abs(Xg - Xo).max() < 1e-5
            check_plans(ctx, wl, plans, range(len(sizes)), rhos, lab,
                        "f32", tag=f"edge d={d} m={m}")


@pytest.mark.parametrize("name,m", [("topic_d64_n200000_k64", 32), ("gmm_d16_n2000000_k256", 16)])
def test_large_d_cached_cost_path(d2, name, m):
    """d=64 (word-vector-bag shape, bf16-exact unit vectors), m=32, m_k in
    [8,64], and d=16 (m=16, m_k in [4,32]): the cost is cached per support
    update instead of recomputed.  For d=64 the support-update sums and the
    cost recomputation run on the matrix cores (FP32 MFMA, used for
    32 <= d <= 64); for d=16 both run on the vector units."""
    print(f"[large_d {name}]", flush=True)
    wl = make_workload(name, N=1500)
    mem = pick_init_members(wl["offsets"], 3, m, 4)
    Xc, Wc = oracle.init_centroids(wl, mem, m)
    lab, _, _ = oracle.assign(wl, Xc, Wc, T=30)
    Xo, Wo, tr, rhos, plans = oracle_barycenters(wl, lab, Xc, Wc, T=30,
                                                 tau=10)
    with _ctx(d2, wl, "f32") as ctx:
        ctx.centroids_set(Xc, Wc)
        ctx.labels_set(lab)
        ctx.barycenter(iters=30, tau=10, init=d2.D2_INIT_PRODUCT)
        g_tr, _ = ctx.objective(30)
        Xg, Wg = ctx.centroids_get()
        for c in range(3):
            if tr[c] is not None:
                assert _rel(g_tr[:, c], tr[c]) < 1e-5
        assert np.abs(Wg - Wo).max() < 1e-5
        assert np.abs(Xg - Xo).max() < 1e-5
        check_plans(ctx, wl, plans, range(0, 1500, 3), rhos, lab, "f32",
                    tag=name)


def test_warm_start_and_support_update(d2):
    """Second call with the cached-plan warm start (Sec. 5) for members whose
    label did not change; then the standalone support update (Eq. updatex)
    from the cached Pi2."""
    print("[warm_start]", flush=True)
    wl = make_workload("gmm_d3_n65536_k16", N=3000)
    mem = pick_init_members(wl["offsets"], 3, 16, 2)
    Xc, Wc = oracle.init_centroids(wl, mem, 16)
    lab1, _, _ = oracle.assign(wl, Xc, Wc, T=40)
    X1, W1, _, _, plans = oracle_barycenters(wl, lab1, Xc, Wc, T=30)
    lab2, _, _ = oracle.assign(wl, X1, W1, T=40)
    warm = (lab2 == lab1)
    assert 0 < warm.sum() < len(warm) or warm.all()
    X2, W2, tr2, rhos2, plans = oracle_barycenters(wl, lab2, X1, W1,
                                                   plans=plans, warm=warm,
                                                   T=30)
    with _ctx(d2, wl, "f64") as ctx:
        ctx.centroids_set(Xc, Wc)
        ctx.labels_set(lab1)
        ctx.barycenter(iters=30, init=d2.D2_INIT_PRODUCT)
        # continue from the oracle's centroids so both sides see the same x
        ctx.centroids_set(X1, W1)
        ctx.labels_set(lab2)
        ctx.barycenter(iters=30, init=d2.D2_INIT_CACHED)
        g_tr, _ = ctx.objective(30)
        for c in range(3):
            assert _rel(g_tr[:, c], tr2[c]) < 1e-9
        # the warm-started plans entry by entry (both sides started the
        # unchanged-label members from their own cached Pi2)
        check_plans(ctx, wl, plans, range(0, 3000, 3), rhos2, lab2, "f64",
                    tag="warm")
        ctx.support_update()
        Xs, _ = ctx.centroids_get()
    # oracle support update from its final Pi2 equals the barycenter's own
    # final update (T is a multiple of tau), i.e. X2
    np.testing.assert_allclose(Xs, X2, atol=1e-9)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_assignment(d2, dtype):
    """Assignment step: labels equal the oracle's except where the oracle's
    relative margin between best and second-best is below 1e-5; distances
    within 1e-5 (f32) / 1e-10 (f64) relative."""
    print(f"[assign {dtype}]", flush=True)
    wl = make_workload("gmm_d3_n65536_k16", N=2000)
    mem = pick_init_members(wl["offsets"], 6, 16, 9)
    Xc, Wc = oracle.init_centroids(wl, mem, 16)
    lab_o, best_o, dist_o = oracle.assign(wl, Xc, Wc, T=100, want_dist=True)
    srt = np.sort(dist_o, axis=1)
    margin = (srt[:, 1] - srt[:, 0]) / srt[:, 0]
    with _ctx(d2, wl, dtype) as ctx:
        ctx.centroids_set(Xc, Wc)
        lab_g, best_g, nch = ctx.assign(iters=100)
    assert nch == 2000
    tol = 1e-5 if dtype == "f32" else 1e-10
    assert _rel(best_g, best_o) < tol
    ok = (lab_g == lab_o) | (margin < 1e-5)
    assert ok.all(), np.nonzero(~ok)


def test_centroid_init_matches_oracle(d2):
    """Eq. (merge) initialisation computed by the library's host code."""
    print("[init]", flush=True)
    wl = make_workload("gmm_d3_n65536_k16", N=500)
    mem = pick_init_members(wl["offsets"], 4, 8, 3)
    Xo, Wo = oracle.init_centroids(wl, mem, 8)
    with _ctx(d2, wl, "f64") as ctx:
        ctx.centroids_init(mem, 8)
        Xg, Wg = ctx.centroids_get()
    np.testing.assert_allclose(Xg, Xo, atol=1e-14)
    np.testing.assert_allclose(Wg, Wo, atol=1e-14)


def test_clustering_rounds_teacher_forced(d2):
    """Three rounds of the clustering loop on a colour-like set; each round
    the GPU starts from the oracle's centroids and labels (teacher forcing):
    assignment labels agree off near-ties, the warm-started barycenter
    traces agree to 1e-5 (FP32)."""
    print("[cluster_rounds]", flush=True)
    wl = make_workload("gmm_d3_n65536_k16", N=4000)
    K = 4
    mem = pick_init_members(wl["offsets"], K, 16, 5)
    Xc, Wc = oracle.init_centroids(wl, mem, 16)
    plans = oracle.Plans(16, int(wl["offsets"][-1]))
    prev = None
    with _ctx(d2, wl, "f32") as ctx:
        for r in range(3):
            lab_o, _, dist_o = oracle.assign(wl, Xc, Wc, T=100, want_dist=True)
            srt = np.sort(dist_o, axis=1)
            margin = (srt[:, 1] - srt[:, 0]) / srt[:, 0]
            ctx.centroids_set(Xc, Wc)
            lab_g, _, _ = ctx.assign(iters=100)
            assert np.all((lab_g == lab_o) | (margin < 1e-5))
            warm = None if prev is None else (lab_o == prev)
            Xn, Wn, tr, _, plans = oracle_barycenters(
                wl, lab_o, Xc, Wc, plans=plans, warm=warm, T=50)
            ctx.labels_set(lab_o)
            ctx.barycenter(iters=50, init=d2.D2_INIT_PRODUCT if prev is None
                           else d2.D2_INIT_CACHED)
            g_tr, _ = ctx.objective(50)
            for c in range(K):
                if tr[c] is not None:
                    assert _rel(g_tr[:, c], tr[c]) < 1e-5, (r, c)
            Xc, Wc, prev = Xn, Wn, lab_o


def test_cluster_call_runs_and_is_deterministic(d2):
    """d2_cluster end to end twice from the same start: bitwise identical
    centroids and labels (fixed-order reductions, no float atomics)."""
    print("[cluster_determinism]", flush=True)
    wl = make_workload("gmm_d3_n65536_k16", N=5000)
    mem = pick_init_members(wl["offsets"], 8, 16, 1)
    outs = []
    for _ in range(2):
        with _ctx(d2, wl, "f32") as ctx:
            ctx.centroids_init(mem, 16)
            recs = ctx.cluster(3, iters=40)
            outs.append((*ctx.centroids_get(), ctx.labels_get(), recs))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][2], outs[1][2])
    assert outs[0][3][0]["n_changed"] == 5000
    assert [r["n_changed"] for r in outs[0][3]] == \
        [r["n_changed"] for r in outs[1][3]]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_assignment_pruning_is_exact(d2, dtype):
    """The lower-bound pruning of the assignment returns exactly the labels
    and minimal distances of the exhaustive search, while iterating fewer
    (instance, centroid) pairs."""
    print(f"[assign_prune {dtype}]", flush=True)
    wl = make_workload("gmm_d3_n65536_k16", N=4000)
    mem = pick_init_members(wl["offsets"], 16, 16, 23)
    Xc, Wc = oracle.init_centroids(wl, mem, 16)
    with _ctx(d2, wl, dtype) as ctx:
        ctx.centroids_set(Xc, Wc)
        lab_a, best_a, _ = ctx.assign(iters=100, prune=False)
        ev_a, tot = ctx.assign_pairs()
        lab_b, best_b, _ = ctx.assign(iters=100, prune=True)
        ev_b, _ = ctx.assign_pairs()
    assert ev_a == tot == 4000 * 16
    assert ev_b < tot
    assert np.array_equal(lab_a, lab_b)
    assert np.array_equal(best_a, best_b)


@pytest.mark.parametrize("name,N,K,m", [("gmm_d16_n2000000_k256", 240, 100, 16),
                                        ("topic_d64_n200000_k64", 160, 70, 32)])
def test_assignment_pruning_many_centroids(d2, name, N, K, m):
    """More centroids than lanes (the cheap bounds go 64 centroids at a
    time, the last block ragged): pruned = exhaustive bitwise, from the
    smallest-bound start and again from the previous labels; labels and
    distances against the oracle as in test_assignment; pair counts
    ordered (iterated <= costed <= total, costed = total without
    pruning)."""
    print(f"[assign prune many {name} K={K}]", flush=True)
    wl = make_workload(name, N=N)
    if np.sum(np.diff(wl["offsets"]) >= m) >= K:
        mem = pick_init_members(wl["offsets"], K, m, 31)
        Xc, Wc = oracle.init_centroids(wl, mem, m)
    else:
        # too few instances with m points: supports drawn from the pooled
        # instance points, random weights
        rng = np.random.Generator(np.random.PCG64(31))
        Xc = wl["X"][rng.choice(len(wl["X"]), size=(K, m))]
        Wc = rng.random((K, m)) + 0.05
        Wc /= Wc.sum(1, keepdims=True)
    with _ctx(d2, wl, "f32") as ctx:
        ctx.centroids_set(Xc, Wc)
        lab_a, best_a, _ = ctx.assign(iters=100, prune=False)
        ev_a, tot = ctx.assign_pairs()
        co_a = ctx.assign_pairs_costed()
        # labels of the exhaustive call are the previous labels now
        lab_c, best_c, nch = ctx.assign(iters=100, prune=True)
        ev_c, _ = ctx.assign_pairs()
        co_c = ctx.assign_pairs_costed()
    with _ctx(d2, wl, "f32") as ctx:
        ctx.centroids_set(Xc, Wc)
        lab_b, best_b, _ = ctx.assign(iters=100, prune=True)
        ev_b, _ = ctx.assign_pairs()
        co_b = ctx.assign_pairs_costed()
    assert ev_a == co_a == tot == N * K
    assert ev_b <= co_b <= tot and ev_b < tot
    assert ev_c <= co_c <= tot and ev_c < tot
    assert nch == 0
    for lab, best in ((lab_b, best_b), (lab_c, best_c)):
        assert np.array_equal(lab, lab_a)
        assert np.array_equal(best, best_a)
    lab_o, best_o, dist_o = oracle.assign(wl, Xc, Wc, T=100, want_dist=True)
    srt = np.sort(dist_o, axis=1)
    margin = (srt[:, 1] - srt[:, 0]) / srt[:, 0]
    assert _rel(best_a, best_o) < 1e-5
    ok = (lab_a == lab_o) | (margin < 1e-5)
    assert ok.all(), np.nonzero(~ok)


def test_graph_replay_matches_eager(d2):
    """The captured launch sequence replayed several times (labels, warm
    start and centroids changing in between, eager assignment work between
    replays) gives bitwise the results of host-issued launches."""
    print("[graph_replay]", flush=True)
    wl = make_workload("gmm_d3_n65536_k16", N=5000)
    mem = pick_init_members(wl["offsets"], 6, 16, 8)
    with _ctx(d2, wl, "f32") as g, _ctx(d2, wl, "f32") as e:
        e.set_graph(False)
        g.centroids_init(mem, 16)
        e.centroids_init(mem, 16)
        for r in range(4):
            lab_g, _, _ = g.assign(iters=60)
            lab_e, _, _ = e.assign(iters=60)
            assert np.array_equal(lab_g, lab_e)
            init = d2.D2_INIT_PRODUCT if r == 0 else d2.D2_INIT_CACHED
            sg = g.barycenter(iters=30, init=init)
            se = e.barycenter(iters=30, init=init)
            assert sg["graph"] == 1 and se["graph"] == 0
            assert sg["launches"] == se["launches"]
            Xg, Wg = g.centroids_get()
            Xe, We = e.centroids_get()
            assert np.array_equal(Xg, Xe) and np.array_equal(Wg, We), r
            tg, _ = g.objective(30)
            te, _ = e.objective(30)
            assert np.array_equal(tg, te)


def test_graph_replay_with_buckets_matches_eager(d2):
    """Slot buckets (every class its own launch) and assignment slot classes
    run side by side on forked streams; the captured graph with those
    parallel branches, replayed over several rounds, gives bitwise the
    results of host-issued launches."""
    print("[graph_replay buckets]", flush=True)
    wl = make_workload("topic_d64_n200000_k64", N=1500)
    mem = pick_init_members(wl["offsets"], 3, 32, 6)
    with _ctx(d2, wl, "f32") as g, _ctx(d2, wl, "f32") as e:
        e.set_graph(False)
        for ctx in (g, e):
            ctx.set_bucketing(0)
            ctx.centroids_init(mem, 32)
        for r in range(3):
            lab_g, best_g, _ = g.assign(iters=40)
            lab_e, best_e, _ = e.assign(iters=40)
            assert np.array_equal(lab_g, lab_e) and np.array_equal(best_g,
                                                                   best_e)
            init = d2.D2_INIT_PRODUCT if r == 0 else d2.D2_INIT_CACHED
            sg = g.barycenter(iters=20, init=init)
            se = e.barycenter(iters=20, init=init)
            assert sg["graph"] == 1 and se["graph"] == 0
            assert sg["launches"] == se["launches"]
            Xg, Wg = g.centroids_get()
            Xe, We = e.centroids_get()
            assert np.array_equal(Xg, Xe) and np.array_equal(Wg, We), r
            tg, _ = g.objective(20)
            te, _ = e.objective(20)
            assert np.array_equal(tg, te)


def test_autotune_then_parity(d2):
    """The autotuner restores the centroids, picks a valid schedule, and the
    tuned barycenter still matches the oracle."""
    print("[autotune]", flush=True)
    wl = make_workload("gmm_d3_n65536_k16", N=6000)
    mem = pick_init_members(wl["offsets"], 4, 16, 12)
    Xc, Wc = oracle.init_centroids(wl, mem, 16)
    lab, _, _ = oracle.assign(wl, Xc, Wc, T=40)
    _, _, tr, _, _ = oracle_barycenters(wl, lab, Xc, Wc, T=40)
    with _ctx(d2, wl, "f32") as ctx:
        ctx.centroids_set(Xc, Wc)
        ctx.labels_set(lab)
        sch = ctx.autotune(iters=10)
        assert sch["chunk"] in (16, 32, 64, 128, 256)
        assert sch["waves"] in (2, 4) and sch["ms"] > 0
        assert sch["bucket"] in (100, 10)
        X0, W0 = ctx.centroids_get()
        assert np.array_equal(X0, Xc)
        np.testing.assert_allclose(W0, Wc / Wc.sum(1, keepdims=True),
                                   atol=1e-16)
        ctx.barycenter(iters=40, init=d2.D2_INIT_CACHED)
        g_tr, _ = ctx.objective(40)
        for c in range(4):
            if tr[c] is not None:
                assert _rel(g_tr[:, c], tr[c]) < 1e-5


@pytest.mark.parametrize("name,N,K,m", [("topic_d64_n200000_k64", 1200, 5, 32),
                                        ("gmm_d16_n2000000_k256", 1500, 4, 16)])
def test_assignment_split_by_slot_class(d2, name, N, K, m):
    """Larger tiles (d = 64 / 16, m_k up to 64 / 32): the assignment runs
    one launch per slot class; labels and distances as in
    test_assignment."""
    print(f"[assign split {name}]", flush=True)
    wl = make_workload(name, N=N)
    mem = pick_init_members(wl["offsets"], K, m, 21)
    Xc, Wc = oracle.init_centroids(wl, mem, m)
    lab_o, best_o, dist_o = oracle.assign(wl, Xc, Wc, T=100, want_dist=True)
    srt = np.sort(dist_o, axis=1)
    margin = (srt[:, 1] - srt[:, 0]) / srt[:, 0]
    with _ctx(d2, wl, "f32") as ctx:
        ctx.centroids_set(Xc, Wc)
        lab_g, best_g, _ = ctx.assign(iters=100)
    assert _rel(best_g, best_o) < 1e-5
    ok = (lab_g == lab_o) | (margin < 1e-5)
    assert ok.all(), np.nonzero(~ok)


def test_slot_buckets_match_oracle(d2):
    """The plan update split into one launch per slot bucket (threshold 0:
    every class present its own launch; 100: one launch) gives the same
    centroids and objective trace, against the oracle, on the d = 64
    shape whose m_k spans four slot classes."""
    print("[slot buckets]", flush=True)
    wl = make_workload("topic_d64_n200000_k64", N=1500)
    mem = pick_init_members(wl["offsets"], 3, 32, 4)
    Xc, Wc = oracle.init_centroids(wl, mem, 32)
    lab, _, _ = oracle.assign(wl, Xc, Wc, T=30)
    Xo, Wo, tr, rhos, plans = oracle_barycenters(wl, lab, Xc, Wc, T=30,
                                                 tau=10)
    res = {}
    with _ctx(d2, wl, "f32") as ctx:
        for pct in (0, 10, 100):
            ctx.set_bucketing(pct)
            ctx.centroids_set(Xc, Wc)
            ctx.labels_set(lab)
            st = ctx.barycenter(iters=30, tau=10, init=d2.D2_INIT_PRODUCT)
            g_tr, _ = ctx.objective(30)
            Xg, Wg = ctx.centroids_get()
            for c in range(3):
                if tr[c] is not None:
                    assert _rel(g_tr[:, c], tr[c]) < 1e-5, (pct, c)
            assert np.abs(Wg - Wo).max() < 1e-5, pct
            assert np.abs(Xg - Xo).max() < 1e-5, pct
            check_plans(ctx, wl, plans, range(0, 1500, 7), rhos, lab, "f32",
                        tag=f"buckets {pct}")
            res[pct] = (st["launches"], Xg)
    # more buckets, more launches per iteration
    assert res[0][0] > res[100][0]
    np.testing.assert_allclose(res[0][1], res[100][1], rtol=0, atol=1e-6)


@pytest.mark.parametrize("d,m,mk_hi", [(37, 20, 40), (33, 13, 50)])
def test_matrix_core_paths_ragged(d2, d, m, mk_hi):
    """Odd d in the matrix-core range (support sums for d >= 32, cost for
    pad(m) = 32 or 16 with d <= 64), m below its padding, ragged m_k: the
    padded rows, coordinates and columns must not leak into the result."""
    from synth.generators import gaussian_mixture_workload
    print(f"[mfma ragged d={d} m={m}]", flush=True)
    wl = gaussian_mixture_workload(77 + d, 900, d, 4, mk_hi, 12, 3, 0.1, 1.0)
    mem = pick_init_members(wl["offsets"], 3, m, 5)
    Xc, Wc = oracle.init_centroids(wl, mem, m)
    lab, _, _ = oracle.assign(wl, Xc, Wc, T=30)
    Xo, Wo, tr, rhos, plans = oracle_barycenters(wl, lab, Xc, Wc, T=30,
                                                 tau=10)
    with _ctx(d2, wl, "f32") as ctx:
        ctx.centroids_set(Xc, Wc)
        ctx.labels_set(lab)
        ctx.barycenter(iters=30, tau=10, init=d2.D2_INIT_PRODUCT)
        g_tr, _ = ctx.objective(30)
        Xg, Wg = ctx.centroids_get()
        for c in range(3):
            if tr[c] is not None:
                assert _rel(g_tr[:, c], tr[c]) < 1e-5, c
        assert np.abs(Wg - Wo).max() < 1e-5
        assert np.abs(Xg - Xo).max() < 1e-5
        check_plans(ctx, wl, plans, range(0, 900, 2), rhos, lab, "f32",
                    tag=f"mfma d={d} m={m}")


@pytest.mark.parametrize("d,m,mk_hi", [(5, 16, 30), (37, 20, 40),
                                       (13, 9, 60), (7, 40, 30), (6, 5, 50)])
def test_assignment_bound_odd_shapes(d2, d, m, mk_hi):
    """Pruned assignment with odd d (stride padding), m below its tile
    padding (tiles of 64, 32, 16 and 8 rows: the transport's column sums by
    reduce-scatter and per lane), ragged m_k up to mk_hi and more centroids
    than lanes, on points
    far from the origin: pruning stays exact (labels and distances bitwise
    those of the exhaustive search) and labels / distances match the oracle
    as in test_assignment."""
    from synth.generators import gaussian_mixture_workload
    print(f"[assign bound d={d} m={m} mk_hi={mk_hi}]", flush=True)
    wl = gaussian_mixture_workload(91 + d, 300, d, 4, mk_hi, 24, 6, 0.1, 1.0)
    K = 70
    if m <= mk_hi:
        mem = pick_init_members(wl["offsets"], K, m, 13)
        Xc, Wc = oracle.init_centroids(wl, mem, m)
    else:
        # centroids with more support points than any instance: points
        # drawn from the whole workload, Dirichlet weights
        rng = np.random.default_rng(17 + m)
        X = wl["X"]
        Xc = X[rng.integers(0, len(X), size=K * m)].reshape(K, m, d)
        Wc = rng.dirichlet(np.ones(m), size=K)
    with _ctx(d2, wl, "f32") as ctx:
        ctx.centroids_set(Xc, Wc)
        lab_a, best_a, _ = ctx.assign(iters=50, prune=False)
        lab_b, best_b, _ = ctx.assign(iters=50, prune=True)
        ev_b, tot = ctx.assign_pairs()
    assert ev_b < tot
    assert np.array_equal(lab_a, lab_b)
    assert np.array_equal(best_a, best_b)
    lab_o, best_o, dist_o = oracle.assign(wl, Xc, Wc, T=50, want_dist=True)
    srt = np.sort(dist_o, axis=1)
    margin = (srt[:, 1] - srt[:, 0]) / srt[:, 0]
    assert _rel(best_a, best_o) < 1e-5
    ok = (lab_a == lab_o) | (margin < 1e-5)
    assert ok.all(), np.nonzero(~ok)


@pytest.mark.parametrize("name,N,K,m", [("gmm_d16_n2000000_k256", 3000, 100, 16),
                                        ("topic_d64_n200000_k64", 1500, 70, 32),
                                        ("gmm_d3_n65536_k16", 4000, 16, 16)])
def test_assignment_cross_round_bounds_exact(d2, name, N, K, m):
    """Four assignment rounds with centroids moving in between (first a
    B-ADMM update and a jitter of every support point, the large move of an
    early round; then small jitters, the moves of late rounds): the pruned
    assignment with cross-round bounds returns bitwise the labels and
    minimal distances of the exhaustive search and of pruning without
    stored bounds, never forms more cost blocks than pruning without them,
    and forms fewer once the moves are small."""
    print(f"[cross-round bounds {name} K={K}]", flush=True)
    wl = make_workload(name, N=N)
    d = wl["X"].shape[1]
    rng = np.random.Generator(np.random.PCG64(77))
    if np.sum(np.diff(wl["offsets"]) >= m) >= K:
        mem = pick_init_members(wl["offsets"], K, m, 41)
        Xc, Wc = oracle.init_centroids(wl, mem, m)
    else:
        Xc = wl["X"][rng.choice(len(wl["X"]), size=(K, m))]
        Wc = rng.random((K, m)) + 0.05
        Wc /= Wc.sum(1, keepdims=True)
    with _ctx(d2, wl, "f32") as A, _ctx(d2, wl, "f32") as B, \
            _ctx(d2, wl, "f32") as C:
        C.set_assign_bounds(False)
        for r in range(4):
            for ctx in (A, B, C):
                ctx.centroids_set(Xc, Wc)
            la, ba, _ = A.assign(iters=60, prune=True)
            lb, bb, _ = B.assign(iters=60, prune=False)
            lc, bc, _ = C.assign(iters=60, prune=True)
            co_a, co_c = A.assign_pairs_costed(), C.assign_pairs_costed()
            print(f"  round {r}: cost blocks with bounds {co_a}, without "
                  f"{co_c} of {N * K}", flush=True)
            assert np.array_equal(la, lb) and np.array_equal(ba, bb), r
            assert np.array_equal(lc, lb) and np.array_equal(bc, bb), r
            assert co_a <= co_c, r
            if r >= 2:
                assert co_a < co_c, r
            # move the centroids: after the first round a short B-ADMM
            # update on these labels and a jitter of every support point,
            # later only a small jitter
            if r == 0:
                A.barycenter(iters=20, init=d2.D2_INIT_PRODUCT)
                Xc, Wc = A.centroids_get()
                scale = 0.02 * np.abs(Xc).mean()
            else:
                scale = 1e-3 * np.abs(Xc).mean()
            Xc = Xc + scale * rng.standard_normal(Xc.shape)
            Wc = Wc / Wc.sum(1, keepdims=True)


@pytest.mark.parametrize("name,m", [("gmm_d3_n65536_k16", 16),
                                    ("gmm_d16_n2000000_k256", 16)])
def test_cache_policy_is_bitwise_neutral(d2, name, m):
    """The streaming (non-temporal) plan-state accesses of the per-iteration
    kernel change where lines are kept, not what is computed: forced on and
    forced off give bitwise the same traces, centroids and plans (on the
    on-the-fly cost path, d = 3, and the cached-cost path, d = 16)."""
    print(f"[cache policy {name}]", flush=True)
    wl = make_workload(name, N=3000)
    mem = pick_init_members(wl["offsets"], 3, m, 9)
    Xc, Wc = oracle.init_centroids(wl, mem, m)
    lab, _, _ = oracle.assign(wl, Xc, Wc, T=20)
    out = []
    for policy in (1, 2):
        with _ctx(d2, wl, "f32") as ctx:
            ctx.set_cache_policy(policy)
            ctx.centroids_set(Xc, Wc)
            ctx.labels_set(lab)
            ctx.barycenter(iters=25, tau=10, init=d2.D2_INIT_PRODUCT)
            tr, _ = ctx.objective(25)
            X, W = ctx.centroids_get()
            P = [ctx.plans_get(k) for k in range(0, 3000, 97)]
            out.append((tr, X, W, P))
    (t1, x1, w1, p1), (t2, x2, w2, p2) = out
    assert np.array_equal(t1, t2) and np.array_equal(x1, x2)
    assert np.array_equal(w1, w2)
    for a, b in zip(p1, p2):
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


@pytest.mark.parametrize("shift", [0.0, 1000.0])
def test_assignment_batched_bounds_far_from_origin(d2, shift):
    """The batched candidate bounds (FP32, d <= 16, K >= 32) use the Gram
    form of the cost over points centred on the instance mean, with a
    rounding margin.  With every point and centroid shifted far from the
    origin (where the uncentred expansion would cancel), pruned = exhaustive
    bitwise, from the smallest-bound start and from the previous labels."""
    print(f"[assign batched bounds shift={shift}]", flush=True)
    wl = make_workload("gmm_d16_n2000000_k256", N=1200)
    K, m = 48, 16
    rng = np.random.Generator(np.random.PCG64(77))
    Xc = wl["X"][rng.choice(len(wl["X"]), size=(K, m))]
    Wc = rng.random((K, m)) + 0.05
    Wc /= Wc.sum(1, keepdims=True)
    wl = dict(wl, X=wl["X"] + shift)
    Xc = Xc + shift
    with _ctx(d2, wl, "f32") as ctx:
        ctx.centroids_set(Xc, Wc)
        lab_a, best_a, _ = ctx.assign(iters=60, prune=False)
        lab_c, best_c, _ = ctx.assign(iters=60, prune=True)
        ev_c, tot = ctx.assign_pairs()
    with _ctx(d2, wl, "f32") as ctx:
        ctx.centroids_set(Xc, Wc)
        lab_b, best_b, _ = ctx.assign(iters=60, prune=True)
        ev_b, _ = ctx.assign_pairs()
    print(f"  pairs iterated: {ev_b} / {ev_c} of {tot}", flush=True)
    assert ev_b < tot and ev_c < tot
    for lab, best in ((lab_b, best_b), (lab_c, best_c)):
        assert np.array_equal(lab, lab_a)
        assert np.array_equal(best, best_a)

"""Pins of the FP64 oracle against values that do not come from the oracle.

Each test names the passage of the paper it checks and the independent
source of truth: an LP solve (scipy/HiGHS), a library routine (cdist,
linear_sum_assignment, scipy.optimize), a closed form or an invariant.
All CPU-only.
"""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment, linprog, minimize
from scipy.spatial.distance import cdist

from synth.generators import make_workload, pick_init_members


def _rand_dist(rng, m, d, alpha=1.0):
    return rng.random((m, d)), rng.dirichlet(alpha * np.ones(m))


def _w2_1d(a, wa, b, wb):
    """W_2^2 of two 1-D discrete distributions by the quantile formula."""
    ia, ib = np.argsort(a), np.argsort(b)
    a, wa, b, wb = a[ia], wa[ia], b[ib], wb[ib]
    ca, cb = np.cumsum(wa), np.cumsum(wb)
    ts = np.unique(np.concatenate([[0.0], ca, cb]))
    ts = ts[(ts >= 0) & (ts <= ca[-1] + 1e-15)]
    tot = 0.0
    for t0, t1 in zip(ts[:-1], ts[1:]):
        mid = 0.5 * (t0 + t1)
        qa = a[min(np.searchsorted(ca, mid), len(a) - 1)]
        qb = b[min(np.searchsorted(cb, mid), len(b) - 1)]
        tot += (t1 - t0) * (qa - qb) ** 2
    return tot


# ---------------------------------------------------------------- cost (a1)
def test_cost_block_matches_cdist(oracle_mod):
    """Sec. 2 item 6: C_ij = ||x_i - x^(k)_j||^2, against scipy cdist."""
    rng = np.random.default_rng(1)
    for m, mk, d in [(1, 1, 1), (8, 5, 3), (16, 31, 16), (32, 9, 64)]:
        x, y = rng.standard_normal((m, d)), rng.standard_normal((mk, d))
        C = oracle_mod.cost_block(x, y)
        np.testing.assert_allclose(C, cdist(x, y, "sqeuclidean"), rtol=1e-13,
                                   atol=1e-13)


# ------------------------------------------------------- exact W2 (Eq. primal)
def test_exact_w2_matches_assignment_and_quantiles(oracle_mod):
    """Eq. (primal): uniform equal-size case = linear assignment; 1-D case =
    quantile formula."""
    rng = np.random.default_rng(2)
    for _ in range(5):
        m = 6
        x, y = rng.random((m, 3)), rng.random((m, 3))
        u = np.full(m, 1.0 / m)
        C = cdist(x, y, "sqeuclidean")
        r, c = linear_sum_assignment(C)
        v, _ = oracle_mod.exact_w2(x, u, y, u)
        assert abs(v - C[r, c].sum() / m) < 1e-9
    for _ in range(5):
        a, wa = _rand_dist(rng, 5, 1)
        b, wb = _rand_dist(rng, 7, 1)
        v, _ = oracle_mod.exact_w2(a, wa, b, wb)
        assert abs(v - _w2_1d(a[:, 0], wa, b[:, 0], wb)) < 1e-9


# ------------------------------------------- B-ADMM with w fixed (Sec. 4 pilot)
@pytest.mark.parametrize("m,mk,d", [(4, 6, 2), (5, 7, 3), (8, 8, 1)])
def test_badmm_ot_converges_to_exact_w2(oracle_mod, m, mk, d):
    """With the centroid weights fixed the B-ADMM updates solve the transport
    LP in the limit (Sec. 4, first pilot study: indiscernible from LP at 5000
    iterations).  Pins the signs and scaling of both closed forms and of the
    dual step: a wrong sign or a dropped Lambda stops convergence."""
    rng = np.random.default_rng(3 + m)
    for _ in range(4):
        x, w = _rand_dist(rng, m, d)
        y, wy = _rand_dist(rng, mk, d)
        ex, _ = oracle_mod.exact_w2(x, w, y, wy)
        v = oracle_mod.badmm_ot(x, w, y, wy, T=5000)
        assert abs(v - ex) <= 1e-4 * ex + 1e-12, (v, ex)


def test_badmm_ot_plans_meet_marginals(oracle_mod):
    """Pi1 lies in Delta_{k,1} (column sums = instance weights, Eq. badmmc0)
    and Pi2 in Delta_{k,2}(w) (row sums = w, Eq. badmmc1) after any number of
    iterations; Lambda sums to zero (both plans carry unit mass)."""
    rng = np.random.default_rng(4)
    x, w = _rand_dist(rng, 6, 3)
    y, wy = _rand_dist(rng, 9, 3)
    for T in (1, 3, 50):
        _, (p1, p2, lam) = oracle_mod.badmm_ot(x, w, y, wy, T=T,
                                               return_plans=True)
        np.testing.assert_allclose(p1.sum(0), wy, atol=1e-14)
        np.testing.assert_allclose(p2.sum(1), w, atol=1e-14)
        assert abs(lam.sum()) < 1e-13


def _kl(p, q):
    return np.sum(p * np.log(p / q))


def test_pi1_step_is_the_constrained_kl_minimiser(oracle_mod):
    """Eq. (badmm0) per instance with eps = 0: Pi1^{n+1} minimises
    <C + Lambda^n, Pi> + rho KL(Pi, Pi2^n) over Delta_{k,1}.  The state
    (Pi2^n, Lambda^n) comes from an n-step run, Pi1^{n+1} from an (n+1)-step
    run; scipy SLSQP solves the problem independently."""
    rng = np.random.default_rng(5)
    m, mk = 3, 4
    x, w = _rand_dist(rng, m, 2)
    y, wy = _rand_dist(rng, mk, 2)
    C = cdist(x, y, "sqeuclidean")
    rho = 2.0 * C.mean()
    _, (_, p2, lam) = oracle_mod.badmm_ot(x, w, y, wy, T=2, eps=0.0,
                                          return_plans=True)
    _, (p1n, _, _) = oracle_mod.badmm_ot(x, w, y, wy, T=3, eps=0.0,
                                         return_plans=True)

    def obj(v):
        P = v.reshape(m, mk)
        return np.sum((C + lam) * P) + rho * _kl(P, p2)

    cons = [{"type": "eq", "fun": (lambda v, j=j: v.reshape(m, mk)[:, j].sum()
                                   - wy[j])} for j in range(mk)]
    res = minimize(obj, p2.reshape(-1), method="SLSQP", constraints=cons,
                   bounds=[(1e-12, 1)] * (m * mk),
                   options={"ftol": 1e-15, "maxiter": 500})
    np.testing.assert_allclose(res.x.reshape(m, mk), p1n, atol=2e-6)


def test_pi2_step_is_the_constrained_kl_minimiser(oracle_mod):
    """Eq. (badmm1) with w fixed and eps = 0: Pi2^{n+1} minimises
    -<Lambda^n, Pi> + rho KL(Pi, Pi1^{n+1}) over Delta_{k,2}(w)."""
    rng = np.random.default_rng(6)
    m, mk = 3, 4
    x, w = _rand_dist(rng, m, 2)
    y, wy = _rand_dist(rng, mk, 2)
    C = cdist(x, y, "sqeuclidean")
    rho = 2.0 * C.mean()
    _, (_, _, lam) = oracle_mod.badmm_ot(x, w, y, wy, T=2, eps=0.0,
                                         return_plans=True)
    _, (p1n, p2n, _) = oracle_mod.badmm_ot(x, w, y, wy, T=3, eps=0.0,
                                           return_plans=True)

    def obj(v):
        P = v.reshape(m, mk)
        return -np.sum(lam * P) + rho * _kl(P, p1n)

    cons = [{"type": "eq", "fun": (lambda v, i=i: v.reshape(m, mk)[i].sum()
                                   - w[i])} for i in range(m)]
    res = minimize(obj, p1n.reshape(-1), method="SLSQP", constraints=cons,
                   bounds=[(1e-12, 1)] * (m * mk),
                   options={"ftol": 1e-15, "maxiter": 500})
    np.testing.assert_allclose(res.x.reshape(m, mk), p2n, atol=2e-6)


# ------------------------------------------------------------ barycenter (Alg. 4)
def _tiny_cluster(rng, N, m, mk_max, d):
    sizes = rng.integers(1, mk_max + 1, size=N)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = rng.random((off[-1], d))
    W = np.concatenate([rng.dirichlet(np.ones(s)) for s in sizes])
    return {"offsets": off, "X": X, "W": W}


def _fullbatch_lp(wl, x):
    """Eq. (fullbatch-lp) at fixed support x: min over w in Delta_m and
    couplings with row sums w and column sums w^(k); returns (obj/N, w)."""
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    N = len(off) - 1
    m = x.shape[0]
    blocks = [(off[k], off[k + 1] - off[k]) for k in range(N)]
    nv = m + sum(m * mk for _, mk in blocks)
    c = np.zeros(nv)
    rows, rhs = [], []
    col = m
    for (a, mk) in blocks:
        C = cdist(x, X[a:a + mk], "sqeuclidean")
        c[col:col + m * mk] = C.reshape(-1)          # row-major (i, j)
        for i in range(m):                           # row sums = w_i
            r = np.zeros(nv)
            r[col + i * mk:col + (i + 1) * mk] = 1.0
            r[i] = -1.0
            rows.append(r); rhs.append(0.0)
        for j in range(mk):                          # column sums = w^(k)_j
            r = np.zeros(nv)
            r[col + j:col + m * mk:mk] = 1.0
            rows.append(r); rhs.append(W[a + j])
        col += m * mk
    r = np.zeros(nv); r[:m] = 1.0
    rows.append(r); rhs.append(1.0)
    res = linprog(c, A_eq=np.array(rows), b_eq=np.array(rhs), bounds=(0, None),
                  method="highs")
    assert res.status == 0
    return res.fun / N, res.x[:m]


def test_fixed_support_barycenter_near_full_lp(oracle_mod):
    """Fixed support (no x update, tau > T): the B-ADMM weights are feasible
    for Eq. (centroid), so their exact objective is >= the full-batch LP
    optimum (Eq. fullbatch-lp) -- hard bound -- and close to it (Table 1
    reports 0.2-0.6 % gaps; we allow 3 %)."""
    rng = np.random.default_rng(7)
    gaps = []
    for trial in range(6):
        N, m, d = 6, 4, 2
        wl = _tiny_cluster(rng, N, m, 4, d)
        x = rng.random((m, d))
        w0 = np.full(m, 1.0 / m)
        out = oracle_mod.barycenter(wl, np.arange(N), x, w0, T=2000,
                                    tau=10 ** 6)
        lp, _ = _fullbatch_lp(wl, x)
        ft = oracle_mod.f_true(wl, range(N), x, out["w"])
        assert ft >= lp - 1e-9
        gaps.append((ft - lp) / lp)
    assert np.median(gaps) < 0.01 and max(gaps) < 0.03, gaps


def test_r1_is_reverse_kl_consensus(oracle_mod):
    """Eq. (badmmw): after one iteration (Lambda^0 = 0, so Pi1~ = Pi1 + eps),
    w^1 minimises sum_k KL(w~^(k), w) over the simplex (scipy SLSQP)."""
    rng = np.random.default_rng(8)
    wl = _tiny_cluster(rng, 5, 3, 4, 2)
    x = rng.random((3, 2))
    out = oracle_mod.barycenter(wl, np.arange(5), x, np.full(3, 1 / 3), T=1,
                                tau=10 ** 6, eps=0.0)
    off = wl["offsets"]
    wts = []
    for k in range(5):
        p1, _, _ = out["plans"].block(off, k)
        r = p1.sum(1)
        wts.append(r / r.sum())
    wts = np.array(wts)
    res = minimize(lambda v: np.sum(wts * (np.log(wts) - np.log(v))),
                   np.full(3, 1 / 3), method="SLSQP",
                   constraints=[{"type": "eq", "fun": lambda v: v.sum() - 1}],
                   bounds=[(1e-9, 1)] * 3, options={"ftol": 1e-15})
    np.testing.assert_allclose(out["w"], res.x, atol=1e-6)


def test_r2_is_hellinger_consensus(oracle_mod):
    """Eq. (badmmw2): sqrt(w) proportional to the mean of sqrt(w~^(k)), i.e.
    the simplex point maximising sum_k sum_i sqrt(w_i w~_i^(k))."""
    rng = np.random.default_rng(9)
    wl = _tiny_cluster(rng, 5, 3, 4, 2)
    x = rng.random((3, 2))
    out = oracle_mod.barycenter(wl, np.arange(5), x, np.full(3, 1 / 3), T=1,
                                tau=10 ** 6, eps=0.0, rule=2)
    off = wl["offsets"]
    wts = []
    for k in range(5):
        p1, _, _ = out["plans"].block(off, k)
        r = p1.sum(1)
        wts.append(r / r.sum())
    wts = np.array(wts)
    res = minimize(lambda v: -np.sum(np.sqrt(v * wts)), np.full(3, 1 / 3),
                   method="SLSQP",
                   constraints=[{"type": "eq", "fun": lambda v: v.sum() - 1}],
                   bounds=[(1e-9, 1)] * 3, options={"ftol": 1e-15})
    np.testing.assert_allclose(out["w"], res.x, atol=1e-6)


def test_support_update_minimises_transport_cost(oracle_mod):
    """Eq. (updatex): after the final support update (T a multiple of tau)
    x minimises sum_k <C(x, x^(k)), Pi2^(k)> for the returned Pi2 (BFGS)."""
    rng = np.random.default_rng(10)
    wl = _tiny_cluster(rng, 7, 4, 5, 3)
    off = wl["offsets"]
    x0 = rng.random((4, 3))
    out = oracle_mod.barycenter(wl, np.arange(7), x0, np.full(4, 0.25), T=20,
                                tau=10)
    blocks = [out["plans"].block(off, k)[1] for k in range(7)]

    def f(v):
        xx = v.reshape(4, 3)
        return sum(np.sum(cdist(xx, wl["X"][off[k]:off[k + 1]], "sqeuclidean")
                          * blocks[k]) for k in range(7))

    res = minimize(f, np.zeros(12), method="BFGS", options={"gtol": 1e-12})
    np.testing.assert_allclose(out["x"], res.x.reshape(4, 3), atol=1e-6)


def test_single_support_point_is_the_mean(oracle_mod):
    """m = 1 (the K-means special case): w = 1, x = (1/N) sum_k sum_j
    w^(k)_j x^(k)_j after the first support update, and the objective is the
    mean weighted squared distance to that point."""
    rng = np.random.default_rng(11)
    wl = _tiny_cluster(rng, 9, 1, 6, 3)
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    x0 = rng.random((1, 3))
    out = oracle_mod.barycenter(wl, np.arange(9), x0, np.ones(1), T=11, tau=10)
    mean = np.zeros(3)
    for k in range(9):
        mean += W[off[k]:off[k + 1]] @ X[off[k]:off[k + 1]]
    mean /= 9
    np.testing.assert_allclose(out["x"][0], mean, atol=1e-12)
    assert abs(out["w"][0] - 1.0) < 1e-15
    f10 = np.mean([W[off[k]:off[k + 1]] @ ((X[off[k]:off[k + 1]] - mean) ** 2)
                   .sum(1) for k in range(9)])
    assert abs(out["ftrace"][10] - f10) < 1e-12


def test_identical_members_fixed_point(oracle_mod):
    """All members equal P, started at x = support of P, w = weights of P and
    Pi2 = diag(w): one iteration leaves the centroid unchanged (exact fixed
    point of Eq. (centroid), objective 0)."""
    rng = np.random.default_rng(12)
    m, d, N = 5, 3, 4
    y, wy = _rand_dist(rng, m, d)
    wl = {"offsets": np.arange(0, (N + 1) * m, m).astype(np.int64),
          "X": np.tile(y, (N, 1)), "W": np.tile(wy, N)}
    plans = oracle_mod.Plans(m, N * m)
    for k in range(N):
        plans.P2[k * m * m:(k + 1) * m * m] = np.diag(wy).T.reshape(-1)
    out = oracle_mod.barycenter(wl, np.arange(N), y, wy, plans=plans,
                                warm=np.ones(N), T=10, tau=10)
    np.testing.assert_allclose(out["w"], wy, rtol=1e-12)
    np.testing.assert_allclose(out["x"], y, atol=1e-12)
    assert abs(out["ftrace"][-1]) < 1e-12


def test_barycenter_invariants_every_iteration(oracle_mod):
    """Column sums of every Pi1 = w^(k); row sums of every Pi2 = w; w in the
    simplex; sum Lambda^(k) = 0; ftrace matches <C, Pi1> from cdist."""
    wl = make_workload("gmm_d3_n256", N=24)
    off = wl["offsets"]
    mem = pick_init_members(off, 1, 8, 0)
    Xc, Wc = oracle_mod.init_centroids(wl, mem, 8)
    for T in (1, 7, 30):
        out = oracle_mod.barycenter(wl, np.arange(24), Xc[0], Wc[0], T=T,
                                    tau=10 ** 6)
        assert abs(out["w"].sum() - 1) < 1e-14 and np.all(out["w"] >= 0)
        f = 0.0
        for k in range(24):
            p1, p2, lam = out["plans"].block(off, k)
            np.testing.assert_allclose(p1.sum(0), wl["W"][off[k]:off[k + 1]],
                                       atol=1e-15)
            np.testing.assert_allclose(p2.sum(1), out["w"], atol=1e-15)
            assert abs(lam.sum()) < 1e-13
            f += np.sum(cdist(Xc[0], wl["X"][off[k]:off[k + 1]],
                              "sqeuclidean") * p1)
        assert abs(out["ftrace"][-1] - f / 24) < 1e-13


def test_rho_is_rho0_times_mean_cost(oracle_mod):
    """Eq. (rho), read as rho0 * mean_{k,i,j} c(x_i, x^(k)_j)."""
    wl = make_workload("gmm_d3_n256", N=10)
    off = wl["offsets"]
    x = wl["X"][:8]
    out = oracle_mod.barycenter(wl, np.arange(10), x, np.full(8, 1 / 8), T=1)
    allc = np.concatenate([cdist(x, wl["X"][off[k]:off[k + 1]],
                                 "sqeuclidean").ravel() for k in range(10)])
    assert abs(out["rho"] - 2.0 * allc.mean()) < 1e-13


def test_barycenter_thread_count_invariant(oracle_mod):
    """Fixed reduction order: results do not depend on the thread count."""
    wl = make_workload("gmm_d3_n65536_k16", N=300)
    mem = pick_init_members(wl["offsets"], 1, 16, 0)
    Xc, Wc = oracle_mod.init_centroids(wl, mem, 16)
    nt = oracle_mod.num_threads()
    try:
        oracle_mod.set_num_threads(1)
        a = oracle_mod.barycenter(wl, np.arange(300), Xc[0], Wc[0], T=20)
        oracle_mod.set_num_threads(max(nt, 4))
        b = oracle_mod.barycenter(wl, np.arange(300), Xc[0], Wc[0], T=20)
    finally:
        oracle_mod.set_num_threads(nt)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["w"], b["w"])
    assert np.array_equal(a["ftrace"], b["ftrace"])


def test_replicated_members_give_identical_centroid(oracle_mod):
    """Duplicating every member leaves Eq. (centroid) unchanged, so B-ADMM
    (whose updates are per-member plus a member mean) returns the same
    centroid up to rounding."""
    rng = np.random.default_rng(13)
    wl = _tiny_cluster(rng, 6, 4, 5, 2)
    off = wl["offsets"]
    sizes = np.diff(off)
    wl2 = {"offsets": np.concatenate([[0], np.cumsum(np.tile(sizes, 2))]),
           "X": np.tile(wl["X"], (2, 1)), "W": np.tile(wl["W"], 2)}
    x0, w0 = rng.random((4, 2)), np.full(4, 0.25)
    a = oracle_mod.barycenter(wl, np.arange(6), x0, w0, T=40, tau=10)
    b = oracle_mod.barycenter(wl2, np.arange(12), x0, w0, T=40, tau=10)
    np.testing.assert_allclose(a["x"], b["x"], atol=1e-12)
    np.testing.assert_allclose(a["w"], b["w"], atol=1e-12)
    np.testing.assert_allclose(a["ftrace"], b["ftrace"], rtol=1e-12)


# ------------------------------------------------------------- init (Eq. merge)
def test_ward_merge_pair_choice_and_moments(oracle_mod):
    """Eq. (merge): each merge takes the pair minimising
    w_a w_b ||x_a - x_b||^2 / (w_a + w_b) (checked against a pdist-based
    search), preserves total mass and the weighted mean, and the transport
    bound W^2(P, P') <= w_a||x_a - xbar||^2 + w_b||x_b - xbar||^2 holds."""
    from scipy.spatial.distance import pdist, squareform
    rng = np.random.default_rng(14)
    for _ in range(5):
        y, wy = _rand_dist(rng, 9, 3)
        D = squareform(pdist(y, "sqeuclidean"))
        crit = np.outer(wy, wy) * D / (wy[:, None] + wy[None, :])
        crit[np.tril_indices(9)] = np.inf
        a, b = np.unravel_index(np.argmin(crit), crit.shape)
        x, w = oracle_mod.ward_merge(y, wy, 8)
        xbar = (wy[a] * y[a] + wy[b] * y[b]) / (wy[a] + wy[b])
        keep = [q for q in range(9) if q != b]
        exp_x = y[keep].copy()
        exp_x[keep.index(a)] = xbar
        np.testing.assert_allclose(x, exp_x, atol=1e-15)
        assert abs(w.sum() - 1) < 1e-15
        np.testing.assert_allclose(w @ x, wy @ y, atol=1e-15)
        bound = wy[a] * ((y[a] - xbar) ** 2).sum() + wy[b] * ((y[b] - xbar) ** 2).sum()
        v, _ = oracle_mod.exact_w2(x, w, y, wy)
        assert v <= bound + 1e-12
        x4, w4 = oracle_mod.ward_merge(y, wy, 4)
        np.testing.assert_allclose(w4 @ x4, wy @ y, atol=1e-14)
        xs, ws = oracle_mod.ward_merge(y, wy, 9)
        assert np.array_equal(xs, y) and np.array_equal(ws, wy)


# ------------------------------------------------------ assignment (Alg. 1)
def test_assign_is_argmin_of_pair_values(oracle_mod):
    """Assignment step: label = argmin over centroids of the B-ADMM transport
    value (ties to the lowest index); on well-separated data it agrees with
    the exact-W^2 argmin (LP)."""
    wl = make_workload("gmm_d3_n65536_k16", N=40)
    off = wl["offsets"]
    mem = pick_init_members(off, 4, 16, 3)
    Xc, Wc = oracle_mod.init_centroids(wl, mem, 16)
    lab, best, dist = oracle_mod.assign(wl, Xc, Wc, T=100, want_dist=True)
    for k in range(40):
        a, b = off[k], off[k + 1]
        for c in range(4):
            v = oracle_mod.badmm_ot(Xc[c], Wc[c], wl["X"][a:b], wl["W"][a:b],
                                    T=100)
            assert v == dist[k, c]
        assert lab[k] == int(np.argmin(dist[k]))
        assert best[k] == dist[k].min()
    ex = np.array([[oracle_mod.exact_w2(Xc[c], Wc[c], wl["X"][off[k]:off[k + 1]],
                                        wl["W"][off[k]:off[k + 1]])[0]
                    for c in range(4)] for k in range(40)])
    srt = np.sort(ex, axis=1)
    clear = (srt[:, 1] - srt[:, 0]) > 0.2 * srt[:, 0]
    assert clear.sum() >= 10
    assert np.array_equal(lab[clear], np.argmin(ex, axis=1)[clear])


def test_cluster_loop_with_one_point_is_lloyd_on_means(oracle_mod):
    """Algorithm "D2 Clustering" with m = 1: W^2(Q, P) = ||mu_P - x_Q||^2 +
    var(P), so labels follow the nearest instance mean and each centroid
    becomes the mean of its members' means -- Lloyd's K-means on the
    instance means (own numpy Lloyd from the same start)."""
    wl = make_workload("gmm_d3_n65536_k16", N=200)
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    N = len(off) - 1
    means = np.array([W[off[k]:off[k + 1]] @ X[off[k]:off[k + 1]]
                      for k in range(N)])
    mem = pick_init_members(off, 5, 1, 21)
    Xc, Wc = oracle_mod.init_centroids(wl, mem, 1)
    np.testing.assert_allclose(Xc[:, 0], means[mem], atol=1e-14)
    out = oracle_mod.cluster(wl, Xc, Wc, rounds=4, T=10, tau=10)
    cen = means[mem].copy()
    for _ in range(4):
        lab = np.argmin(cdist(means, cen, "sqeuclidean"), axis=1)
        for c in range(5):
            if np.any(lab == c):
                cen[c] = means[lab == c].mean(0)
    assert np.array_equal(out["labels"], lab)
    np.testing.assert_allclose(out["Xc"][:, 0], cen, atol=1e-12)


def test_assignment_lower_bound_holds(oracle_mod):
    """The pruning bound used by the assignment: any plan with the instance's
    column sums (Pi1 after any number of iterations) costs at least
    sum_j w_j min_i C_ij; checked on the oracle's transport values and on
    the exact W^2 (LP)."""
    rng = np.random.default_rng(31)
    for _ in range(30):
        m, mk = rng.integers(1, 9), rng.integers(1, 9)
        x, w = _rand_dist(rng, m, 3)
        y, wy = _rand_dist(rng, mk, 3)
        lb = float(wy @ cdist(x, y, "sqeuclidean").min(axis=0))
        for T in (1, 5, 100):
            assert oracle_mod.badmm_ot(x, w, y, wy, T=T) >= lb * (1 - 1e-12)
        assert oracle_mod.exact_w2(x, w, y, wy)[0] >= lb * (1 - 1e-9)


def test_cheap_assignment_bound_below_full_bound(oracle_mod):
    """The cheap pruning bound (triangle inequality around the centroid mean
    mu_c with support radius rad_c and the instance mean mu_P):
    sum_j w_j max(0, |dist(mu_P, mu_c) - |y_j - mu_P|| - rad_c)^2 never
    exceeds sum_j w_j min_i C_ij, which never exceeds the transport value."""
    rng = np.random.default_rng(37)
    for _ in range(50):
        m, mk, d = rng.integers(1, 9), rng.integers(1, 9), rng.integers(1, 6)
        x, w = _rand_dist(rng, m, d)
        y, wy = _rand_dist(rng, mk, d)
        x = x + rng.normal(size=d) * rng.uniform(0, 3)
        C = cdist(x, y, "sqeuclidean")
        full = float(wy @ C.min(axis=0))
        mu_c = w @ x
        rad = np.sqrt(((x - mu_c) ** 2).sum(1)).max()
        mu_p = wy @ y
        dl = np.linalg.norm(mu_p - mu_c)
        rj = np.linalg.norm(y - mu_p, axis=1)
        gap = np.maximum(0.0, np.abs(dl - rj) - rad)
        cheap = float(wy @ gap ** 2)
        assert cheap <= full * (1 + 1e-12) + 1e-15
        assert full <= oracle_mod.badmm_ot(x, w, y, wy, T=50) * (1 + 1e-12)

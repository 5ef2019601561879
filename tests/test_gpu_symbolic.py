"""Symbolic supports on the GPU (Sec. 5: a finite symbol set with a given
symbol-to-symbol dissimilarity; the support step is skipped) against the
FP64 oracle, through the C ABI.  Bars as in test_gpu_parity: FP64 objective
trace / weights rel 1e-10, plan entries 1e-12, Lambda / rho 1e-10; FP32
objective trace rel 1e-5, weights and plan entries 1e-6, Lambda / rho
2e-5; assignment labels equal except at oracle margins below 1e-5, best
distances within 1e-5 relative (FP32) / 1e-10 (FP64)."""
import numpy as np
import pytest

import oracle
from synth.generators import make_workload, symbol_init_centroids
from tests._helpers import plan_errors

pytestmark = pytest.mark.gpu

PLAN_TOL = {"f64": (1e-12, 1e-12, 1e-10, 1e-12),
            "f32": (1e-6, 1e-6, 2e-5, 1e-6)}


@pytest.fixture(scope="module")
def d2():
    from paper_1510_00012_amd import d2 as mod
    mod.load_library()
    return mod


@pytest.fixture(scope="module")
def protein1():
    return make_workload("protein_g1_n10742_k10", N=2000)


@pytest.fixture(scope="module")
def protein3():
    return make_workload("protein_g3_n10742_k10", N=700)


def _ctx(d2, wl, dtype):
    ctx = d2.D2Context(0, dtype)
    ctx.load_instances_symbolic(wl["offsets"], wl["sym"], wl["W"], wl["D"])
    return ctx


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def _oracle_round(wl, lab, csym, Wc, T, plans, warm=None):
    K, m = csym.shape
    Wo, tr, rhos = Wc.copy(), [None] * K, np.zeros(K)
    for c in range(K):
        mem = np.nonzero(lab == c)[0]
        if len(mem) == 0:
            continue
        wm = None if warm is None else warm[mem].astype(np.uint8)
        out = oracle.barycenter_sym(wl, mem, csym[c], Wc[c], plans=plans,
                                    warm=wm, T=T)
        Wo[c], tr[c], rhos[c] = out["w"], out["ftrace"], out["rho"]
    return Wo, tr, rhos


def _check(ctx, wl, lab, Wo, tr, rhos, plans, T, dtype, tag, calls=1):
    """Bars per call: the second call starts from each side's own cached
    plans, which carry the first call's rounding."""
    g_tr, g_rho = ctx.objective(T)
    _, Wg = ctx.centroids_get()
    tol = 1e-10 if dtype == "f64" else 1e-5
    worst = max(_rel(g_tr[:, c], tr[c]) for c in range(len(tr))
                if tr[c] is not None)
    wrho = max(abs(g_rho[c] / rhos[c] - 1) for c in range(len(tr))
               if tr[c] is not None)
    errs = plan_errors(ctx, wl, plans, range(0, len(lab), 3),
                       lambda k: rhos[lab[k]])
    print(f"  {tag} {dtype}: trace rel {worst:.3g}, rho rel {wrho:.3g}, "
          f"weights {np.abs(Wg - Wo).max():.3g}, Pi1 {errs[0]:.3g} Pi2 "
          f"{errs[1]:.3g} Lambda/rho {errs[2]:.3g} marginals {errs[3]:.3g}",
          flush=True)
    assert worst < tol * calls and wrho < tol
    assert np.abs(Wg - Wo).max() < (1e-10 if dtype == "f64" else 1e-6) * calls
    for e, t in zip(errs, PLAN_TOL[dtype]):
        assert e <= t * calls


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("gram", [1, 3])
def test_symbolic_barycenter_matches_oracle(d2, protein1, protein3, dtype,
                                            gram):
    """All clusters in one batched call (the cached-cost path with the cost
    gathered from the symbol table), then a warm-started second call after
    a relabelling of a tenth of the instances: objective traces, rho,
    weights and every third instance's plans against the oracle; the
    centroid symbols stay as set."""
    wl = protein1 if gram == 1 else protein3
    print(f"[symbolic gram={gram} {dtype}]", flush=True)
    K, m, T = wl["K"], wl["m"], 50
    N = len(wl["offsets"]) - 1
    lab = wl["classes"].astype(np.int32)
    csym, Wc = symbol_init_centroids(wl, lab, K, m)
    plans = oracle.Plans(m, int(wl["offsets"][-1]))
    with _ctx(d2, wl, dtype) as ctx:
        ctx.centroids_set_symbolic(csym, Wc)
        ctx.labels_set(lab)
        ctx.barycenter(iters=T, init=d2.D2_INIT_PRODUCT)
        Wo, tr, rhos = _oracle_round(wl, lab, csym, Wc, T, plans)
        _check(ctx, wl, lab, Wo, tr, rhos, plans, T, dtype, "call 1")
        Xg, _ = ctx.centroids_get()
        assert np.array_equal(Xg[:, :, 0], csym.astype(np.float64))
        # second call: a tenth of the labels moved, the rest warm-started
        rng = np.random.Generator(np.random.PCG64(gram))
        lab2 = lab.copy()
        mv = rng.choice(N, size=N // 10, replace=False)
        lab2[mv] = (lab2[mv] + 1) % K
        ctx.centroids_set_symbolic(csym, Wo)
        ctx.labels_set(lab2)
        ctx.barycenter(iters=T, init=d2.D2_INIT_CACHED)
        Wo2, tr2, rhos2 = _oracle_round(wl, lab2, csym, Wo, T, plans,
                                        warm=(lab2 == lab))
        _check(ctx, wl, lab2, Wo2, tr2, rhos2, plans, T, dtype, "call 2",
               calls=2)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_symbolic_assignment_matches_oracle(d2, protein1, protein3, dtype):
    """Labels and minimal distances over symbolic supports (pruned and
    exhaustive give the same bits), against the oracle's exhaustive
    assignment; two pruned calls in a row with the same symbols reuse the
    cross-round bounds and form fewer cost blocks where the bound can
    prune at all (amino-acid centroids hold all 20 symbols, so their bound
    sum_j w_j min_i D[x_i, y_j] is 0; tripeptide centroids hold 32 of
    8000)."""
    for wl in (protein1, protein3):
        K, m = wl["K"], wl["m"]
        lab0 = wl["classes"].astype(np.int32)
        csym, Wc = symbol_init_centroids(wl, lab0, K, m)
        rng = np.random.Generator(np.random.PCG64(3))
        Wc = rng.dirichlet(np.ones(m), size=K)
        lab_o, best_o, dist_o = oracle.assign_sym(wl, csym, Wc, T=60,
                                                  want_dist=True)
        srt = np.sort(dist_o, axis=1)
        margin = (srt[:, 1] - srt[:, 0]) / srt[:, 0]
        with _ctx(d2, wl, dtype) as A, _ctx(d2, wl, dtype) as B:
            A.centroids_set_symbolic(csym, Wc)
            B.centroids_set_symbolic(csym, Wc)
            la, ba, _ = A.assign(iters=60, prune=True)
            lb, bb, _ = B.assign(iters=60, prune=False)
            assert np.array_equal(la, lb) and np.array_equal(ba, bb)
            r = _rel(ba, best_o)
            ok = (la == lab_o) | (margin < 1e-5)
            print(f"  symbolic assignment S={wl['S']} {dtype}: distance rel "
                  f"{r:.3g}, {int((la != lab_o).sum())} label differences "
                  f"({int((~ok).sum())} outside near-ties)", flush=True)
            assert r < (1e-10 if dtype == "f64" else 1e-5)
            assert ok.all()
            c1 = A.assign_pairs_costed()
            # new weights, same symbols: the stored bounds stay valid
            A.centroids_set_symbolic(csym, Wc[::-1].copy())
            B.centroids_set_symbolic(csym, Wc[::-1].copy())
            la2, ba2, _ = A.assign(iters=60, prune=True)
            lb2, bb2, _ = B.assign(iters=60, prune=False)
            assert np.array_equal(la2, lb2) and np.array_equal(ba2, bb2)
            c2 = A.assign_pairs_costed()
            print(f"  cost blocks: first call {c1}, second {c2}", flush=True)
            assert c2 <= c1
            if wl["S"] > m:
                assert c2 < c1


def test_symbolic_checkpoint_and_errors(d2, protein1, tmp_path):
    """A checkpoint of a symbolic run restores the centroid symbols and the
    plan cache (the continuation is bitwise the uninterrupted one); the
    vector-only calls are refused with D2_EINVAL and symbols out of range
    are rejected."""
    wl = protein1
    K, m = wl["K"], wl["m"]
    lab = wl["classes"].astype(np.int32)
    csym, Wc = symbol_init_centroids(wl, lab, K, m)
    path = str(tmp_path / "sym.ckpt")

    def run(ctx, rounds):
        out = None
        for _ in range(rounds):
            ctx.assign(iters=40)
            ctx.barycenter(iters=30, init=d2.D2_INIT_CACHED)
            out = ctx.centroids_get()[1], ctx.labels_get()
        return out

    with _ctx(d2, wl, "f32") as A, _ctx(d2, wl, "f32") as B:
        for ctx in (A, B):
            ctx.centroids_set_symbolic(csym, Wc)
            ctx.labels_set(lab)
            ctx.barycenter(iters=30, init=d2.D2_INIT_PRODUCT)
        run(A, 2)
        A.checkpoint_save(path)
        wa, la = run(A, 2)
        run(B, 2)
        B.centroids_set_symbolic((csym + 1) % wl["S"], Wc)  # clobbered
        B.checkpoint_load(path)
        Xb, _ = B.centroids_get()
        assert np.array_equal(Xb[:, :, 0], csym.astype(np.float64))
        wb, lb = run(B, 2)
        assert np.array_equal(wa, wb) and np.array_equal(la, lb)
        for call in (lambda: A.centroids_set(np.zeros((K, m, 1)), Wc),
                     lambda: A.support_update(),
                     lambda: A.centroids_init(np.arange(K), m),
                     lambda: A.centroids_set_symbolic(csym + wl["S"], Wc)):
            with pytest.raises(d2.D2Error) as e:
                call()
            assert e.value.status == d2.D2_EINVAL
        bad = wl["sym"].copy()
        bad[5] = wl["S"]
        with pytest.raises(d2.D2Error) as e:
            A.load_instances_symbolic(wl["offsets"], bad, wl["W"], wl["D"])
        assert e.value.status == d2.D2_EINVAL and "instance" in str(e.value)

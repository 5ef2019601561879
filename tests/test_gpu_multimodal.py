"""Multi-modal instances on the GPU (Sec. 5: an instance is an array of
distributions; the assignment distance sums the modalities' squared
distances, and each modality's centroids are updated separately) against
the FP64 oracle, through the C ABI.  Bars: labels equal except at oracle
margins below 1e-5, minimal summed distances within 1e-5 relative (FP32) /
1e-10 (FP64); the per-modality centroid updates as in test_gpu_parity."""
import numpy as np
import pytest

import oracle
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


def _check_labels(lab_g, best_g, lab_o, best_o, tot, dtype, tag):
    srt = np.sort(tot, axis=1)
    margin = (srt[:, 1] - srt[:, 0]) / srt[:, 0]
    ok = (lab_g == lab_o) | (margin < 1e-5)
    r = _rel(best_g, best_o)
    print(f"  {tag} {dtype}: distance rel {r:.3g}, "
          f"{int((lab_g != lab_o).sum())} label differences "
          f"({int((~ok).sum())} outside near-ties)", flush=True)
    assert r < (1e-10 if dtype == "f64" else 1e-5)
    assert ok.all()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_protein_ngram_modalities(d2, dtype):
    """Amino-acid and tripeptide histograms of the same sequences: the
    summed assignment against the oracle, the labels shared by both
    modality contexts, then each modality's centroid update on the
    oracle's labels against the oracle."""
    print(f"[multi-modal protein 1+3-gram {dtype}]", flush=True)
    wl = make_workload("protein_g13_n10742_k10", N=900)
    mods, K = wl["modalities"], wl["K"]
    lab0 = wl["classes"].astype(np.int32)
    rng = np.random.Generator(np.random.PCG64(8))
    cents = []
    for mod, m in zip(mods, wl["m"]):
        csym, _ = symbol_init_centroids(mod, lab0, K, m)
        cents.append((csym, rng.dirichlet(np.ones(m), size=K)))
    dists = [oracle.assign_sym(mod, cs, wc, T=60, want_dist=True)[2]
             for mod, (cs, wc) in zip(mods, cents)]
    lab_o, best_o, tot = oracle.assign_multi(dists)
    ctxs = []
    try:
        for mod, (cs, wc) in zip(mods, cents):
            ctx = d2.D2Context(0, dtype)
            ctxs.append(ctx)
            ctx.load_instances_symbolic(mod["offsets"], mod["sym"], mod["W"],
                                        mod["D"])
            ctx.centroids_set_symbolic(cs, wc)
        lab_g, best_g, nch = d2.assign_multi(ctxs, iters=60)
        assert nch == len(lab_g)
        _check_labels(lab_g, best_g, lab_o, best_o, tot, dtype, "1+3-gram")
        for ctx in ctxs:
            assert np.array_equal(ctx.labels_get(), lab_g)
        # each modality's centroid update on the oracle's labels
        T = 40
        for mod, (cs, wc), ctx in zip(mods, cents, ctxs):
            ctx.labels_set(lab_o)
            ctx.barycenter(iters=T, init=d2.D2_INIT_PRODUCT)
            g_tr, _ = ctx.objective(T)
            _, Wg = ctx.centroids_get()
            for c in range(K):
                mem = np.nonzero(lab_o == c)[0]
                if len(mem) == 0:
                    continue
                out = oracle.barycenter_sym(mod, mem, cs[c], wc[c], T=T)
                tol = 1e-10 if dtype == "f64" else 1e-5
                assert _rel(g_tr[:, c], out["ftrace"]) < tol
                assert np.abs(Wg[c] - out["w"]).max() < tol
    finally:
        for ctx in ctxs:
            ctx.close()


def test_vector_and_symbol_modalities_and_cluster_loop(d2):
    """A vector modality (3-d Gaussian-mixture supports) beside a symbolic
    one: the summed assignment against the oracle; then the multi-modal
    clustering loop runs rounds, reports its records, and two runs from the
    same start agree bitwise."""
    print("[multi-modal vector + symbol]", flush=True)
    N, K = 800, 6
    wa = make_workload("gmm_d3_n65536_k16", N=N)
    wb = make_workload("protein_g1_n10742_k10", N=N)
    mem = pick_init_members(wa["offsets"], K, 8, 31)
    Xa, Wa = oracle.init_centroids(wa, mem, 8)
    cs, _ = symbol_init_centroids(wb, wb["classes"] % K, K, 20)
    rng = np.random.Generator(np.random.PCG64(12))
    Wb = rng.dirichlet(np.ones(20), size=K)
    da = oracle.assign(wa, Xa, Wa, T=60, want_dist=True)[2]
    db = oracle.assign_sym(wb, cs, Wb, T=60, want_dist=True)[2]
    lab_o, best_o, tot = oracle.assign_multi([da, db])

    def contexts():
        A = d2.D2Context(0, "f32")
        A.load_instances(wa["offsets"], wa["X"], wa["W"])
        A.centroids_set(Xa, Wa)
        B = d2.D2Context(0, "f32")
        B.load_instances_symbolic(wb["offsets"], wb["sym"], wb["W"], wb["D"])
        B.centroids_set_symbolic(cs, Wb)
        return [A, B]

    runs = []
    for rep in range(2):
        ctxs = contexts()
        try:
            lab_g, best_g, _ = d2.assign_multi(ctxs, iters=60)
            if rep == 0:
                _check_labels(lab_g, best_g, lab_o, best_o, tot, "f32",
                              "vector+symbol")
            recs = d2.cluster_multi(ctxs, rounds=3, iters=30, assign_iters=60)
            assert [r["round"] for r in recs] == [0, 1, 2]
            assert all(np.isfinite(r["assign_obj"]) for r in recs)
            runs.append((ctxs[0].labels_get(), ctxs[0].centroids_get(),
                         ctxs[1].centroids_get()))
        finally:
            for ctx in ctxs:
                ctx.close()
    (l0, a0, b0), (l1, a1, b1) = runs
    assert np.array_equal(l0, l1)
    for x, y in zip(a0 + b0, a1 + b1):
        assert np.array_equal(x, y)

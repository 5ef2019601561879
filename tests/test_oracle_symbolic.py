"""Pins of the oracle's symbolic-support and multi-modal functions (Sec. 5:
supports drawn from a finite symbol set with a given symbol-to-symbol
dissimilarity, the support step skipped; instances made of several
distributions whose squared distances add in the assignment).

Each pin checks the oracle against something it does not compute itself:
the Euclidean path it reduces to on embedded symbols, exact transport LPs
(HiGHS), the full-batch LP barycenter at fixed support, and brute force."""
import numpy as np
import pytest
from scipy.optimize import linprog

from synth.generators import protein_symbol_workload


def _rand_sym_workload(rng, N, S, mk_max, asym=False):
    sizes = rng.integers(1, mk_max + 1, size=N)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    sym = np.concatenate([rng.choice(S, size=s, replace=False)
                          for s in sizes]).astype(np.int32)
    W = np.concatenate([rng.dirichlet(np.ones(s)) for s in sizes])
    if asym:
        D = rng.random((S, S)) * 2.0
    else:
        E = rng.standard_normal((S, 3))
        D = ((E[:, None, :] - E[None, :, :]) ** 2).sum(-1)
    return {"offsets": off, "sym": sym, "W": W, "D": D, "S": S}


def _lp_w2(C, w, wy):
    """min <C, P> over couplings with row sums w and column sums wy."""
    m, mk = C.shape
    A = []
    for i in range(m):
        r = np.zeros((m, mk)); r[i, :] = 1.0; A.append(r.ravel())
    for j in range(mk):
        r = np.zeros((m, mk)); r[:, j] = 1.0; A.append(r.ravel())
    res = linprog(C.ravel(), A_eq=np.array(A), b_eq=np.concatenate([w, wy]),
                  bounds=(0, None), method="highs")
    assert res.status == 0
    return res.fun


def test_symbolic_run_equals_euclidean_run_on_embedded_symbols(oracle_mod):
    """With D the squared Euclidean distances of symbol embeddings e_a, the
    symbolic barycenter is the Euclidean one with support points e_sym at
    fixed support: same rho, objective trace, weights and plans."""
    rng = np.random.default_rng(11)
    S, d = 9, 3
    E = rng.standard_normal((S, d))
    D = np.array([[sum((E[a, t] - E[b, t]) ** 2 for t in range(d))
                   for b in range(S)] for a in range(S)])
    wl = _rand_sym_workload(rng, 12, S, 5)
    wl["D"] = D
    xsym = np.array([0, 3, 5, 8], dtype=np.int32)
    w0 = np.full(4, 0.25)
    mem = np.arange(12)
    a = oracle_mod.barycenter_sym(wl, mem, xsym, w0, T=60)
    wle = {"offsets": wl["offsets"], "X": E[wl["sym"]], "W": wl["W"]}
    b = oracle_mod.barycenter(wle, mem, E[xsym], w0, T=60, tau=10 ** 6)
    assert abs(a["rho"] - b["rho"]) <= 1e-12 * b["rho"]
    assert np.allclose(a["ftrace"], b["ftrace"], rtol=1e-11, atol=0)
    assert np.allclose(a["w"], b["w"], rtol=0, atol=1e-12)
    for A_, B_ in ((a["plans"].P1, b["plans"].P1), (a["plans"].P2, b["plans"].P2),
                   (a["plans"].L, b["plans"].L)):
        assert np.allclose(A_, B_, rtol=0, atol=1e-12)


@pytest.mark.parametrize("m,mk", [(3, 4), (4, 6), (5, 5)])
def test_symbolic_transport_value_converges_to_lp_of_the_gathered_cost(
        oracle_mod, m, mk):
    """The assignment distance over symbols with an asymmetric table: the
    transport value for the block C_ij = D[x_i, y_j] tends to that block's
    LP optimum (T = 5000, 1e-4 relative), and the transposed reading
    D[y_j, x_i] has a different optimum (so an orientation slip fails)."""
    rng = np.random.default_rng(20 + m)
    S = 12
    differs = 0
    for _ in range(4):
        wl = _rand_sym_workload(rng, 1, S, mk, asym=True)
        wl["offsets"] = np.array([0, mk], dtype=np.int64)
        wl["sym"] = rng.choice(S, size=mk, replace=False).astype(np.int32)
        wl["W"] = rng.dirichlet(np.ones(mk))
        xsym = rng.choice(S, size=m, replace=False).astype(np.int32)
        w = rng.dirichlet(np.ones(m))
        C = wl["D"][xsym][:, wl["sym"]]
        ex = _lp_w2(C, w, wl["W"])
        _, best, dist = oracle_mod.assign_sym(wl, xsym[None, :], w[None, :],
                                              T=5000, want_dist=True)
        assert abs(best[0] - ex) <= 1e-4 * ex + 1e-12, (best[0], ex)
        assert dist[0, 0] == best[0]
        v = oracle_mod.ot_cost(C, w, wl["W"], T=5000)
        assert abs(v - best[0]) <= 1e-12 * ex
        ext = _lp_w2(wl["D"][wl["sym"]][:, xsym].T, w, wl["W"])
        differs += abs(ext - ex) > 1e-2 * ex
    assert differs > 0


def _fullbatch_lp_cost(blocks, W, off, m):
    """Eq. (fullbatch-lp) with given cost blocks (m x m_k each)."""
    N = len(blocks)
    nv = m + sum(C.size for C in blocks)
    c = np.zeros(nv)
    rows, rhs = [], []
    col = m
    for k, C in enumerate(blocks):
        mk = C.shape[1]
        c[col:col + m * mk] = C.reshape(-1)
        for i in range(m):
            r = np.zeros(nv); r[col + i * mk:col + (i + 1) * mk] = 1.0
            r[i] = -1.0; rows.append(r); rhs.append(0.0)
        for j in range(mk):
            r = np.zeros(nv); r[col + j:col + m * mk:mk] = 1.0
            rows.append(r); rhs.append(W[off[k] + j])
        col += m * mk
    r = np.zeros(nv); r[:m] = 1.0; rows.append(r); rhs.append(1.0)
    res = linprog(c, A_eq=np.array(rows), b_eq=np.array(rhs), bounds=(0, None),
                  method="highs")
    assert res.status == 0
    return res.fun / N


def test_symbolic_barycenter_near_full_lp(oracle_mod):
    """Symbolic supports are a fixed-support barycenter: the B-ADMM weights'
    exact objective (LP per member) is >= the full-batch LP optimum (hard)
    and within a few % of it (Table 1 reports 0.2-0.6 %)."""
    rng = np.random.default_rng(5)
    gaps = []
    for trial in range(5):
        S, m = 8, 4
        wl = _rand_sym_workload(rng, 6, S, 4, asym=(trial % 2 == 1))
        xsym = rng.choice(S, size=m, replace=False).astype(np.int32)
        out = oracle_mod.barycenter_sym(wl, np.arange(6), xsym,
                                        np.full(m, 1.0 / m), T=2000)
        off = wl["offsets"]
        blocks = [wl["D"][xsym][:, wl["sym"][off[k]:off[k + 1]]]
                  for k in range(6)]
        lp = _fullbatch_lp_cost(blocks, wl["W"], off, m)
        ft = np.mean([_lp_w2(C, out["w"], wl["W"][off[k]:off[k + 1]])
                      for k, C in enumerate(blocks)])
        assert ft >= lp - 1e-9
        gaps.append((ft - lp) / lp)
    assert np.median(gaps) < 0.01 and max(gaps) < 0.03, gaps


def test_symbolic_barycenter_invariants(oracle_mod):
    """Every member's Pi1 has the instance weights as column sums and Pi2
    the centroid weights as row sums; Lambda sums to 0 per member."""
    wl = protein_symbol_workload(6001, 60, gram=1)
    xsym = np.arange(20, dtype=np.int32)
    out = oracle_mod.barycenter_sym(wl, np.arange(60), xsym,
                                    np.full(20, 0.05), T=40)
    off = wl["offsets"]
    for k in range(60):
        P1, P2, L = out["plans"].block(off, k)
        assert np.allclose(P1.sum(0), wl["W"][off[k]:off[k + 1]], atol=1e-12)
        assert np.allclose(P2.sum(1), out["w"], atol=1e-12)
        assert abs(L.sum()) < 1e-12


def test_assign_sym_is_argmin_of_pair_values(oracle_mod):
    """Labels are the argmin over centroids of the pair values computed one
    by one on the gathered blocks, ties to the lowest index (a duplicated
    centroid ties exactly)."""
    rng = np.random.default_rng(9)
    wl = _rand_sym_workload(rng, 30, 10, 6, asym=True)
    Xs = np.stack([rng.choice(10, size=4, replace=False) for _ in range(5)])
    Xs[4] = Xs[1]
    Wc = rng.dirichlet(np.ones(4), size=5)
    Wc[4] = Wc[1]
    lab, best, dist = oracle_mod.assign_sym(wl, Xs, Wc, T=50, want_dist=True)
    off = wl["offsets"]
    for k in range(30):
        y = wl["sym"][off[k]:off[k + 1]]
        vals = [oracle_mod.ot_cost(wl["D"][Xs[c]][:, y], Wc[c],
                                   wl["W"][off[k]:off[k + 1]], T=50)
                for c in range(5)]
        assert np.array_equal(dist[k], vals)
        assert lab[k] == int(np.argmin(vals)) and lab[k] != 4
        assert best[k] == min(vals)


def test_assign_multi_sums_the_modalities(oracle_mod):
    """Multi-modal assignment (Sec. 5): the combined distance is the sum of
    the modalities' distances.  Brute force per instance; one modality
    gives the single-modality labels; a modality repeated twice doubles
    the distances and keeps the labels."""
    rng = np.random.default_rng(4)
    d1 = rng.random((40, 6))
    d2 = rng.random((40, 6))
    d2[3] = d2[3, 0]  # all tied: lowest index wins
    d1[3] = 0.0
    lab, best, tot = oracle_mod.assign_multi([d1, d2])
    for k in range(40):
        s = [d1[k, c] + d2[k, c] for c in range(6)]
        c0 = min(range(6), key=lambda c: (s[c], c))
        assert lab[k] == c0 and best[k] == s[c0]
    assert lab[3] == 0
    l1, b1, _ = oracle_mod.assign_multi([d1])
    assert np.array_equal(l1, np.argmin(d1, axis=1))
    l2, b2, _ = oracle_mod.assign_multi([d1, d1])
    assert np.array_equal(l2, l1) and np.array_equal(b2, 2 * b1)

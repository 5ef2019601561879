"""Seeded synthetic discrete-distribution workloads.

This module only draws random inputs: ragged discrete distributions
(support points + probability weights) stored in the concatenated layout of
the paper's notation (Sec. 2: X = (x^(1), ..., x^(N)) in R^{d x n},
n = sum_k m_k), plus initial-centroid member choices.  It contains none of
the method's arithmetic and is shared by the FP64 oracle, the tests and the
benchmark so that both sides consume bit-identical inputs.

Layout of a workload (a plain dict of numpy arrays):
  offsets : int64[N+1]   instance k owns support rows offsets[k]:offsets[k+1]
  X       : float64[n, d] support points, row-major (one row per point)
  W       : float64[n]    weights, each instance's weights sum to 1
  classes : int64[N]      latent generating class (for information only)
The paper's datasets (pixel-colour distributions, 20newsgroups word-vector
bags, the Table 2 synthetic set) are not available; these generators stand
in for them with the shapes listed in each function.

Draw order (all from one numpy Generator(PCG64(seed))), per workload:
  1. mixture/topic centres, 2. per-instance support sizes, 3. per-instance
  latent class, 4. per-point component choice, 5. per-point noise,
  6. per-point weight draws.  Changing any of these changes every later draw.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "WORKLOADS",
    "make_workload",
    "gaussian_mixture_workload",
    "topic_sphere_workload",
    "pick_init_members",
    "round_to_bf16",
    "warmstart_clusters",
    "deepsets_init_params",
    "protein_symbol_workload",
    "symbol_init_centroids",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _ragged_dirichlet(rng, sizes, alpha):
    """Dirichlet(alpha * 1_{m_k}) draws for every instance, concatenated."""
    n = int(sizes.sum())
    g = rng.gamma(alpha, 1.0, size=n)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    # guard against an all-underflowed instance (possible for tiny alpha)
    sums = np.add.reduceat(g, offs[:-1])
    bad = sums <= 0.0
    if np.any(bad):
        for k in np.nonzero(bad)[0]:
            g[offs[k]:offs[k + 1]] = 1.0
        sums = np.add.reduceat(g, offs[:-1])
    return g / np.repeat(sums, sizes)


def gaussian_mixture_workload(seed, N, d, mk_lo, mk_hi, n_comp, n_class,
                              sigma, alpha, fixed_mk=None):
    """Instances whose support points come from an isotropic Gaussian mixture.

    Component means ~ U[0,1]^d.  Latent class l owns the contiguous block of
    n_comp // n_class components; an instance picks its class uniformly, and
    each of its points picks one of the class's components uniformly, then
    x = mean + sigma * N(0, I_d).  Support sizes are uniform integers in
    [mk_lo, mk_hi] (or all equal to fixed_mk).  Weights ~ Dirichlet(alpha).
    """
    rng = _rng(seed)
    means = rng.uniform(0.0, 1.0, size=(n_comp, d))
    if fixed_mk is not None:
        sizes = np.full(N, int(fixed_mk), dtype=np.int64)
    else:
        sizes = rng.integers(mk_lo, mk_hi + 1, size=N).astype(np.int64)
    classes = rng.integers(0, n_class, size=N).astype(np.int64)
    per_class = n_comp // n_class
    n = int(sizes.sum())
    pt_class = np.repeat(classes, sizes)
    comp = pt_class * per_class + rng.integers(0, per_class, size=n)
    X = means[comp] + sigma * rng.standard_normal(size=(n, d))
    W = _ragged_dirichlet(rng, sizes, alpha)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return {"offsets": offsets, "X": np.ascontiguousarray(X, dtype=np.float64),
            "W": W.astype(np.float64), "classes": classes, "d": d}


def round_to_bf16(a):
    """Round float64 values to the nearest bfloat16 value (ties to even).

    The result is returned as float64 holding exactly representable bf16
    values, so FP64, FP32 and BF16 consumers all see the same numbers.
    """
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16) << np.uint64(16)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _zipf_bounded(rng, a, hi, size):
    """Zipf(a) draws (support 1, 2, ...) redrawn until <= hi."""
    out = rng.zipf(a, size=size).astype(np.int64)
    bad = out > hi
    while np.any(bad):
        out[bad] = rng.zipf(a, size=int(bad.sum()))
        bad = out > hi
    return out


def topic_sphere_workload(seed, N, d=64, n_topic=512, n_class=64, noise=0.3,
                          zipf_a=1.2, mk_base=7, mk_max=64, count_max=1000,
                          bf16=True):
    """Bag-of-word-vector style instances on the unit sphere.

    Topic centres are normalised N(0, I_d) vectors; class l owns topics
    [l*t, (l+1)*t) with t = n_topic // n_class.  A point takes a topic of its
    instance's class uniformly and is normalise(t + (noise/sqrt(d)) N(0,I_d)),
    i.e. about `noise` radians of angular spread.  Support sizes are
    mk_base + Z with Z ~ Zipf(zipf_a) redrawn until the size is <= mk_max;
    weights are Zipf(zipf_a) counts (redrawn until <= count_max), normalised.
    Points are rounded once to bf16 (so every consumer sees the same values).
    """
    rng = _rng(seed)
    topics = rng.standard_normal(size=(n_topic, d))
    topics /= np.linalg.norm(topics, axis=1, keepdims=True)
    sizes = mk_base + _zipf_bounded(rng, zipf_a, mk_max - mk_base, N)
    classes = rng.integers(0, n_class, size=N).astype(np.int64)
    per_class = n_topic // n_class
    n = int(sizes.sum())
    pt_class = np.repeat(classes, sizes)
    top = pt_class * per_class + rng.integers(0, per_class, size=n)
    X = topics[top] + (noise / np.sqrt(d)) * rng.standard_normal(size=(n, d))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    if bf16:
        X = round_to_bf16(X)
    counts = _zipf_bounded(rng, zipf_a, count_max, n).astype(np.float64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    sums = np.add.reduceat(counts, offsets[:-1])
    W = counts / np.repeat(sums, sizes)
    return {"offsets": offsets, "X": np.ascontiguousarray(X, dtype=np.float64),
            "W": W, "classes": classes, "d": d}


def protein_symbol_workload(seed, N, gram=1, n_family=10, len_lo=80,
                            len_hi=400, alpha=0.5, n_amino=20, emb_dim=4,
                            mk_cap=64):
    """n-gram histograms of synthetic protein sequences over a symbol set
    (stand-in for the paper's protein-sequence data: symbolic supports with
    a given symbol-to-symbol dissimilarity, Sec. 5).

    Each sequence belongs to one of n_family families; a family is a
    first-order Markov chain over the n_amino residues (initial
    distribution and transition rows Dirichlet(alpha)).  Sequence lengths
    are uniform in [len_lo, len_hi].  Symbols: gram = 1, the residues
    (S = n_amino); gram = 3, the tripeptides a n_amino^2 + b n_amino + c
    (S = n_amino^3).  An instance is the set of distinct n-grams of its
    sequence with their relative counts, cut to the mk_cap most frequent
    (ties to the smaller symbol) and renormalised.  The dissimilarity table:
    residues get random embeddings e_a ~ N(0, I_emb_dim) and
    D1[a, b] = sum_t (e_a,t - e_b,t)^2 (direct differences); for 3-grams
    D[(a,b,c), (x,y,z)] = D1[a,x] + D1[b,y] + D1[c,z].

    Draw order: 1. embeddings, 2. family initial distributions, 3. family
    transition rows, 4. per-sequence family, 5. per-sequence length,
    6. residues, position by position for all sequences.
    Returns offsets, sym (int32, n), W, D (S x S), classes, S."""
    rng = _rng(seed)
    A = n_amino
    emb = rng.standard_normal((A, emb_dim))
    init = rng.dirichlet(np.full(A, alpha), size=n_family)
    trans = rng.dirichlet(np.full(A, alpha), size=(n_family, A))
    fam = rng.integers(0, n_family, size=N)
    lens = rng.integers(len_lo, len_hi + 1, size=N)
    L = int(lens.max())
    seq = np.zeros((N, L), dtype=np.int64)
    cinit = np.cumsum(init, axis=1)
    ctrans = np.cumsum(trans, axis=2)
    u = rng.random(N)
    seq[:, 0] = np.minimum((u[:, None] > cinit[fam]).sum(1), A - 1)
    for t in range(1, L):
        u = rng.random(N)
        rows = ctrans[fam, seq[:, t - 1]]
        seq[:, t] = np.minimum((u[:, None] > rows).sum(1), A - 1)
    D1 = np.zeros((A, A))
    for a in range(A):
        for b in range(A):
            acc = 0.0
            for t in range(emb_dim):
                df = emb[a, t] - emb[b, t]
                acc += df * df
            D1[a, b] = acc
    def modality(gram):
        if gram == 1:
            S = A
            D = D1
        elif gram == 3:
            S = A ** 3
            idx = np.arange(S)
            a, b, c = idx // (A * A), (idx // A) % A, idx % A
            D = D1[a][:, a] + D1[b][:, b] + D1[c][:, c]
        else:
            raise ValueError("gram must be 1 or 3")
        syms, ws, sizes = [], [], []
        for k in range(N):
            s_ = seq[k, :lens[k]]
            if gram == 3:
                s_ = s_[:-2] * (A * A) + s_[1:-1] * A + s_[2:]
            vals, cnt = np.unique(s_, return_counts=True)
            order = np.lexsort((vals, -cnt))[:mk_cap]
            vals, cnt = vals[order], cnt[order].astype(np.float64)
            syms.append(vals)
            ws.append(cnt / cnt.sum())
            sizes.append(len(vals))
        offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        return {"offsets": offsets,
                "sym": np.concatenate(syms).astype(np.int32),
                "W": np.concatenate(ws), "D": np.ascontiguousarray(D),
                "classes": fam.astype(np.int64), "S": S}

    if isinstance(gram, (tuple, list)):
        # one instance = the histograms of several n-gram orders of the same
        # sequence (multi-modal instances, Sec. 5)
        return {"modalities": [modality(g) for g in gram],
                "classes": fam.astype(np.int64)}
    return modality(gram)


def symbol_init_centroids(wl, labels, K, m):
    """Initial symbolic centroids: for cluster c the m symbols carrying the
    most weight summed over its members (ties to the smaller symbol;
    clusters with fewer distinct symbols are filled up in the same order
    over all instances), with uniform weights 1/m.  Returns csym (K x m,
    int32) and Wc (K x m)."""
    off, sym, W = wl["offsets"], wl["sym"], wl["W"]
    S = wl["S"]
    inst = np.repeat(np.arange(len(off) - 1), np.diff(off))
    tot_all = np.bincount(sym, weights=W, minlength=S)
    rank_all = np.lexsort((np.arange(S), -tot_all))
    csym = np.zeros((K, m), dtype=np.int32)
    for c in range(K):
        sel = labels[inst] == c
        tot = np.bincount(sym[sel], weights=W[sel], minlength=S)
        order = np.lexsort((np.arange(S), -tot))
        chosen = [int(v) for v in order if tot[v] > 0][:m]
        for v in rank_all:
            if len(chosen) == m:
                break
            if int(v) not in chosen:
                chosen.append(int(v))
        csym[c] = chosen
    return csym, np.full((K, m), 1.0 / m)


# The paper's workloads as parameter sets.  N can be overridden to get a
# smaller instance of the same distribution (tests use this).
WORKLOADS = {
    # pixel-colour-like, one cluster (Sec. 4 pilot shapes): d=3, m_k=8
    "gmm_d3_n256": dict(kind="gmm", N=256, d=3, mk_lo=8, mk_hi=8, n_comp=4,
                        n_class=1, sigma=0.1, alpha=1.0, K=1, m=8, T=200,
                        rounds=0, seed=1000),
    # full clustering loop, colour-like: d=3, m_k in [4,16]
    "gmm_d3_n65536_k16": dict(kind="gmm", N=65536, d=3, mk_lo=4, mk_hi=16,
                              n_comp=32, n_class=16, sigma=0.05, alpha=0.5,
                              K=16, m=16, T=100, rounds=10, seed=2000),
    # word-vector bags: d=64, heavy-tailed m_k in [8,64]
    "topic_d64_n200000_k64": dict(kind="topic", N=200000, d=64, K=64, m=32,
                                  T=100, rounds=1, seed=3000),
    # Table 2 synthetic scale: d=16, m_k in [4,32]
    "gmm_d16_n2000000_k256": dict(kind="gmm", N=2000000, d=16, mk_lo=4,
                                  mk_hi=32, n_comp=1024, n_class=256,
                                  sigma=0.1, alpha=1.0, K=256, m=16, T=50,
                                  rounds=5, seed=4000),
    # protein-sequence-like symbolic supports (Sec. 5): amino-acid
    # histograms (S = 20, m = 20) and tripeptide histograms (S = 8000,
    # m = 32), N = 10,742 sequences, K = 10 families
    "protein_g1_n10742_k10": dict(kind="protein", N=10742, gram=1, K=10,
                                  m=20, T=100, rounds=5, seed=6000),
    "protein_g3_n10742_k10": dict(kind="protein", N=10742, gram=3, K=10,
                                  m=32, T=100, rounds=5, seed=6100),
    # multi-modal instances (Sec. 5): each sequence's amino-acid and
    # tripeptide histograms, centroid sizes 20 and 32
    "protein_g13_n10742_k10": dict(kind="protein", N=10742, gram=(1, 3),
                                   K=10, m=(20, 32), T=100, rounds=5,
                                   seed=6200),
}


def make_workload(name, seed=None, N=None, replicate=0):
    """Build a named workload; seed defaults to the workload's own seed +
    replicate."""
    p = dict(WORKLOADS[name])
    if seed is None:
        seed = p["seed"] + int(replicate)
    if N is None:
        N = p["N"]
    if p["kind"] == "gmm":
        wl = gaussian_mixture_workload(seed, N, p["d"], p["mk_lo"], p["mk_hi"],
                                       p["n_comp"], p["n_class"], p["sigma"],
                                       p["alpha"])
    elif p["kind"] == "protein":
        wl = protein_symbol_workload(seed, N, gram=p["gram"])
    else:
        wl = topic_sphere_workload(seed, N, d=p["d"])
    wl.update(K=p["K"], m=p["m"], T=p["T"], rounds=p["rounds"], name=name,
              seed=seed)
    return wl


def pick_init_members(offsets, K, m, seed):
    """Choose K distinct instances with at least m support points.

    These are the random members that seed the K initial centroids (the
    paper initialises a centroid from a randomly chosen cluster member with at
    least m support points, Sec. 5).  Returned as int64[K] instance indices.
    """
    sizes = np.diff(np.asarray(offsets))
    elig = np.nonzero(sizes >= m)[0]
    if len(elig) < K:
        raise ValueError(f"only {len(elig)} instances have >= {m} points; need {K}")
    rng = _rng(int(seed) + 7777777)
    return np.sort(rng.choice(elig, size=K, replace=False)).astype(np.int64)


def _loguniform_int(rng, lo, hi, size):
    return np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi + 1), size=size))
                    ).astype(np.int64).clip(lo, hi)


def warmstart_clusters(family, n_clusters, seed, nc_lo=64, nc_hi=2048,
                       contam_max=0.2):
    """Whole clusters for training / evaluating the learned warm start.

    Every cluster is its own small world, so that a network has to infer
    the barycenter from the members rather than memorise a fixed set of
    classes.  Cluster c has N_c ~ log-uniform{nc_lo..nc_hi} member
    instances; a fraction f_c ~ U[0, contam_max] of them are contaminated
    (drawn from other classes).  Instances of a cluster are stored
    contiguously; `labels` gives each instance's cluster.  The first member
    of every cluster has the maximal support size, so that a member with at
    least m points exists for the plain initial centroid.

    family "gmm3" (the colour-like family of gmm_d3_n65536_k16): d = 3, m_k ~ U{4..16};
      own class = 2 Gaussian components with means ~ U[0,1]^3, sigma 0.05;
      contamination = 2 further components; weights Dirichlet(0.5).
    family "topic64" (the word-vector-like family of
    topic_d64_n200000_k64): d = 64,
      m_k = 7 + Zipf(1.2) <= 64; own class = 8 unit topic vectors,
      contamination = 8 more; points normalise(t + (0.3/8) N(0, I)),
      rounded to bf16; weights Zipf(1.2) counts <= 1000.

    Draw order: N_c, f_c, class centres, contamination flags, support
    sizes, component choice, noise, weights.
    """
    rng = _rng(seed)
    C = int(n_clusters)
    nc = _loguniform_int(rng, nc_lo, nc_hi, C)
    frac = rng.uniform(0.0, contam_max, size=C)
    N = int(nc.sum())
    labels = np.repeat(np.arange(C, dtype=np.int32), nc)
    first = np.concatenate([[0], np.cumsum(nc)[:-1]])
    if family == "gmm3":
        d, ncomp, mk_lo, mk_hi = 3, 2, 4, 16
        centres = rng.uniform(0.0, 1.0, size=(C, 2 * ncomp, d))
    elif family == "topic64":
        d, ncomp, mk_hi = 64, 8, 64
        centres = rng.standard_normal(size=(C, 2 * ncomp, d))
        centres /= np.linalg.norm(centres, axis=2, keepdims=True)
    else:
        raise ValueError(family)
    contam = rng.uniform(size=N) < frac[labels]
    if family == "gmm3":
        sizes = rng.integers(mk_lo, mk_hi + 1, size=N).astype(np.int64)
    else:
        sizes = 7 + _zipf_bounded(rng, 1.2, mk_hi - 7, N)
    sizes[first] = mk_hi
    contam[first] = False
    n = int(sizes.sum())
    pt_cl = np.repeat(labels, sizes)
    pt_off = np.repeat(contam.astype(np.int64) * ncomp, sizes)
    comp = pt_off + rng.integers(0, ncomp, size=n)
    mean = centres[pt_cl, comp]
    if family == "gmm3":
        X = mean + 0.05 * rng.standard_normal(size=(n, d))
        W = _ragged_dirichlet(rng, sizes, 0.5)
    else:
        X = mean + (0.3 / np.sqrt(d)) * rng.standard_normal(size=(n, d))
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        X = round_to_bf16(X)
        counts = _zipf_bounded(rng, 1.2, 1000, n).astype(np.float64)
        offs = np.concatenate([[0], np.cumsum(sizes)])
        W = counts / np.repeat(np.add.reduceat(counts, offs[:-1]), sizes)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return {"offsets": offsets, "X": np.ascontiguousarray(X, dtype=np.float64),
            "W": W.astype(np.float64), "labels": labels, "K": C, "d": d,
            "first": first.astype(np.int64), "family": family, "seed": seed}


def deepsets_init_params(m, d, H, seed):
    """Initial parameters of the warm-start network (flat float64 vector in
    the order W1 (din x H), b1, W2, b2, V1, e1, V2, e2, V3 (H x outp), e3,
    din = roundup(d+1, 16), outp = roundup(m(d+1), 32)): He-normal
    matrices, zero biases, zero padding rows / columns."""
    rng = _rng(seed)
    din = (d + 1 + 15) // 16 * 16
    out = m * (d + 1)
    outp = (out + 31) // 32 * 32
    W1 = np.zeros((din, H))
    W1[:d + 1] = rng.standard_normal((d + 1, H)) * np.sqrt(2.0 / (d + 1))
    mats = [rng.standard_normal((H, H)) * np.sqrt(2.0 / H) for _ in range(3)]
    V3 = np.zeros((H, outp))
    V3[:, :out] = rng.standard_normal((H, out)) * np.sqrt(1.0 / H)
    z = np.zeros
    parts = [W1, z(H), mats[0], z(H), mats[1], z(H), mats[2], z(H), V3,
             z(outp)]
    return np.concatenate([q.reshape(-1) for q in parts])

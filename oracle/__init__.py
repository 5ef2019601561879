"""FP64 CPU oracle for the B-ADMM barycenter / D2-clustering hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and
by bench.py's CPU-baseline leg, never by the product package.  It shares no
code with the HIP library (its arithmetic lives in oracle.c, compiled with
gcc; exact transport values come from scipy's HiGHS LP solver).

Functions and the passages they follow (Ye, Wu, Wang, Li, "Fast Discrete
Distribution Clustering Using Wasserstein Barycenter with Sparse Support"):
  cost_block      Sec. 2 notation, item 6 (squared-Euclidean cost matrix)
  ward_merge      Sec. 5, Eq. (merge) (centroid initialisation)
  init_centroids  Sec. 5 (random member, merged down to m points)
  barycenter      Sec. 3.2, Algorithm "Centroid Update with B-ADMM"
  badmm_ot        Sec. 3.2 closed forms with w fixed (the Sec. 4 pilot use)
  assign          Algorithm "D2 Clustering", assignment loop
  barycenter_sym, assign_sym, ot_cost
                  the same over symbolic supports (Sec. 5: a finite symbol
                  set with a given symbol-to-symbol dissimilarity table; the
                  support is fixed, only weights are updated)
  assign_multi    Sec. 5 multi-modal instances: the assignment distance is
                  the sum over modalities
  cluster         Algorithm "D2 Clustering" with the Sec. 5 warm start
  exact_w2        Eq. (primal), solved as an LP (HiGHS)
  f_true          Eq. (centroid): (1/N) sum_k W^2(P, P^(k))
  round_feasible  a plan rounded to exact marginals (Altschuler, Weed and
                  Rigollet 2017, Algorithm 2), so Eq. (badmm_prob)'s cost
                  can be evaluated at a feasible point
  feasible_objective  (1/N) sum_k <C^(k), round(Pi1^(k))>, an upper bound
                  on Eq. (centroid) at the current centroid
The learned warm start (not part of the paper) has its own FP64 reference
in oracle/deepsets.py.
Every function here is pinned by tests/test_oracle_*.py against values that
do not come from this module (LP solves, closed forms, invariants).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.orc_cost_block.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   _f64p, _f64p, _f64p]
    lib.orc_ward_merge.argtypes = [ctypes.c_int, ctypes.c_int, _f64p, _f64p,
                                   ctypes.c_int, _f64p, _f64p]
    lib.orc_ward_merge.restype = ctypes.c_int
    lib.orc_barycenter.argtypes = [
        ctypes.c_int64, _i64p, _i64p, ctypes.c_int, _f64p, _f64p, ctypes.c_int,
        _f64p, _f64p, _u8p, _f64p, _f64p, _f64p, ctypes.c_double, ctypes.c_int,
        ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, _f64p, _f64p,
        _f64p]
    lib.orc_barycenter.restype = ctypes.c_int
    lib.orc_ot.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _f64p,
                           _f64p, _f64p, _f64p, ctypes.c_double, ctypes.c_int,
                           ctypes.c_double, _f64p, _f64p, _f64p]
    lib.orc_ot.restype = ctypes.c_double
    lib.orc_assign.argtypes = [ctypes.c_int64, _i64p, ctypes.c_int, _f64p,
                               _f64p, ctypes.c_int, ctypes.c_int, _f64p, _f64p,
                               ctypes.c_double, ctypes.c_int, ctypes.c_double,
                               _i32p, _f64p, _f64p]
    lib.orc_barycenter_sym.argtypes = [
        ctypes.c_int64, _i64p, _i64p, _i32p, _f64p, ctypes.c_int, _i32p,
        ctypes.c_int, _f64p, _f64p, _u8p, _f64p, _f64p, _f64p,
        ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int, _f64p,
        _f64p, _f64p]
    lib.orc_barycenter_sym.restype = ctypes.c_int
    lib.orc_ot_cost.argtypes = [ctypes.c_int, ctypes.c_int, _f64p, _f64p,
                                _f64p, ctypes.c_double, ctypes.c_int,
                                ctypes.c_double, _f64p, _f64p, _f64p]
    lib.orc_ot_cost.restype = ctypes.c_double
    lib.orc_assign_sym.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p,
                                   ctypes.c_int, ctypes.c_int, _i32p, _f64p,
                                   ctypes.c_int, _f64p, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_double, _i32p,
                                   _f64p, _f64p]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(t: int) -> None:
    _load().orc_set_num_threads(int(t))


def cost_block(x, y):
    """C_ij = ||x_i - y_j||^2 as an (m, mk) array (Sec. 2, item 6)."""
    x, y = _f64(x), _f64(y)
    m, d = x.shape
    mk = y.shape[0]
    out = np.empty(m * mk, dtype=np.float64)
    _load().orc_cost_block(m, mk, d, _p(x, _f64p), _p(y, _f64p), _p(out, _f64p))
    return out.reshape(mk, m).T.copy()


def ward_merge(y, wy, m):
    """Merge a distribution's support greedily down to m points (Eq. merge)."""
    y, wy = _f64(y), _f64(wy)
    mk, d = y.shape
    x = np.empty((m, d)), np.empty(m)
    rc = _load().orc_ward_merge(mk, d, _p(y, _f64p), _p(wy, _f64p), m,
                                _p(x[0], _f64p), _p(x[1], _f64p))
    if rc != 0:
        raise ValueError("ward_merge needs at least m support points")
    return x


def init_centroids(wl, members, m):
    """Centroid c = member members[c] merged down to m points (Sec. 5)."""
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    d = X.shape[1]
    K = len(members)
    Xc = np.empty((K, m, d))
    Wc = np.empty((K, m))
    for c, k in enumerate(members):
        a, b = off[k], off[k + 1]
        Xc[c], Wc[c] = ward_merge(X[a:b], W[a:b], m)
    return Xc, Wc


class Plans:
    """Concatenated m x n plan arrays Pi1, Pi2, Lambda (Sec. 2, item 9)."""

    def __init__(self, m, n):
        self.m = m
        self.P1 = np.zeros(m * n)
        self.P2 = np.zeros(m * n)
        self.L = np.zeros(m * n)

    def block(self, off, k):
        """(Pi1, Pi2, Lambda) of instance k as (m, m_k) arrays."""
        m = self.m
        a, b = m * off[k], m * off[k + 1]
        mk = off[k + 1] - off[k]
        return tuple(A[a:b].reshape(mk, m).T.copy()
                     for A in (self.P1, self.P2, self.L))


def barycenter(wl, members, x, w, plans=None, warm=None, rho0=2.0, tau=10,
               T=100, eps=1e-16, rule=1, xplan=0):
    """B-ADMM barycenter of the instances `members` (Algorithm B-ADMM).

    Returns dict(x, w, ftrace, rtrace, rho, plans); rtrace[n] is the
    residual (1/N) sum_k sum_ij |Pi1 - Pi2| after iteration n.  `plans` (a Plans) is updated in
    place; warm[q] != 0 starts member q from its cached Pi2 in plans.P2.
    """
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    m, d = np.asarray(x).shape
    n = int(off[-1])
    if plans is None:
        plans = Plans(m, n)
    mem = np.ascontiguousarray(members, dtype=np.int64)
    xo, wo = _f64(x).copy(), _f64(w).copy()
    wa = None if warm is None else np.ascontiguousarray(warm, dtype=np.uint8)
    ftr = np.zeros(max(T, 1))
    rtr = np.zeros(max(T, 1))
    rho = np.zeros(1)
    rc = _load().orc_barycenter(
        len(mem), _p(mem, _i64p), _p(off, _i64p), d, _p(X, _f64p), _p(W, _f64p),
        m, _p(xo, _f64p), _p(wo, _f64p), _p(wa, _u8p), _p(plans.P1, _f64p),
        _p(plans.P2, _f64p), _p(plans.L, _f64p), float(rho0), int(tau), int(T),
        float(eps), int(rule), int(xplan), _p(ftr, _f64p), _p(rtr, _f64p),
        _p(rho, _f64p))
    if rc != 0:
        raise ValueError("orc_barycenter: bad arguments")
    return {"x": xo, "w": wo, "ftrace": ftr[:T], "rtrace": rtr[:T],
            "rho": float(rho[0]), "plans": plans}


def badmm_ot(x, w, y, wy, rho0=2.0, T=100, eps=1e-16, return_plans=False):
    """B-ADMM transport value <C, Pi1> between (w, x) and (wy, y)."""
    x, w, y, wy = _f64(x), _f64(w), _f64(y), _f64(wy)
    m, d = x.shape
    mk = y.shape[0]
    bufs = [np.empty(m * mk) for _ in range(3)] if return_plans else [None] * 3
    v = _load().orc_ot(m, mk, d, _p(x, _f64p), _p(w, _f64p), _p(y, _f64p),
                       _p(wy, _f64p), float(rho0), int(T), float(eps),
                       *[_p(b, _f64p) for b in bufs])
    if not return_plans:
        return v
    return v, tuple(b.reshape(mk, m).T.copy() for b in bufs)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def barycenter_sym(wl, members, xsym, w, plans=None, warm=None, rho0=2.0,
                   T=100, eps=1e-16, rule=1):
    """B-ADMM barycenter over symbolic supports (Sec. 5): `wl` holds
    offsets, the instances' symbols `sym` (n), weights `W` and the S x S
    table `D`; the centroid's symbols xsym (m) stay fixed.  Returns dict(w,
    ftrace, rtrace, rho, plans) as barycenter does."""
    off, sym, W, D = wl["offsets"], _i32(wl["sym"]), wl["W"], _f64(wl["D"])
    S = D.shape[0]
    xs_ = _i32(xsym)
    m = len(xs_)
    n = int(off[-1])
    if plans is None:
        plans = Plans(m, n)
    mem = np.ascontiguousarray(members, dtype=np.int64)
    wo = _f64(w).copy()
    wa = None if warm is None else np.ascontiguousarray(warm, dtype=np.uint8)
    ftr = np.zeros(max(T, 1))
    rtr = np.zeros(max(T, 1))
    rho = np.zeros(1)
    rc = _load().orc_barycenter_sym(
        len(mem), _p(mem, _i64p), _p(off, _i64p), _p(sym, _i32p),
        _p(W, _f64p), m, _p(xs_, _i32p), S, _p(D, _f64p), _p(wo, _f64p),
        _p(wa, _u8p), _p(plans.P1, _f64p), _p(plans.P2, _f64p),
        _p(plans.L, _f64p), float(rho0), int(T), float(eps), int(rule),
        _p(ftr, _f64p), _p(rtr, _f64p), _p(rho, _f64p))
    if rc != 0:
        raise ValueError("orc_barycenter_sym: bad arguments")
    return {"w": wo, "ftrace": ftr[:T], "rtrace": rtr[:T],
            "rho": float(rho[0]), "plans": plans}


def ot_cost(C, w, wy, rho0=2.0, T=100, eps=1e-16):
    """B-ADMM transport value <C, Pi1> for a given (m, mk) cost block."""
    C = _f64(C)
    m, mk = C.shape
    Ccm = np.ascontiguousarray(C.T).ravel()  # column-major m x mk
    return _load().orc_ot_cost(m, mk, _p(Ccm, _f64p), _p(_f64(w), _f64p),
                               _p(_f64(wy), _f64p), float(rho0), int(T),
                               float(eps), None, None, None)


def assign_sym(wl, Xsym, Wc, rho0=2.0, T=100, eps=1e-16, want_dist=False):
    """Symbolic assignment: labels, best D and (optionally) all D (N x K),
    centroid c having symbols Xsym[c] (m) and weights Wc[c]."""
    off, sym, W, D = wl["offsets"], _i32(wl["sym"]), wl["W"], _f64(wl["D"])
    N = len(off) - 1
    Xsym, Wc = _i32(Xsym), _f64(Wc)
    K, m = Xsym.shape
    lab = np.empty(N, dtype=np.int32)
    best = np.empty(N)
    dist = np.empty(N * K) if want_dist else None
    _load().orc_assign_sym(N, _p(off, _i64p), _p(sym, _i32p), _p(W, _f64p),
                           K, m, _p(Xsym, _i32p), _p(Wc, _f64p), D.shape[0],
                           _p(D, _f64p), float(rho0), int(T), float(eps),
                           _p(lab, _i32p), _p(best, _f64p), _p(dist, _f64p))
    return lab, best, (dist.reshape(N, K) if want_dist else None)


def assign_multi(dists):
    """Sec. 5 multi-modal instances: the combined distance of (instance,
    centroid) is the sum of the per-modality distances (each an N x K
    array); labels = argmin with ties to the lowest centroid."""
    tot = np.zeros_like(np.asarray(dists[0], dtype=np.float64))
    for dm in dists:
        tot = tot + np.asarray(dm, dtype=np.float64)
    lab = np.argmin(tot, axis=1).astype(np.int32)
    return lab, tot[np.arange(len(lab)), lab], tot


def assign(wl, Xc, Wc, rho0=2.0, T=100, eps=1e-16, want_dist=False):
    """Labels argmin_c D(Q_c, P_k) (ties -> lowest c), best D, and all D."""
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    N = len(off) - 1
    Xc, Wc = _f64(Xc), _f64(Wc)
    K, m, d = Xc.shape
    lab = np.empty(N, dtype=np.int32)
    best = np.empty(N)
    dist = np.empty(N * K) if want_dist else None
    _load().orc_assign(N, _p(off, _i64p), d, _p(X, _f64p), _p(W, _f64p), K, m,
                       _p(Xc, _f64p), _p(Wc, _f64p), float(rho0), int(T),
                       float(eps), _p(lab, _i32p), _p(best, _f64p),
                       _p(dist, _f64p))
    return lab, best, (dist.reshape(N, K) if want_dist else None)


def cluster(wl, Xc, Wc, rounds, T=100, tau=10, rho0=2.0, eps=1e-16, rule=1,
            T_assign=100, callback=None):
    """D2-clustering (Algorithm "D2 Clustering") with B-ADMM centroids.

    Each round: assignment, then for every non-empty cluster a B-ADMM call
    started from the cached Pi2 for members whose label did not change and
    from the product coupling otherwise (Sec. 5); Lambda restarts at 0.
    Empty clusters keep their centroid.  Returns dict(Xc, Wc, labels, hist).
    """
    off = wl["offsets"]
    m = Xc.shape[1]
    n = int(off[-1])
    Xc, Wc = _f64(Xc).copy(), _f64(Wc).copy()
    plans = Plans(m, n)
    prev = None
    hist = []
    for r in range(rounds):
        lab, best, _ = assign(wl, Xc, Wc, rho0=rho0, T=T_assign, eps=eps)
        changed = int(len(lab)) if prev is None else int(np.sum(lab != prev))
        fin = np.zeros(len(Wc))
        for c in range(len(Wc)):
            mem = np.nonzero(lab == c)[0]
            if len(mem) == 0:
                continue
            warm = None if prev is None else (prev[mem] == c).astype(np.uint8)
            out = barycenter(wl, mem, Xc[c], Wc[c], plans=plans, warm=warm,
                             rho0=rho0, tau=tau, T=T, eps=eps, rule=rule)
            Xc[c], Wc[c] = out["x"], out["w"]
            fin[c] = out["ftrace"][-1] if T > 0 else 0.0
        rec = {"round": r, "changed": changed, "assign_obj": float(best.mean()),
               "f_plan": fin}
        hist.append(rec)
        if callback:
            callback(rec, Xc, Wc, lab)
        prev = lab
    return {"Xc": Xc, "Wc": Wc, "labels": prev, "hist": hist, "plans": plans}


def exact_w2(x, w, y, wy):
    """W_2^2 between (w, x) and (wy, y) by the transport LP Eq. (primal)."""
    from scipy.optimize import linprog

    C = cost_block(x, y)
    m, mk = C.shape
    A = np.zeros((m + mk, m * mk))
    for i in range(m):
        A[i, i * mk:(i + 1) * mk] = 1.0  # row sums (row-major flatten)
    for j in range(mk):
        A[m + j, j::mk] = 1.0            # column sums
    b = np.concatenate([_f64(w), _f64(wy)])
    res = linprog(C.reshape(-1), A_eq=A, b_eq=b, bounds=(0, None),
                  method="highs")
    if res.status != 0:
        raise RuntimeError("LP failed: " + res.message)
    return float(res.fun), res.x.reshape(m, mk)


def f_true(wl, members, x, w):
    """(1/N) sum_k W^2(P, P^(k)) over `members` (Eq. (centroid))."""
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    tot = 0.0
    for k in members:
        a, b = off[k], off[k + 1]
        tot += exact_w2(x, w, X[a:b], W[a:b])[0]
    return tot / len(members)


def round_feasible(P, a, b):
    """Round a nonnegative m x m_k matrix to a coupling with row sums a and
    column sums b (Altschuler, Weed and Rigollet 2017, Algorithm 2): scale
    rows down to at most a, then columns down to at most b, then add the
    rank-one correction err_r err_c^T / |err_r|_1."""
    P = _f64(P)
    a, b = _f64(a), _f64(b)
    r = P.sum(1)
    xr = np.ones_like(r)
    big = r > a
    xr[big] = a[big] / r[big]
    P1 = xr[:, None] * P
    c = P1.sum(0)
    yc = np.ones_like(c)
    big = c > b
    yc[big] = b[big] / c[big]
    P2 = P1 * yc[None, :]
    er = a - P2.sum(1)
    ec = b - P2.sum(0)
    E = er.sum()
    if E > 0:
        P2 = P2 + np.outer(er, ec) / E
    return P2


def feasible_objective(wl, members, x, w, plans):
    """(1/N) sum_k <C^(k), round(Pi1^(k))> over `members`, each Pi1 from
    `plans` rounded to marginals (w, w^(k)) by round_feasible."""
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    tot = 0.0
    for k in members:
        a, b = off[k], off[k + 1]
        P1 = plans.block(off, k)[0]
        R = round_feasible(P1, w, W[a:b])
        tot += float((R * cost_block(x, X[a:b])).sum())
    return tot / len(members)

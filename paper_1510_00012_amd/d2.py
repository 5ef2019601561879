"""Python binding of libd2.so (include/d2.h): argument marshalling only.

Every step of the B-ADMM barycenter / D2-clustering path runs in the HIP
library; this module converts numpy arrays to C pointers and C status codes
to exceptions.  There is no CPU fallback: if the library cannot be loaded or
no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libd2.so")

D2_OK, D2_EINVAL, D2_ENOMEM, D2_EDEVICE, D2_ENUMERIC, D2_ESTATE = range(6)
D2_F32, D2_F64 = 0, 1
D2_INIT_PRODUCT, D2_INIT_CACHED, D2_INIT_LEARNED = 0, 1, 2
STATUS_NAMES = {0: "D2_OK", 1: "D2_EINVAL", 2: "D2_ENOMEM", 3: "D2_EDEVICE",
                4: "D2_ENUMERIC", 5: "D2_ESTATE"}

# every symbol include/d2.h declares
EXPORTS = [
    "d2_create", "d2_destroy", "d2_last_error", "d2_load_instances",
    "d2_centroids_set", "d2_centroids_get", "d2_centroids_init",
    "d2_labels_set", "d2_labels_get", "d2_assign", "d2_barycenter",
    "d2_support_update", "d2_cluster", "d2_objective", "d2_plans_get",
    "d2_sizes", "d2_set_profiling", "d2_kernel_stats", "d2_set_schedule",
    "d2_assign_pairs", "d2_set_graph", "d2_autotune",
    "d2_set_bucketing", "d2_objective_feasible", "d2_residual",
    "d2_copy_probe", "d2_set_assign_bounds", "d2_load_instances_device",
    "d2_checkpoint_save", "d2_checkpoint_load", "d2_set_warm_start",
    "d2_ws_save", "d2_ws_load", "d2_ws_param_count", "d2_ws_create",
    "d2_ws_destroy", "d2_ws_last_error", "d2_ws_params_set",
    "d2_ws_params_get", "d2_ws_targets_from", "d2_ws_grad",
    "d2_ws_train_step", "d2_ws_propose", "d2_assign_noalloc",
    "d2_load_instances_symbolic", "d2_centroids_set_symbolic",
    "d2_assign_multi", "d2_cluster_multi", "d2_subgradient",
    "d2_set_cache_policy", "d2_set_rho",
]


class D2Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class BadmmParams(ctypes.Structure):
    _fields_ = [("rho0", ctypes.c_double), ("eps", ctypes.c_double),
                ("tau", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("xplan", ctypes.c_int32),
                ("init", ctypes.c_int32), ("fixed_support", ctypes.c_int32)]


class OtParams(ctypes.Structure):
    _fields_ = [("rho0", ctypes.c_double), ("eps", ctypes.c_double),
                ("iters", ctypes.c_int32), ("prune", ctypes.c_int32)]


class BadmmStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("n_empty", ctypes.c_int32),
                ("launches", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class RoundInfo(ctypes.Structure):
    _fields_ = [("round", ctypes.c_int32), ("n_changed", ctypes.c_int64),
                ("assign_obj", ctypes.c_double), ("ms_assign", ctypes.c_double),
                ("ms_barycenter", ctypes.c_double)]


class WsOpt(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("clip", ctypes.c_double)]


class SgParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("zeta", ctypes.c_double),
                ("tau", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("fixed_support", ctypes.c_int32),
                ("max_pivots", ctypes.c_int32)]


class SgStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("lp_failed", ctypes.c_int32),
                ("pivots", ctypes.c_int64), ("launches", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("ms", ctypes.c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


ROUND_CB = ctypes.CFUNCTYPE(None, ctypes.POINTER(RoundInfo), ctypes.c_void_p)

_lib = None
_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


def load_library(path: str = LIB_PATH):
    """Load libd2.so and declare the C signatures (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is missing: build it with "
                      "`python -m paper_1510_00012_amd.build`")
    try:
        # PyTorch ships its own HIP runtime under the same soname as the
        # system one libd2.so links against.  Loading torch first makes the
        # library bind to that runtime, so that the process holds a single
        # HIP runtime and torch tensors / streams can be handed to the
        # library; loaded the other way round, torch finds no GPU.
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    sig = {
        "d2_create": ([ctypes.POINTER(_p), ctypes.c_int, ctypes.c_int, _p],
                      ctypes.c_int),
        "d2_destroy": ([_p], None),
        "d2_last_error": ([_p], ctypes.c_char_p),
        "d2_load_instances": ([_p, _i64, _i32, _p, _p, _p], ctypes.c_int),
        "d2_centroids_set": ([_p, _i32, _i32, _p, _p], ctypes.c_int),
        "d2_centroids_get": ([_p, _p, _p], ctypes.c_int),
        "d2_centroids_init": ([_p, _i32, _i32, _p], ctypes.c_int),
        "d2_labels_set": ([_p, _p], ctypes.c_int),
        "d2_labels_get": ([_p, _p], ctypes.c_int),
        "d2_assign": ([_p, ctypes.POINTER(OtParams), _p, _p, _p],
                      ctypes.c_int),
        "d2_barycenter": ([_p, ctypes.POINTER(BadmmParams),
                           ctypes.POINTER(BadmmStats)], ctypes.c_int),
        "d2_support_update": ([_p], ctypes.c_int),
        "d2_cluster": ([_p, _i32, ctypes.POINTER(BadmmParams),
                        ctypes.POINTER(OtParams), ROUND_CB, _p], ctypes.c_int),
        "d2_objective": ([_p, _p, _i32, _p], ctypes.c_int),
        "d2_residual": ([_p, _p, _i32], ctypes.c_int),
        "d2_plans_get": ([_p, _i64, _p, _p, _p], ctypes.c_int),
        "d2_sizes": ([_p, _p, _p, _p, _p, _p], ctypes.c_int),
        "d2_set_profiling": ([_p, _i32], ctypes.c_int),
        "d2_set_schedule": ([_p, _i32, _i32], ctypes.c_int),
        "d2_set_bucketing": ([_p, _i32], ctypes.c_int),
        "d2_assign_pairs": ([_p, _p, _p, _p], ctypes.c_int),
        "d2_set_graph": ([_p, _i32], ctypes.c_int),
        "d2_set_assign_bounds": ([_p, _i32], ctypes.c_int),
        "d2_load_instances_device": ([_p, _i64, _i32, _p, _p, _p],
                                     ctypes.c_int),
        "d2_checkpoint_save": ([_p, ctypes.c_char_p], ctypes.c_int),
        "d2_checkpoint_load": ([_p, ctypes.c_char_p], ctypes.c_int),
        "d2_set_warm_start": ([_p, _p, _i32], ctypes.c_int),
        "d2_ws_save": ([_p, ctypes.c_char_p], ctypes.c_int),
        "d2_ws_load": ([_p, ctypes.c_char_p], ctypes.c_int),
        "d2_autotune": ([_p, ctypes.POINTER(BadmmParams), _p, _p, _p, _p],
                        ctypes.c_int),
        "d2_kernel_stats": ([_p, ctypes.POINTER(KernelStat), _i32, _p, _i32],
                            ctypes.c_int),
        "d2_objective_feasible": ([_p, _p, _p], ctypes.c_int),
        "d2_copy_probe": ([ctypes.c_int, _i64, _i32, _p, _p], ctypes.c_int),
        "d2_ws_param_count": ([_i32, _i32, _i32], _i64),
        "d2_ws_create": ([ctypes.POINTER(_p), _i32, _i32, _i32, _i32, _p],
                         ctypes.c_int),
        "d2_ws_destroy": ([_p], None),
        "d2_ws_last_error": ([_p], ctypes.c_char_p),
        "d2_ws_params_set": ([_p, _p], ctypes.c_int),
        "d2_ws_params_get": ([_p, _p], ctypes.c_int),
        "d2_ws_targets_from": ([_p, _p], ctypes.c_int),
        "d2_ws_grad": ([_p, _p, _p, _i32, _p, _p], ctypes.c_int),
        "d2_ws_train_step": ([_p, _p, _p, _i32, ctypes.POINTER(WsOpt), _p],
                             ctypes.c_int),
        "d2_ws_propose": ([_p, _p, _i32, _p, _p, _p], ctypes.c_int),
        "d2_load_instances_symbolic": ([_p, _i64, _p, _p, _p, _i32, _p],
                                       ctypes.c_int),
        "d2_centroids_set_symbolic": ([_p, _i32, _i32, _p, _p], ctypes.c_int),
        "d2_set_cache_policy": ([_p, _i32], ctypes.c_int),
        "d2_set_rho": ([_p, _p], ctypes.c_int),
        "d2_subgradient": ([_p, ctypes.POINTER(SgParams),
                            ctypes.POINTER(SgStats)], ctypes.c_int),
        "d2_assign_multi": ([_i32, _p, ctypes.POINTER(OtParams), _p, _p, _p],
                            ctypes.c_int),
        "d2_cluster_multi": ([_i32, _p, _i32, ctypes.POINTER(BadmmParams),
                              ctypes.POINTER(OtParams), ROUND_CB, _p],
                             ctypes.c_int),
        "d2_assign_noalloc": ([_i32, _p, ctypes.c_int, _i64, _i32, _i32, _p,
                               _p, _p, _i32, _i32, _p, _p,
                               ctypes.POINTER(OtParams), _p, _p,
                               ctypes.c_char_p, _i32], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def badmm_params(iters=100, tau=10, rho0=2.0, eps=1e-16, rule=1,
                 init=D2_INIT_CACHED, fixed_support=False):
    return BadmmParams(rho0=rho0, eps=eps, tau=tau, iters=iters, rule=rule,
                       xplan=0, init=init, fixed_support=int(fixed_support))


def ot_params(iters=100, rho0=2.0, eps=1e-16, prune=True):
    return OtParams(rho0=rho0, eps=eps, iters=iters, prune=int(bool(prune)))


SCHEDULES = os.path.join(_HERE, "schedules.json")


def schedule_key(offsets, K, m, d, dtype="f32", arch="gfx950"):
    mk = np.diff(np.asarray(offsets))
    return f"{arch}|{dtype}|{len(mk)}|{K}|{m}|{d}|{int(mk.max())}"


def tuned_schedule(key):
    """(chunk, waves, bucketing) recorded for a workload signature, or
    None."""
    import json
    try:
        tab = json.load(open(SCHEDULES))
    except OSError:
        return None
    ent = tab.get(key)
    return None if ent is None else (int(ent["chunk"]), int(ent["waves"]),
                                     int(ent.get("bucket", 100)))


class D2Context:
    """One library context (device buffers, stream, cached plans)."""

    def __init__(self, device=0, dtype="f32", stream=None):
        self.lib = load_library()
        self.dtype = dtype
        h = _p()
        dt = D2_F64 if dtype in ("f64", "float64", np.float64) else D2_F32
        st = self.lib.d2_create(ctypes.byref(h), int(device), dt,
                                None if stream is None else _p(int(stream)))
        if st != D2_OK:
            raise D2Error(st, "d2_create failed (no usable HIP device?)")
        self.h = h
        self.N = self.n = self.d = self.K = self.m = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.d2_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _chk(self, st):
        if st != D2_OK:
            msg = self.lib.d2_last_error(self.h)
            raise D2Error(st, msg.decode() if msg else "")

    # ------------------------------------------------------------ data
    def load_instances(self, offsets, X, W):
        off = _c(offsets, np.int64)
        X = _c(X, np.float64)
        W = _c(W, np.float64)
        N = len(off) - 1
        d = X.shape[1] if X.ndim == 2 else 1
        self._chk(self.lib.d2_load_instances(self.h, N, d, _ptr(off), _ptr(X),
                                             _ptr(W)))
        self.offsets, self.N, self.n, self.d = off, N, int(off[-1]), d

    def load_instances_device(self, offsets, dX, dW, d):
        """Borrow device buffers (integer device addresses, e.g. a torch
        tensor's data_ptr()) holding X (n x roundup(d, 4), zero padded) and
        W (n) in the context's dtype; the caller keeps them alive."""
        off = _c(offsets, np.int64)
        N = len(off) - 1
        self._chk(self.lib.d2_load_instances_device(
            self.h, N, int(d), _ptr(off), _p(int(dX)), _p(int(dW))))
        self.offsets, self.N, self.n, self.d = off, N, int(off[-1]), int(d)

    def load_instances_symbolic(self, offsets, sym, W, D):
        """Instances over a symbol set: sym (n) symbol ids, W (n) weights,
        D (S x S) the symbol-to-symbol cost table."""
        off = _c(offsets, np.int64)
        sym = _c(sym, np.int32)
        W = _c(W, np.float64)
        D = _c(D, np.float64)
        self._chk(self.lib.d2_load_instances_symbolic(
            self.h, len(off) - 1, _ptr(off), _ptr(sym), _ptr(W), D.shape[0],
            _ptr(D)))
        self.offsets, self.N, self.n, self.d = off, len(off) - 1, int(off[-1]), 1

    def centroids_set_symbolic(self, csym, Wc):
        csym = _c(csym, np.int32)
        Wc = _c(Wc, np.float64)
        K, m = csym.shape
        self._chk(self.lib.d2_centroids_set_symbolic(self.h, K, m, _ptr(csym),
                                                     _ptr(Wc)))
        self.K, self.m = K, m

    def checkpoint_save(self, path):
        self._chk(self.lib.d2_checkpoint_save(self.h, os.fsencode(path)))

    def checkpoint_load(self, path):
        """Restore centroids, labels, plan cache and schedule (the context
        must hold the same instances)."""
        self._chk(self.lib.d2_checkpoint_load(self.h, os.fsencode(path)))
        N, n, d, K, m = (ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(),
                         ctypes.c_int32(), ctypes.c_int32())
        self._chk(self.lib.d2_sizes(self.h, ctypes.byref(N), ctypes.byref(n),
                                    ctypes.byref(d), ctypes.byref(K),
                                    ctypes.byref(m)))
        self.K, self.m = K.value, m.value

    def set_warm_start(self, ws, gate=True):
        """Attach a D2WarmStart for init=D2_INIT_LEARNED (None detaches).
        gate: False / 0 none, True / 1 the product-coupling bound, an int
        >= 2 a B-ADMM probe of that many iterations."""
        self._ws = ws
        g = int(gate) if not isinstance(gate, bool) else int(gate)
        self._chk(self.lib.d2_set_warm_start(
            self.h, None if ws is None else ws.h, g))

    def centroids_set(self, Xc, Wc):
        Xc = _c(Xc, np.float64)
        Wc = _c(Wc, np.float64)
        K, m = Wc.shape
        self._chk(self.lib.d2_centroids_set(self.h, K, m, _ptr(Xc), _ptr(Wc)))
        self.K, self.m = K, m

    def centroids_init(self, members, m):
        mem = _c(members, np.int64)
        self._chk(self.lib.d2_centroids_init(self.h, len(mem), int(m),
                                             _ptr(mem)))
        self.K, self.m = len(mem), int(m)

    def centroids_get(self):
        Xc = np.empty((self.K, self.m, self.d))
        Wc = np.empty((self.K, self.m))
        self._chk(self.lib.d2_centroids_get(self.h, _ptr(Xc), _ptr(Wc)))
        return Xc, Wc

    def labels_set(self, labels):
        lab = _c(labels, np.int32)
        self._chk(self.lib.d2_labels_set(self.h, _ptr(lab)))

    def labels_get(self):
        lab = np.empty(self.N, dtype=np.int32)
        self._chk(self.lib.d2_labels_get(self.h, _ptr(lab)))
        return lab

    # ------------------------------------------------------------ steps
    def assign(self, iters=100, rho0=2.0, eps=1e-16, prune=True,
               outputs=True):
        """(labels, minimal distances, labels changed); with outputs=False
        the labels stay in the context and only the change count returns
        (labels and distances None)."""
        lab = np.empty(self.N, dtype=np.int32) if outputs else None
        dist = np.empty(self.N) if outputs else None
        nch = ctypes.c_int64(0)
        p = ot_params(iters, rho0, eps, prune)
        self._chk(self.lib.d2_assign(self.h, ctypes.byref(p), _ptr(lab),
                                     _ptr(dist), ctypes.byref(nch)))
        return lab, dist, int(nch.value)

    def barycenter(self, iters=100, tau=10, rho0=2.0, eps=1e-16, rule=1,
                   init=D2_INIT_CACHED, fixed_support=False):
        p = badmm_params(iters, tau, rho0, eps, rule, init, fixed_support)
        s = BadmmStats()
        self._chk(self.lib.d2_barycenter(self.h, ctypes.byref(p),
                                         ctypes.byref(s)))
        return {"iters": s.iters, "n_empty": s.n_empty,
                "launches": s.launches, "graph": s.graph, "ms": s.ms}

    def subgradient(self, iters=20, tau=10, alpha=0.5, zeta=1.0,
                    fixed_support=False, max_pivots=0):
        """d2_subgradient (Appendix A refinement) on the current labels."""
        p = SgParams(alpha=alpha, zeta=zeta, tau=tau, iters=iters,
                     fixed_support=int(fixed_support), max_pivots=max_pivots)
        s = SgStats()
        self._chk(self.lib.d2_subgradient(self.h, ctypes.byref(p),
                                          ctypes.byref(s)))
        return {"iters": s.iters, "lp_failed": s.lp_failed,
                "pivots": s.pivots, "launches": s.launches, "ms": s.ms}

    def assign_pairs(self):
        """(pairs iterated, total pairs) of the last assignment."""
        e, t = ctypes.c_int64(0), ctypes.c_int64(0)
        self._chk(self.lib.d2_assign_pairs(self.h, ctypes.byref(e), None,
                                           ctypes.byref(t)))
        return int(e.value), int(t.value)

    def assign_pairs_costed(self):
        """Pairs whose cost block the last assignment formed."""
        c = ctypes.c_int64(0)
        self._chk(self.lib.d2_assign_pairs(self.h, None, ctypes.byref(c),
                                           None))
        return int(c.value)

    def support_update(self):
        self._chk(self.lib.d2_support_update(self.h))

    def cluster(self, rounds, iters=100, tau=10, rho0=2.0, eps=1e-16, rule=1,
                assign_iters=100, prune=True, callback=None):
        bp = badmm_params(iters, tau, rho0, eps, rule, D2_INIT_CACHED)
        op = ot_params(assign_iters, rho0, eps, prune)
        recs = []

        def _cb(info, user):
            r = info.contents
            rec = {"round": r.round, "n_changed": r.n_changed,
                   "assign_obj": r.assign_obj,
                   "ms_barycenter": r.ms_barycenter}
            recs.append(rec)
            if callback:
                callback(rec)

        cb = ROUND_CB(_cb)
        self._chk(self.lib.d2_cluster(self.h, int(rounds), ctypes.byref(bp),
                                      ctypes.byref(op), cb, None))
        return recs

    def objective(self, iters):
        tr = np.zeros((iters, self.K))
        rho = np.zeros(self.K)
        self._chk(self.lib.d2_objective(self.h, _ptr(tr), int(iters),
                                        _ptr(rho)))
        return tr, rho

    def residual(self, iters):
        """(iters, K) primal residual trace of the last barycenter."""
        r = np.zeros((iters, self.K))
        self._chk(self.lib.d2_residual(self.h, _ptr(r), int(iters)))
        return r

    def autotune(self, iters=20, tau=10, rho0=2.0, eps=1e-16, rule=1):
        """Pick the fastest (chunk, waves, bucketing) schedule on the
        current labels."""
        p = badmm_params(iters, tau, rho0, eps, rule, D2_INIT_PRODUCT)
        ch, wv, bk = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        ms = ctypes.c_double(0)
        self._chk(self.lib.d2_autotune(self.h, ctypes.byref(p),
                                       ctypes.byref(ch), ctypes.byref(wv),
                                       ctypes.byref(bk), ctypes.byref(ms)))
        return {"chunk": ch.value, "waves": wv.value, "bucket": bk.value,
                "ms": ms.value}

    def set_assign_bounds(self, on=True):
        """Cross-round lower bounds of the pruned assignment on / off."""
        self._chk(self.lib.d2_set_assign_bounds(self.h, int(bool(on))))

    def set_rho(self, rho):
        """Hold rho per cluster (K values) in later barycenter calls; None
        returns to Eq. (rho)."""
        r = None if rho is None else _c(rho, np.float64)
        self._chk(self.lib.d2_set_rho(self.h, _ptr(r)))

    def set_cache_policy(self, policy):
        """0 automatic, 1 default caching, 2 streaming plan state."""
        self._chk(self.lib.d2_set_cache_policy(self.h, int(policy)))

    def set_graph(self, on=True):
        self._chk(self.lib.d2_set_graph(self.h, int(bool(on))))

    def set_schedule(self, chunk_instances, waves_per_group, bucket=None):
        self._chk(self.lib.d2_set_schedule(self.h, int(chunk_instances),
                                           int(waves_per_group)))
        if bucket is not None:
            self.set_bucketing(bucket)

    def set_bucketing(self, min_pct):
        self._chk(self.lib.d2_set_bucketing(self.h, int(min_pct)))

    def set_profiling(self, on=True):
        self._chk(self.lib.d2_set_profiling(self.h, int(bool(on))))

    def kernel_stats(self, reset=False):
        """{kind: (launches, total_ms)} accumulated while profiling."""
        arr = (KernelStat * 16)()
        cnt = ctypes.c_int32(0)
        self._chk(self.lib.d2_kernel_stats(self.h, arr, 16, ctypes.byref(cnt),
                                           int(bool(reset))))
        return {arr[q].name.decode(): (int(arr[q].launches),
                                       float(arr[q].total_ms))
                for q in range(min(cnt.value, 16))}

    def objective_feasible(self):
        """(per-instance, per-cluster) rounded-plan objective of the current
        centroids under the last plans."""
        pi = np.zeros(self.N)
        pc = np.zeros(self.K)
        self._chk(self.lib.d2_objective_feasible(self.h, _ptr(pi), _ptr(pc)))
        return pi, pc

    def plans_get(self, k):
        mk = int(self.offsets[k + 1] - self.offsets[k])
        bufs = [np.empty(self.m * mk) for _ in range(3)]
        self._chk(self.lib.d2_plans_get(self.h, int(k), *[_ptr(b) for b in bufs]))
        return tuple(b.reshape(mk, self.m).T.copy() for b in bufs)


def copy_probe(device=0, mib=2048, reps=10):
    """(GB/s, ms) of the library's plain device-copy kernel over a buffer of
    `mib` MiB (read + write bytes per second of the fastest repetition)."""
    lib = load_library()
    g, t = ctypes.c_double(0), ctypes.c_double(0)
    st = lib.d2_copy_probe(int(device), int(mib) << 20, int(reps),
                           ctypes.byref(g), ctypes.byref(t))
    if st != D2_OK:
        raise D2Error(st, "d2_copy_probe failed")
    return g.value, t.value


def assign_noalloc(N, d, mk_max, offsets, X, W, K, m, Xc, Wc, labels, dist,
                   dtype="f32", iters=100, rho0=2.0, eps=1e-16, prune=True,
                   device=0, stream=None):
    """d2_assign_noalloc: every array argument is an integer device address
    (e.g. a torch tensor's data_ptr()); the call only enqueues work on
    `stream` (a hipStream_t as an integer, None: the null stream)."""
    lib = load_library()
    p = ot_params(iters, rho0, eps, prune)
    err = ctypes.create_string_buffer(256)
    st = lib.d2_assign_noalloc(
        int(device), stream, D2_F32 if dtype == "f32" else D2_F64, int(N),
        int(d), int(mk_max), offsets, X, W, int(K), int(m), Xc, Wc,
        ctypes.byref(p), labels, dist, err, len(err))
    if st != D2_OK:
        raise D2Error(st, err.value.decode())


def _ctx_array(ctxs):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.h for c in ctxs])
    return arr


def assign_multi(ctxs, iters=100, rho0=2.0, eps=1e-16):
    """d2_assign_multi over the modality contexts `ctxs` (D2Context list):
    (labels, minimal summed distances, labels changed)."""
    c0 = ctxs[0]
    lab = np.empty(c0.N, dtype=np.int32)
    dist = np.empty(c0.N)
    nch = ctypes.c_int64(0)
    p = ot_params(iters, rho0, eps, False)
    c0._chk(c0.lib.d2_assign_multi(len(ctxs), _ctx_array(ctxs),
                                   ctypes.byref(p), _ptr(lab), _ptr(dist),
                                   ctypes.byref(nch)))
    return lab, dist, int(nch.value)


def cluster_multi(ctxs, rounds, iters=100, tau=10, rho0=2.0, eps=1e-16,
                  rule=1, assign_iters=100):
    """d2_cluster_multi: per-round records (dicts) of the callback."""
    c0 = ctxs[0]
    recs = []

    def cb(info, user):
        i = info.contents
        recs.append({"round": i.round, "n_changed": i.n_changed,
                     "assign_obj": i.assign_obj,
                     "ms_barycenter": i.ms_barycenter})

    ccb = ROUND_CB(cb)
    bp = badmm_params(iters, tau, rho0, eps, rule, D2_INIT_CACHED, False)
    op = ot_params(assign_iters, rho0, eps, False)
    c0._chk(c0.lib.d2_cluster_multi(len(ctxs), _ctx_array(ctxs), rounds,
                                    ctypes.byref(bp), ctypes.byref(op), ccb,
                                    None))
    return recs


def ws_param_count(m, d, hidden):
    return int(load_library().d2_ws_param_count(int(m), int(d), int(hidden)))


class D2WarmStart:
    """Deep-sets warm-start network (d2_ws_* calls)."""

    def __init__(self, m, d, hidden, theta, device=0):
        self.lib = load_library()
        self.m, self.d, self.hidden = int(m), int(d), int(hidden)
        self.np = ws_param_count(m, d, hidden)
        if self.np < 0:
            raise D2Error(D2_EINVAL, "network size outside the limits")
        th = _c(theta, np.float32)
        if th.size != self.np:
            raise D2Error(D2_EINVAL, f"theta has {th.size} values, "
                          f"expected {self.np}")
        h = _p()
        st = self.lib.d2_ws_create(ctypes.byref(h), int(device), self.m,
                                   self.d, self.hidden, _ptr(th))
        if st != D2_OK:
            raise D2Error(st, "d2_ws_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.d2_ws_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != D2_OK:
            msg = self.lib.d2_ws_last_error(self.h)
            raise D2Error(st, msg.decode() if msg else "")

    def params_get(self):
        th = np.empty(self.np, dtype=np.float32)
        self._chk(self.lib.d2_ws_params_get(self.h, _ptr(th)))
        return th

    def params_set(self, theta):
        th = _c(theta, np.float32)
        if th.size != self.np:
            raise D2Error(D2_EINVAL, "theta size")
        self._chk(self.lib.d2_ws_params_set(self.h, _ptr(th)))

    def save(self, path):
        self._chk(self.lib.d2_ws_save(self.h, os.fsencode(path)))

    def load(self, path):
        self._chk(self.lib.d2_ws_load(self.h, os.fsencode(path)))

    def targets_from(self, ctx):
        self._chk(self.lib.d2_ws_targets_from(self.h, ctx.h))

    def grad(self, ctx, clusters):
        ids = _c(clusters, np.int32)
        g = np.empty(self.np, dtype=np.float32)
        loss = ctypes.c_double(0)
        self._chk(self.lib.d2_ws_grad(self.h, ctx.h, _ptr(ids), ids.size,
                                      ctypes.byref(loss), _ptr(g)))
        return loss.value, g

    def train_step(self, ctx, clusters, lr=1e-3, beta1=0.9, beta2=0.999,
                   eps=1e-8, clip=1.0, want_loss=True):
        ids = _c(clusters, np.int32)
        opt = WsOpt(lr=lr, beta1=beta1, beta2=beta2, eps=eps, clip=clip)
        loss = ctypes.c_double(0)
        self._chk(self.lib.d2_ws_train_step(
            self.h, ctx.h, _ptr(ids), ids.size, ctypes.byref(opt),
            ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def propose(self, ctx, gate=True):
        """Replace accepted clusters' centroids in ctx; returns
        (accepted[K], bound_prop[K], bound_plain[K])."""
        acc = np.zeros(ctx.K, dtype=np.int32)
        bp = np.zeros(ctx.K)
        bq = np.zeros(ctx.K)
        self._chk(self.lib.d2_ws_propose(self.h, ctx.h, int(bool(gate)),
                                         _ptr(acc), _ptr(bp), _ptr(bq)))
        return acc, bp, bq

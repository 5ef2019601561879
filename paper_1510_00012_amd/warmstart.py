"""Learned warm start: training-data generation, training and evaluation.

Everything numeric runs in the HIP library through the d2_* / d2_ws_* calls;
this module only draws seeded inputs, orders the calls and reports.

  targets   the batched B-ADMM centroid update (Sec. 3.2) run to T_tgt
            iterations on every training cluster at once, from the plain
            initial centroid (Sec. 5: a random member merged down to m
            points); the resulting centroids are the network's targets.
  training  Adam on random batches of training clusters.
  eval      held-out clusters: plain initial centroid vs the gated network
            proposal, both followed by B-ADMM.  The objective at a given
            iteration count T is the rounded-plan objective
            (d2_objective_feasible, an upper bound on Eq. (centroid) at the
            centroid reached after T iterations).  A cluster reaches the
            target once that objective is <= (1 + 1e-4) F*, F* the plain
            run's objective after T_max iterations; T runs over a ladder,
            each a fresh run from the initial centroid.  Seconds to target
            = initialisation wall time + T_hit x the batched run's device
            time per iteration.

Usage: python -m paper_1510_00012_amd.warmstart --family gmm3 --out r.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from paper_1510_00012_amd import d2 as D2
from synth.generators import deepsets_init_params, warmstart_clusters

FAMILIES = {
    # gmm_d3_n65536_k16-like colour distributions and topic_d64_n200000_k64-like word-vector bags
    "gmm3": dict(m=16, n_train=4000, n_eval=500, nc_lo=64, nc_hi=2048,
                 steps=3000, batch=32, lr=1e-3),
    "topic64": dict(m=32, n_train=1000, n_eval=200, nc_lo=64, nc_hi=512,
                    steps=2000, batch=16, lr=1e-3),
}
LADDER = [10, 20, 30, 50, 75, 100, 150, 200, 300, 500, 750, 1000, 1500, 2000]


def family_context(family, n_clusters, seed, nc_lo, nc_hi, m, dtype="f32"):
    """Context with every cluster's instances, labels = cluster ids and the
    plain initial centroids (each cluster's first member merged to m)."""
    wl = warmstart_clusters(family, n_clusters, seed=seed, nc_lo=nc_lo,
                            nc_hi=nc_hi)
    ctx = D2.D2Context(0, dtype)
    ctx.load_instances(wl["offsets"], wl["X"], wl["W"])
    t0 = time.perf_counter()
    ctx.centroids_init(wl["first"], m)
    t_init = time.perf_counter() - t0
    ctx.labels_set(wl["labels"])
    return wl, ctx, t_init


def train(ws, ctx, K, steps, batch, lr, seed, log_every=100):
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = []
    t0 = time.perf_counter()
    for it in range(steps):
        ids = rng.choice(K, size=min(batch, K), replace=False).astype(np.int32)
        # step size: constant, then a tenth for the last quarter
        step_lr = lr if it < 0.75 * steps else 0.1 * lr
        want = (it % log_every == 0) or it == steps - 1
        loss = ws.train_step(ctx, ids, lr=step_lr, want_loss=want)
        if want:
            hist.append((it, float(loss)))
            print(f"  step {it:5d} loss {loss:.5f}", flush=True)
    return hist, time.perf_counter() - t0


def run_protocol(ctx, X0, W0, T, tau, fix=0):
    """T B-ADMM iterations from (X0, W0) with the product plan; with fix > 0
    the first min(T, fix) iterations keep the support fixed (the plans
    settle on the initial support) and the rest continue from the cached
    plans with support updates.  Returns the device milliseconds."""
    ctx.centroids_set(X0, W0)
    if fix <= 0:
        return ctx.barycenter(iters=T, tau=tau, init=D2.D2_INIT_PRODUCT)["ms"]
    t1 = min(T, fix)
    ms = ctx.barycenter(iters=t1, tau=tau, init=D2.D2_INIT_PRODUCT,
                        fixed_support=True)["ms"]
    if T > t1:
        ms += ctx.barycenter(iters=T - t1, tau=tau,
                             init=D2.D2_INIT_CACHED)["ms"]
    return ms


def ladder_objectives(ctx, X0, W0, ladder, tau, fix=0):
    """Rounded-plan objective per cluster after T iterations from (X0, W0),
    for every T in the ladder; also device ms per iteration of the last."""
    F = np.zeros((len(ladder), X0.shape[0]))
    ms_it = None
    for q, T in enumerate(ladder):
        ms = run_protocol(ctx, X0, W0, T, tau, fix)
        F[q] = ctx.objective_feasible()[1]
        ms_it = ms / T
    return F, ms_it


def hit_iterations(F, Fstar, ladder, rel=1e-4):
    ok = F <= (1.0 + rel) * Fstar[None, :]
    T = np.full(F.shape[1], np.inf)
    for c in range(F.shape[1]):
        idx = np.nonzero(ok[:, c])[0]
        if len(idx):
            T[c] = ladder[idx[0]]
    return T


def evaluate(ws, family, cfg, seed, tau=10, ladder=LADDER, fix=50):
    m = cfg["m"]
    wl, ctx, t_plain = family_context(family, cfg["n_eval"], seed,
                                      cfg["nc_lo"], cfg["nc_hi"], m)
    K = cfg["n_eval"]
    Xp, Wp = ctx.centroids_get()
    # warm: plain init, then the gated proposal
    ctx.centroids_set(Xp, Wp)
    t0 = time.perf_counter()
    acc, bprop, bplain = ws.propose(ctx, gate=True)
    t_prop = time.perf_counter() - t0
    Xw, Ww = ctx.centroids_get()
    Fp, ms_p = ladder_objectives(ctx, Xp, Wp, ladder, tau)
    Fstar = Fp[-1]
    Tp = hit_iterations(Fp, Fstar, ladder)
    # the plain run's final centroids as a proposal: what a perfect
    # prediction of the converged centroid would give
    ctx.centroids_set(Xp, Wp)
    ctx.barycenter(iters=ladder[-1], tau=tau, init=D2.D2_INIT_PRODUCT)
    Xc, Wc = ctx.centroids_get()
    variants = {"warm": (Xw, Ww, 0, t_plain + t_prop),
                f"warm_fix{fix}": (Xw, Ww, fix, t_plain + t_prop),
                f"plain_fix{fix}": (Xp, Wp, fix, t_plain),
                "converged": (Xc, Wc, 0, None),
                f"converged_fix{fix}": (Xc, Wc, fix, None)}

    def summary(T, t_init, ms_it):
        reached = np.isfinite(T)
        sec = (t_init or 0.0) + np.where(reached, T, np.nan) * ms_it * 1e-3
        return {
            "frac_reached": float(reached.mean()),
            "median_iters": float(np.median(T)) if reached.mean() >= 0.5
            else None,
            "p90_iters": float(np.quantile(T, 0.9)) if reached.mean() >= 0.9
            else None,
            "median_seconds": float(np.nanmedian(sec))
            if reached.mean() >= 0.5 and t_init is not None else None,
            "init_seconds": t_init,
            "device_ms_per_iter": ms_it,
        }

    rep = {
        "n_clusters": K,
        "instances": int(len(wl["offsets"]) - 1),
        "ladder": list(ladder),
        "plain": summary(Tp, t_plain, ms_p),
        "fallback_rate": float((acc == 0).mean()),
        "propose_seconds": t_prop,
        "median_rel_gap": {"plain": [float(np.median(Fp[q] / Fstar - 1))
                                     for q in range(len(ladder))]},
    }
    for name, (X0, W0, fx, t_init) in variants.items():
        F, ms = ladder_objectives(ctx, X0, W0, ladder, tau, fx)
        T = hit_iterations(F, Fstar, ladder)
        rep[name] = summary(T, t_init, ms)
        rep[name]["final_below_plain"] = float((F[-1] <= Fstar).mean())
        rep["median_rel_gap"][name] = [float(np.median(F[q] / Fstar - 1))
                                       for q in range(len(ladder))]
        print(f"  {name}: reached {rep[name]['frac_reached']:.3f} "
              f"median iters {rep[name]['median_iters']}", flush=True)
    ctx.close()
    return rep


def run(family, seed=0, steps=None, out=None, t_target=1000, tau=10,
        save_params=None, params=None, untrained=True, fix=50):
    cfg = dict(FAMILIES[family])
    if steps is not None:
        cfg["steps"] = steps
    m = cfg["m"]
    H = 128
    d = 3 if family == "gmm3" else 64
    theta0 = deepsets_init_params(m, d, H, seed=200 + seed).astype(np.float32)
    rep = {"family": family, "m": m, "d": d, "hidden": H, "config": cfg,
           "target_iters": t_target, "tau": tau}
    if params is None:
        print(f"[warmstart {family}] training set", flush=True)
        t0 = time.perf_counter()
        wl, ctx, _ = family_context(family, cfg["n_train"], 100 + seed,
                                    cfg["nc_lo"], cfg["nc_hi"], m)
        rep["datagen_seconds"] = time.perf_counter() - t0
        st = ctx.barycenter(iters=t_target, tau=tau, init=D2.D2_INIT_PRODUCT)
        print(f"  targets: {len(wl['offsets']) - 1} instances, "
              f"{st['ms']:.1f} ms device", flush=True)
        ws = D2.D2WarmStart(m, d, H, theta0)
        ws.targets_from(ctx)
        # loss floor: a perfect prediction leaves the entropy of w*
        _, Wt = ctx.centroids_get()
        Wt = np.clip(Wt, 1e-300, None)
        rep["target_entropy_mean"] = float(np.mean(-(Wt * np.log(Wt)).sum(1)))
        hist, t_train = train(ws, ctx, cfg["n_train"], cfg["steps"],
                              cfg["batch"], cfg["lr"], seed=300 + seed)
        ctx.close()
        rep.update(train_instances=int(len(wl["offsets"]) - 1),
                   train_seconds=t_train, target_device_ms=st["ms"],
                   loss_history=hist)
        if save_params:
            np.save(save_params, ws.params_get())
    else:
        ws = D2.D2WarmStart(m, d, H, np.load(params))
        rep["params_file"] = os.path.basename(params)
    print(f"[warmstart {family}] evaluation", flush=True)
    rep["eval"] = evaluate(ws, family, cfg, seed=400 + seed, tau=tau, fix=fix)
    if untrained:
        rep["eval_untrained"] = evaluate(D2.D2WarmStart(m, d, H, theta0),
                                         family, cfg, seed=400 + seed,
                                         tau=tau, fix=fix)
    rep["command"] = "python -m paper_1510_00012_amd.warmstart " + " ".join(
        sys.argv[1:])
    if out:
        with open(out, "w") as f:
            json.dump(rep, f, indent=1)
    return rep


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--family", default="gmm3", choices=sorted(FAMILIES))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--out", default=None)
    ap.add_argument("--save-params", default=None)
    ap.add_argument("--params", default=None,
                    help="evaluate these parameters (.npy) without training")
    ap.add_argument("--no-untrained", action="store_true")
    ap.add_argument("--fix", type=int, default=50)
    a = ap.parse_args(argv)
    rep = run(a.family, a.seed, a.steps, a.out, save_params=a.save_params,
              params=a.params, untrained=not a.no_untrained, fix=a.fix)
    ev = rep["eval"]
    print(json.dumps({"family": rep["family"], "plain": ev["plain"],
                      "warm": ev["warm"],
                      "fallback_rate": ev["fallback_rate"]}))
    return 0


if __name__ == "__main__":
    sys.exit(main())

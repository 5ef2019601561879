#!/usr/bin/env python3
"""Benchmark of the B-ADMM / D2-clustering hot path on one MI355X.

One step = one round of D2-clustering over the whole synthetic workload:
the assignment step (B-ADMM transport against every centroid, exact
pruning) followed by the batched B-ADMM barycenter update of all K clusters
(T iterations, support update every tau, cached-plan warm start).  Default
workload: the largest single-GPU configuration, K=256 clusters, N=2,000,000
ragged instances (m_k uniform in [4,32]) in d=16 from a 1024-component
Gaussian mixture, centroid support m=16, T=50; 5 rounds (1 warm-up + 4
timed).  Plans Pi1, Pi2, Lambda and the cost cache stay resident in HBM.

value  = N * T * steps / (wall time of the timed steps): B-ADMM
         instance-iterations per second of whole rounds (assignment time
         included), inputs resident in HBM.
Also reported: the barycenter-only rate, per-kernel HIP-event times, the
roofline of the dominant kernel (and of the plan-update kernel), and the FP64
CPU oracle timed on bounded slices of the same workload (extrapolated to the
whole round, at all host cores and at one thread).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# transcendental (v_exp_f32) issue rate: 256 CUs x 16 lanes/clk x 2.4 GHz
EXP_PEAK_GOPS = 256 * 16 * 2.4


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    # the device code of the plan-update and auxiliary kernels
    for f in ("d2_kernels.hpp", "d2_kinst.hpp"):
        with open(os.path.join(ROOT, "paper_1510_00012_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kind, wl, m, esz):
    """Bytes a launch of `kind` must move (what the method reads/writes).

    iter_ba: read+write Pi1 and Lambda (4 per entry), the support points and
    weights of every column (cost recomputed on the fly for d <= 4, else a
    cached cost entry per plan entry), the offsets and work-list entry of
    every instance."""
    off = wl["offsets"]
    N = len(off) - 1
    n = int(off[-1])
    d = wl["X"].shape[1]
    E = m * n
    per_inst = 2 * 8 + 4
    if kind == "iter_ba":
        cost = n * d * esz if d <= 4 else E * esz
        return 4 * E * esz + cost + n * esz + N * per_inst
    return None


def assign_exps(wl, K, m, iters, frac=1.0):
    """Exponentials the assignment evaluates: 2 per plan entry per
    iteration for every (instance, centroid) pair run through the
    iterations (`frac` of all pairs survive the exact lower-bound pruning;
    their supports are taken at the workload's mean size)."""
    n = int(wl["offsets"][-1])
    return 2.0 * K * m * n * iters * frac


def load_traffic(kernel, workload, src_hash):
    """HBM bytes per launch from committed rocprofv3 counter summaries,
    only if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_source_hash") != src_hash:
        return None
    return rec.get("hbm_bytes_per_launch")


def _subset(wl, idx):
    """Instances idx of a workload as a workload of their own."""
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    idx = np.asarray(idx, dtype=np.int64)
    sizes = off[idx + 1] - off[idx]
    o = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    rows = np.concatenate([np.arange(off[k], off[k + 1]) for k in idx])
    return {"offsets": o, "X": np.ascontiguousarray(X[rows]),
            "W": np.ascontiguousarray(W[rows])}


def cpu_baseline(wl, Xc, Wc, labels, T, tau, T_assign, target_s=20.0):
    """The FP64 oracle on bounded slices of one round of the workload,
    extrapolated to the whole round.

    Barycenter: whole clusters (the GPU's labels, taken in index order) run
    through the oracle's B-ADMM (T iterations, tau) until about 35 % of the
    time budget is used; the time is scaled by (plan entries of the
    workload) / (plan entries of the slice) -- the method's work is linear
    in the plan entries (Sec. 5 complexity).  Assignment: an evenly spaced
    instance sample run through the oracle's exhaustive assignment (T_assign
    iterations per instance-centroid pair), scaled by (support points of the
    workload) / (support points of the sample).  Both legs are timed with
    all host threads and again with one thread (each about a quarter of the
    budget at one thread)."""
    import oracle
    oracle.build(force=False)
    off = wl["offsets"]
    N = len(off) - 1
    K, m = Wc.shape
    sizes = np.diff(off)
    n_tot = int(off[-1])
    members = [np.nonzero(labels == c)[0] for c in range(K)]
    order = [c for c in range(K) if len(members[c])]

    def bary_time(budget):
        t = 0.0
        cols = 0
        used = []
        for c in order:
            sub = _subset(wl, members[c])
            t0 = time.perf_counter()
            oracle.barycenter(sub, np.arange(len(members[c])), Xc[c], Wc[c],
                              T=T, tau=tau)
            t += time.perf_counter() - t0
            cols += int(sizes[members[c]].sum())
            used.append(c)
            if t >= budget:
                break
        return t * n_tot / cols, len(used), cols

    def assign_time(budget, S):
        # the oracle's assignment hands out instances 64 at a time per
        # thread, so an all-thread sample starts at 64 instances per thread
        while True:
            idx = np.linspace(0, N - 1, S).astype(np.int64)
            sub = _subset(wl, idx)
            t0 = time.perf_counter()
            oracle.assign(sub, Xc, Wc, T=T_assign)
            t = time.perf_counter() - t0
            if t >= budget or S >= N:
                return t * n_tot / int(sub["offsets"][-1]), S
            S = int(min(N, S * max(2.0, min(8.0, budget / max(t, 1e-3)))))

    threads = oracle.num_threads()
    tb, nb, cb = bary_time(0.35 * target_s)
    ta, sa = assign_time(0.15 * target_s, min(N, 64 * threads))
    oracle.set_num_threads(1)
    try:
        tb1, nb1, cb1 = bary_time(0.25 * target_s)
        ta1, sa1 = assign_time(0.1 * target_s, 8)
    finally:
        oracle.set_num_threads(threads)
    return {"value": N * T / (ta + tb), "unit": "instance-iterations/s",
            "cores": threads, "kind": "oracle",
            "sample": f"extrapolated from slices of one round: barycenter of "
                      f"{nb} whole clusters ({cb} of {n_tot} support points, "
                      f"{T} it, scaled by plan entries -> {tb:.1f}s), "
                      f"exhaustive assignment of {sa} evenly spaced instances "
                      f"against all {K} centroids ({T_assign} it/pair, scaled "
                      f"by support points -> {ta:.1f}s)",
            "barycenter_s_extrapolated": tb, "assign_s_extrapolated": ta,
            "single_thread": {
                "value": N * T / (ta1 + tb1), "cores": 1,
                "sample": f"barycenter of {nb1} clusters ({cb1} support "
                          f"points -> {tb1:.1f}s), assignment of {sa1} "
                          f"instances (-> {ta1:.1f}s), extrapolated as above"}}


def time_subgradient(ctx, N, iters, tau=10):
    """The subgradient-descent refinement (Appendix A) on the context's
    current labels and centroids: one exact transport LP per instance and
    iteration (device network simplex), timed with HIP events by the
    library."""
    st = ctx.subgradient(iters=iters, tau=tau)
    lps = N * iters
    return {"iters": iters, "lps": lps, "ms": st["ms"],
            "lp_per_s": lps / (st["ms"] / 1000.0),
            "pivots_per_lp": st["pivots"] / lps,
            "lp_failed": st["lp_failed"], "launches": st["launches"]}


def symbolic_bytes(mods, ms, esz=4):
    """Algorithmic bytes of one plan-update iteration over symbolic
    supports (every modality): Pi1 and Lambda read and written and the cost
    cache read per plan entry, symbol id and weight per support point,
    offsets and work id per instance."""
    b = 0
    for md, m in zip(mods, ms):
        n = int(md["offsets"][-1])
        E = m * n
        b += 5 * E * esz + n * (4 + esz) + (len(md["offsets"]) - 1) * 20
    return b


def bench_symbolic(args, wl, d2, torch):
    """Rounds of D2-clustering over symbolic supports (Sec. 5: a symbol-to-
    symbol cost table, no support step); several modalities (Sec. 5, last
    paragraph) assign by the summed distance and update each modality's
    centroids.  Initial centroids: the heaviest symbols of a seeded random
    partition."""
    from synth.generators import symbol_init_centroids
    mods = wl.get("modalities") or [wl]
    ms = wl["m"] if isinstance(wl["m"], tuple) else (wl["m"],)
    K = wl["K"]
    T = args.iters or wl["T"]
    tau, T_assign = 10, 100
    N = len(mods[0]["offsets"]) - 1
    stream = torch.cuda.Stream()
    rng = np.random.Generator(np.random.PCG64(wl["seed"] + 1))
    lab0 = rng.integers(0, K, size=N).astype(np.int32)
    ctxs = []
    for md, m in zip(mods, ms):
        ctx = d2.D2Context(0, "f32", stream=stream.cuda_stream)
        ctx.load_instances_symbolic(md["offsets"], md["sym"], md["W"], md["D"])
        csym, Wc = symbol_init_centroids(md, lab0, K, m)
        ctx.centroids_set_symbolic(csym, Wc)
        ctxs.append(ctx)
    log(f"[bench] symbolic workload {args.workload}: N={N} modalities="
        f"{len(ctxs)} K={K} m={ms} S={[md['S'] for md in mods]} T={T}")

    def step(first):
        if len(ctxs) == 1:
            ctxs[0].assign(iters=T_assign, outputs=False)
        else:
            lab, _, _ = d2.assign_multi(ctxs, iters=T_assign)
            for c in ctxs:
                c.labels_set(lab)
        tot = 0.0
        for c in ctxs:
            st = c.barycenter(iters=T, tau=tau,
                              init=d2.D2_INIT_PRODUCT if first
                              else d2.D2_INIT_CACHED)
            tot += st["ms"]
        return tot

    for w in range(args.warmup):
        step(w == 0)
    bary_ms = []
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for s_ in range(args.steps):
        bary_ms.append(step(args.warmup == 0 and s_ == 0))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    ks = {}
    for c in ctxs:
        c.set_profiling(True)
        c.kernel_stats(reset=True)
    for _ in range(args.profile_rounds):
        step(False)
    torch.cuda.synchronize()
    for c in ctxs:
        c.set_profiling(False)
        for k, v in c.kernel_stats(reset=True).items():
            n0, t0 = ks.get(k, (0, 0.0))
            ks[k] = (n0 + v[0], t0 + v[1])
    M = len(ctxs)
    value = N * T * M * args.steps / elapsed
    rec = {
        "metric": "B-ADMM instance-iterations/s", "value": value,
        "unit": "instance-iterations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: one D2-clustering round "
                               f"over symbolic supports ({M} modalities) = "
                               f"assignment ({T_assign} transport iterations "
                               f"per pair) + batched barycenter ({T} "
                               f"iterations, support fixed) per modality",
                   "N": N, "K": K, "m": list(ms),
                   "S": [md["S"] for md in mods], "T": T,
                   "T_assign": T_assign, "seed": wl["seed"]},
        "barycenter_ms_mean": float(np.mean(bary_ms)),
        "kernel_ms": {k: {"launches": v[0], "total_ms": v[1]}
                      for k, v in ks.items()},
    }
    if "iter_ba" in ks:
        launches, tot = ks["iter_ba"]
        # one plan-update launch per modality and iteration
        avg_s = tot / (launches / M) / 1000.0
        b = symbolic_bytes(mods, ms)
        rec["roofline_plan_update"] = {
            "bound": "hbm", "achieved": b / avg_s / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": b / avg_s / 1e9 / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_iter_ba", "avg_iteration_ms": 1000 * avg_s,
            "bytes_per_iteration": b}
    if args.subgradient and M == 1:
        rec["subgradient"] = time_subgradient(ctxs[0], N, args.subgradient)
    for c in ctxs:
        c.close()
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gmm_d16_n2000000_k256")
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--profile-rounds", type=int, default=3,
                    help="host-issued rounds timed per kernel with HIP events")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter "
                         "calibration for rocprofv3 --pmc runs)")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the launch schedule now instead of using the "
                         "recorded one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--subgradient", type=int, default=0,
                    help="after the rounds, time this many iterations of "
                         "the subgradient-descent refinement (exact LPs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the multi-GPU path (sharding "
              "instances across GPUs with an all-reduce of the per-cluster "
              "weight sums) is not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1510_00012_amd import d2
    from synth.generators import make_workload, pick_init_members

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    t0 = time.perf_counter()
    wl = make_workload(args.workload)
    if "sym" in wl or "modalities" in wl:
        bench_symbolic(args, wl, d2, torch)
        return
    K, m = wl["K"], wl["m"]
    T = args.iters or wl["T"]
    tau, T_assign = 10, 100
    N = len(wl["offsets"]) - 1
    log(f"[bench] workload {args.workload}: N={N} n={wl['offsets'][-1]} "
        f"K={K} m={m} d={wl['X'].shape[1]} T={T} "
        f"(generated in {time.perf_counter() - t0:.1f}s)")
    members = pick_init_members(wl["offsets"], K, m, wl["seed"])
    if args.copy_mib:
        src = torch.ones(args.copy_mib * 262144, dtype=torch.float32,
                         device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] calibration copy of {args.copy_mib} MiB done")
    # achievable-bandwidth reference: the library's plain copy kernel
    copy_gbs, copy_ms = d2.copy_probe(0, 4096, 10)
    log(f"[bench] device-copy probe: {copy_gbs:.0f} GB/s (4 GiB copy, "
        f"{copy_ms:.3f} ms)")
    stream = torch.cuda.Stream()
    ctx = d2.D2Context(0, "f32", stream=stream.cuda_stream)
    ctx.load_instances(wl["offsets"], wl["X"], wl["W"])
    ctx.centroids_init(members, m)

    sched = {}
    key = d2.schedule_key(wl["offsets"], K, m, wl["X"].shape[1])
    rec_sched = None if args.autotune else d2.tuned_schedule(key)
    if rec_sched:
        ctx.set_schedule(*rec_sched)
        sched.update(chunk=rec_sched[0], waves=rec_sched[1],
                     bucket=rec_sched[2], source="recorded")
        log(f"[bench] recorded schedule {sched} for {key}")

    def step(first):
        ctx.assign(iters=T_assign, outputs=False)
        if first and not sched:
            # schedule autotuned on the first labels (no plan cache yet)
            sched.update(ctx.autotune(iters=min(T, 20), tau=tau))
            sched["source"] = "autotuned"
            log(f"[bench] autotuned schedule {sched} for {key}")
        return ctx.barycenter(iters=T, tau=tau,
                              init=d2.D2_INIT_PRODUCT if first
                              else d2.D2_INIT_CACHED)

    for w in range(args.warmup):
        step(w == 0)
        log(f"[bench] warmup round {w} done")
    # timed rounds: the barycenter call replays its captured HIP graph
    bary_ms = []
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for s in range(args.steps):
        st = step(args.warmup == 0 and s == 0)
        bary_ms.append(st["ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    graphed = bool(st["graph"])
    # per-kernel durations: further rounds with every launch bracketed by
    # HIP events on the context's stream (kernels inside a replayed graph
    # cannot be bracketed individually)
    ev_pairs, all_pairs = ctx.assign_pairs()
    costed_pairs = ctx.assign_pairs_costed()
    ctx.set_profiling(True)
    ctx.kernel_stats(reset=True)
    for _ in range(args.profile_rounds):
        step(False)
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    ks = ctx.kernel_stats(reset=True)
    log(f"[bench] timed {args.steps} rounds in {elapsed:.3f}s (graph="
        f"{graphed}); per-kernel ({args.profile_rounds} profiled rounds): "
        + ", ".join(f"{k}={v[1]:.2f}ms/{v[0]}" for k, v in ks.items()))

    ms_step = 1000.0 * elapsed / args.steps
    value = N * T * args.steps / elapsed
    src_hash = kernel_source_hash()
    esz = 4

    def roof(kind):
        launches, tot = ks[kind]
        avg_s = tot / launches / 1000.0
        if kind == "assign":
            ach = assign_exps(wl, K, m, T_assign,
                              ev_pairs / all_pairs if all_pairs else 1.0
                              ) / avg_s / 1e9
            return {"bound": "alu", "achieved": ach, "peak": EXP_PEAK_GOPS,
                    "unit": "Gexp/s", "frac": ach / EXP_PEAK_GOPS,
                    "traffic": None, "kernel": "k_assign",
                    "avg_launch_ms": 1000 * avg_s}
        b = algorithmic_bytes(kind, wl, m, esz)
        ach = b / avg_s / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "copy_probe_gbs": copy_gbs,
                "frac_of_copy_probe": ach / copy_gbs,
                "traffic": load_traffic("k_iter_ba", args.workload, src_hash),
                "kernel": "k_iter_ba", "avg_launch_ms": 1000 * avg_s,
                "bytes_per_launch": b}

    dominant = max(ks.items(), key=lambda kv: kv[1][1])[0] if ks else None
    rec = {
        "metric": "B-ADMM instance-iterations/s",
        "value": value,
        "unit": "instance-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: one D2-clustering round = "
                        f"assignment ({T_assign} B-ADMM transport iterations "
                        f"per instance-centroid pair) + batched barycenter "
                        f"({T} iterations, tau={tau}) over all clusters",
            "N": N, "n_support": int(wl["offsets"][-1]), "K": K, "m": m,
            "d": int(wl["X"].shape[1]), "T": T, "tau": tau,
            "T_assign": T_assign, "seed": wl["seed"],
        },
        "barycenter_inst_iter_per_s": N * T / (np.mean(bary_ms) / 1000.0),
        "barycenter_ms_mean": float(np.mean(bary_ms)),
        "barycenter_graph": graphed,
        "schedule": {"chunk_instances": sched.get("chunk"),
                     "waves_per_group": sched.get("waves"),
                     "bucketing_min_pct": sched.get("bucket"),
                     "source": sched.get("source")},
        "assign_pairs_evaluated_frac": (ev_pairs / all_pairs
                                        if all_pairs else None),
        "assign_pairs_costed_frac": (costed_pairs / all_pairs
                                     if all_pairs else None),
        "kernel_timing": "HIP events around each launch on the context "
                         f"stream, {args.profile_rounds} host-issued rounds "
                         "after the timed rounds",
        "kernel_ms": {k: {"launches": v[0], "total_ms": v[1]}
                      for k, v in ks.items()},
        "roofline": roof(dominant) if dominant else None,
        "roofline_plan_update": roof("iter_ba") if "iter_ba" in ks else None,
        "kernel_source_hash": src_hash,
    }
    if not args.no_cpu_baseline:
        Xc, Wc = ctx.centroids_get()
        labels = ctx.labels_get()
    if args.subgradient:
        rec["subgradient"] = time_subgradient(ctx, N, args.subgradient)
        log(f"[bench] subgradient: {rec['subgradient']}")
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 CPU oracle on slices of the workload")
        rec["cpu_baseline"] = cpu_baseline(wl, Xc, Wc, labels, T, tau,
                                           T_assign,
                                           target_s=args.cpu_seconds)
        log(f"[bench] cpu baseline: {rec['cpu_baseline']['sample']}")
    ctx.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

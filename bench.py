#!/usr/bin/env python3
"""Benchmark of the B-ADMM / D2-clustering hot path on one MI355X.

One step = one round of D2-clustering over the whole synthetic workload:
the assignment step (B-ADMM transport against every centroid) followed by
the batched B-ADMM barycenter update of all K clusters (T iterations,
support update every tau, cached-plan warm start).  Default workload: K=16
clusters, N=65,536 colour-like ragged instances (m_k uniform in [4,16]),
d=3, centroid support m=16, T=100, 10 rounds (1 warm-up + 9 timed).

value  = N * T * steps / (wall time of the timed steps): B-ADMM
         instance-iterations per second of whole rounds (assignment time
         included), inputs resident in HBM.
Also reported: the barycenter-only rate, per-kernel HIP-event times, the
roofline of the dominant kernel (and of the plan-update kernel), and the FP64
CPU oracle timed on a bounded sample of the same workload.
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
    for f in ("d2_kernels.hpp", "d2_api.hip"):
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


def cpu_baseline(wl, Xc, Wc, T, tau, T_assign, target_s=15.0):
    """The FP64 oracle on a bounded sample of the workload: one round
    (assignment of the sample, then B-ADMM per cluster of the sample)."""
    import oracle
    oracle.build(force=False)
    off, X, W = wl["offsets"], wl["X"], wl["W"]
    N = len(off) - 1

    def sub(idx):
        sizes = off[idx + 1] - off[idx]
        o = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        rows = np.concatenate([np.arange(off[k], off[k + 1]) for k in idx])
        return {"offsets": o, "X": X[rows], "W": W[rows]}

    def run(S):
        idx = np.linspace(0, N - 1, S).astype(np.int64)
        sw = sub(idx)
        t0 = time.perf_counter()
        lab, _, _ = oracle.assign(sw, Xc, Wc, T=T_assign)
        t1 = time.perf_counter()
        for c in range(len(Wc)):
            mem = np.nonzero(lab == c)[0]
            if len(mem):
                oracle.barycenter(sw, mem, Xc[c], Wc[c], T=T, tau=tau)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    pa, pb = run(512)
    per = (pa + pb) / 512
    S = int(min(N, max(512, target_s / max(per, 1e-9))))
    ta, tb = run(S)
    return {"value": S * T / (ta + tb), "unit": "instance-iterations/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{S} of {N} instances (evenly spaced), one round: "
                      f"assignment ({T_assign} it/pair, {ta:.1f}s) + "
                      f"barycenter per cluster ({T} it, {tb:.1f}s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=9)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gmm_d3_n65536_k16")
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
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
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
        log("[bench] timing the FP64 CPU oracle on a sample")
        rec["cpu_baseline"] = cpu_baseline(wl, Xc, Wc, T, tau, T_assign,
                                           target_s=args.cpu_seconds)
    ctx.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

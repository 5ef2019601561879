"""Summarise rocprofv3 output into the short text records kept in profiles/.

Usage (after the rocprofv3 runs, on any machine):
  python -m paper_1510_00012_amd.profiling trace  <kernel_stats.csv> <out.md> <cmd>
  python -m paper_1510_00012_amd.profiling counters <counter.csv> <out.md> \
      <cmd> <kernel substrings, comma separated>
  python -m paper_1510_00012_amd.profiling traffic <fetch_counter.csv> \
      <write_counter.csv> <kernel-substring> <workload> <copy_mib> <out.json> \
      <cmd> [dispatches per timed launch]

`traffic` scales the per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the
kernel by the factor that makes the same counters match a plain device copy
of known size recorded in the same run (the library's copy probe, which the
bench runs with 4096 MiB; else the bench's --copy-mib runtime copy), and
records the hash of the kernel sources so that a stale record is ignored.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash():
    h = hashlib.sha256()
    # the device code of the plan-update and auxiliary kernels
    for f in ("d2_kernels.hpp", "d2_kinst.hpp"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def trace_summary(stats_csv, out_md, cmd):
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [
        "# rocprofv3 kernel-trace summary",
        "",
        f"Command: `{cmd}`",
        "",
        f"Kernel source hash: `{kernel_source_hash()}`",
        "",
        "| kernel | calls | avg us | min us | max us | total ms | % |",
        "|---|---|---|---|---|---|---|",
    ]
    for r in rows:
        lines.append(
            f"| `{r['Name'][:90]}` | {r['Calls']} | "
            f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
            f"{float(r['MaxNs']) / 1e3:.2f} | "
            f"{float(r['TotalDurationNs']) / 1e6:.3f} | {r['Percentage']} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_kernel(counter_csv, counter):
    agg = defaultdict(list)
    for r in csv.DictReader(open(counter_csv)):
        if r["Counter_Name"] == counter:
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def traffic(fetch_csv, write_csv, kernel_sub, workload, copy_mib, out_json,
            cmd, group=1):
    """group: dispatches of the kernel that make one unit of the bench's
    per-launch timing (the slot-bucket launches of one B-ADMM iteration
    are timed together), so the bytes are per group of dispatches.
    kernel_sub may list several comma-separated substrings: the first names
    the kernel that every unit launches (its dispatches count the units),
    the others kernels launched within some units (the matrix-core passes
    beside the plan-update kernel), whose bytes are added to those units."""
    group = int(group)
    subs = [k for k in kernel_sub.split(",") if k]
    copy_kib = float(copy_mib) * 1024.0
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")

    def copy_value(agg):
        # the calibration copy: the library's copy probe (every dispatch
        # moves copy_mib MiB; median), else the largest runtime copy
        vals = sorted(v for k, vs in agg.items() if "k_copy_probe" in k
                      for v in vs)
        if vals:
            return vals[len(vals) // 2]
        vals = [v for k, vs in agg.items() if "copyBuffer" in k for v in vs]
        return max(vals) if vals else None

    cf, cw = copy_value(fetch), copy_value(write)
    sf = copy_kib / cf if cf else None
    sw = copy_kib / cw if cw else None

    def kern(agg):
        prim = [v for k, vs in agg.items() if subs[0] in k for v in vs]
        allv = [v for k, vs in agg.items() if any(q in k for q in subs)
                for v in vs]
        return group * sum(allv) / len(prim) if prim else None

    kf, kw = kern(fetch), kern(write)
    rec = {
        "kernel": subs[0],
        "kernels_summed": subs,
        "dispatches_per_launch": group,
        "workload": workload,
        "command": cmd,
        "kernel_source_hash": kernel_source_hash(),
        "fetch_kib_per_dispatch_raw": kf,
        "write_kib_per_dispatch_raw": kw,
        "copy_probe_mib": float(copy_mib),
        "copy_fetch_kib_raw": cf,
        "copy_write_kib_raw": cw,
        "fetch_scale": sf,
        "write_scale": sw,
        "hbm_bytes_per_launch": (kf * sf + kw * sw) * 1024.0
        if None not in (kf, kw, sf, sw) else None,
        "read_bytes_per_launch": kf * sf * 1024.0 if kf and sf else None,
        "write_bytes_per_launch": kw * sw * 1024.0 if kw and sw else None,
    }
    json.dump(rec, open(out_json, "w"), indent=1)
    return rec


def counters(counter_csv, out_md, cmd, kernels, cu_num=256, simd_per_cu=4):
    """Per-kernel averages of the counters of one rocprofv3 --pmc run and
    the derived utilisations: MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES /
    (GRBM_GUI_ACTIVE * SIMDs), VALU busy = SQ_ACTIVE_INST_VALU / (CUs *
    GRBM_GUI_ACTIVE) (the definitions rocprofv3 lists for MfmaUtil and
    VALUBusy).  kernels: comma-separated substrings of the kernels kept."""
    subs = [k for k in kernels.split(",") if k]
    agg = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(counter_csv)):
        name = r["Kernel_Name"]
        if subs and not any(k in name for k in subs):
            continue
        agg[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for v in agg.values() for c in v})
    lines = ["# rocprofv3 counter summary", "", f"Command: `{cmd}`", "",
             f"Kernel source hash: `{kernel_source_hash()}`", "",
             "| kernel | dispatches | " + " | ".join(names) +
             " | MFMA busy % | VALU busy % |",
             "|---" * (len(names) + 4) + "|"]
    rows = {}
    for k in sorted(agg):
        av = {c: sum(v) / len(v) for c, v in agg[k].items()}
        n = max(len(v) for v in agg[k].values())
        g = av.get("GRBM_GUI_ACTIVE")
        mf = (100.0 * av["SQ_VALU_MFMA_BUSY_CYCLES"] / (g * cu_num * simd_per_cu)
              if g and "SQ_VALU_MFMA_BUSY_CYCLES" in av else None)
        vb = (100.0 * av["SQ_ACTIVE_INST_VALU"] / (cu_num * g)
              if g and "SQ_ACTIVE_INST_VALU" in av else None)
        rows[k] = {"dispatches": n, **av, "mfma_busy_pct": mf,
                   "valu_busy_pct": vb}
        fmt = lambda v: "-" if v is None else f"{v:.4g}"
        lines.append(f"| `{k[:80]}` | {n} | " +
                     " | ".join(fmt(av.get(c)) for c in names) +
                     f" | {fmt(mf)} | {fmt(vb)} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    return rows


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace_summary(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(*sys.argv[2:]), indent=1))
    elif sys.argv[1] == "counters":
        counters(*sys.argv[2:6])
    else:
        raise SystemExit(__doc__)

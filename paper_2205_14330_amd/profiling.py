"""Summaries of rocprofv3 output for the renderer's kernels.

kernel_stats():  per-kernel call count and average/min/max duration from a
                 ``--kernel-trace --stats`` run (``*_kernel_stats.csv``).
pmc_traffic():   HBM bytes per launch from two ``--pmc FETCH_SIZE`` and
                 ``--pmc WRITE_SIZE`` runs (``*_counter_collection.csv``, KiB
                 per dispatch).  Each counter is scaled by what it reads for a
                 plain device copy of known size made in the same run (the
                 largest ``copyBuffer`` dispatch), so the result is in bytes
                 actually moved.

steady_stats():  per-kernel statistics from the ``*_kernel_trace.csv`` of the
                 same run, over the launches from the first backward
                 compositing launch on (set-up work such as rendering the
                 training targets comes before it), with the blend-count
                 forward variant named apart.

summary():       all of the above for the training steps of one workload, plus
                 SQ counters per dispatch and the VALU issue share, in one
                 JSON that bench.py reads while its kernel sources match.

Usage:
  python -m paper_2205_14330_amd.profiling stats <kernel_stats.csv> <out.txt> "<command>" [<kernel_trace.csv>]
  python -m paper_2205_14330_amd.profiling traffic <fetch.csv> <write.csv> <copy MiB> <out.json> "<command>"
  python -m paper_2205_14330_amd.profiling summary <workload> <kernel_trace.csv> <fetch.csv> <write.csv> <copy MiB>
                                                   <out.json> "<commands>" [<sq counters.csv> ...]
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# short names of the library's kernels (demangled prefix -> name)
KERNELS = {
    "dpr::k_project": "project",
    "dpr::k_radix_hist": "radix_hist",
    "dpr::k_radix_scatter": "radix_scatter",
    "dpr::k_scan_reduce": "scan_reduce",
    "dpr::k_scan_partials": "scan_partials",
    "dpr::k_scan_down": "scan_down",
    "dpr::k_tile_count": "tile_count",
    "dpr::k_col_segsum": "col_segsum",
    "dpr::k_col_segscan": "col_segscan",
    "dpr::k_col_finish": "col_finish",
    "dpr::k_tile_emit": "tile_emit",
    "dpr::k_composite_bwd": "composite_bwd",
    "dpr::k_composite<false, true,": "composite_fwd_count",   # forward keeping blend counts
    "dpr::k_composite<true, true,": "composite_fwd_count",
    "dpr::k_composite<": "composite_fwd",       # forward, and the backward's recompute pass
    "dpr::k_point_bwd": "point_bwd",
    "dpr::k_fill_u32": "fill",
    "dpr::k_loss_sum": "loss_sum",
    "dpr::k_loss": "loss",
    "dpr::k_upload_zero": "upload_zero",
    "dpr::k_upload": "upload",
}


def short_name(full: str) -> str:
    name = full.replace("void ", "")
    for k, v in KERNELS.items():
        if name.startswith(k):
            return v
    return name.split("(")[0][:48]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def kernel_stats(stats_csv: str):
    agg = collections.OrderedDict()
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows:
        n = short_name(r["Name"])
        e = agg.setdefault(n, {"calls": 0, "total_ns": 0.0, "min_ns": float("inf"), "max_ns": 0.0})
        e["calls"] += int(r["Calls"])
        e["total_ns"] += float(r["TotalDurationNs"])
        e["min_ns"] = min(e["min_ns"], float(r["MinNs"]))
        e["max_ns"] = max(e["max_ns"], float(r["MaxNs"]))
    for e in agg.values():
        e["avg_ns"] = e["total_ns"] / max(e["calls"], 1)
    return agg


def steady_stats(trace_csv: str):
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    first = next((int(r["Start_Timestamp"]) for r in rows if short_name(r["Kernel_Name"]) == "composite_bwd"), None)
    agg = collections.OrderedDict()
    for r in rows:
        t0 = int(r["Start_Timestamp"])
        if first is not None and t0 < first:
            continue
        d = float(int(r["End_Timestamp"]) - t0)
        e = agg.setdefault(short_name(r["Kernel_Name"]), {"calls": 0, "total_ns": 0.0, "min_ns": float("inf"),
                                                          "max_ns": 0.0})
        e["calls"] += 1
        e["total_ns"] += d
        e["min_ns"] = min(e["min_ns"], d)
        e["max_ns"] = max(e["max_ns"], d)
    for e in agg.values():
        e["avg_ns"] = e["total_ns"] / max(e["calls"], 1)
    return collections.OrderedDict(sorted(agg.items(), key=lambda kv: -kv[1]["total_ns"]))


def _table(agg):
    tot = sum(e["total_ns"] for e in agg.values())
    lines = [f"{'kernel':48s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}"]
    for n, e in agg.items():
        lines.append(f"{n:48s} {e['calls']:6d} {e['avg_ns'] / 1e3:10.2f} {e['min_ns'] / 1e3:10.2f} "
                     f"{e['max_ns'] / 1e3:10.2f} {100 * e['total_ns'] / tot:6.1f}")
    return lines


def write_stats_txt(stats_csv: str, out_txt: str, command: str, trace_csv: str = None):
    agg = kernel_stats(stats_csv)
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}", f"# kernel sources: {kernel_source_hash()}",
             "", "## all launches of the run (--stats)"] + _table(agg)
    if trace_csv:
        lines += ["", "## launches from the first backward compositing launch on (--kernel-trace)"]
        lines += _table(steady_stats(trace_csv))
    open(out_txt, "w").write("\n".join(lines) + "\n")
    return agg


def _per_dispatch(counter_csv: str):
    out = collections.defaultdict(list)
    copies = []
    for r in csv.DictReader(open(counter_csv)):
        v = float(r["Counter_Value"]) * 1024.0
        if "copyBuffer" in r["Kernel_Name"]:
            copies.append(v)
        out[short_name(r["Kernel_Name"])].append(v)
    return out, copies


def pmc_traffic(fetch_csv: str, write_csv: str, copy_mib: float):
    f, fc = _per_dispatch(fetch_csv)
    w, wc = _per_dispatch(write_csv)
    known = copy_mib * (1 << 20)
    f_scale = known / max(fc) if fc else 1.0
    w_scale = known / max(wc) if wc else 1.0
    res = {}
    for k in sorted(set(f) | set(w)):
        fb = sum(f.get(k, [0])) / max(len(f.get(k, [])), 1) * f_scale
        wb = sum(w.get(k, [0])) / max(len(w.get(k, [])), 1) * w_scale
        res[k] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                  "dispatches": max(len(f.get(k, [])), len(w.get(k, [])))}
    return res, f_scale, w_scale


# MI355X: 256 CUs x 4 SIMDs; a wave64 VALU instruction with VGPR operands
# issues every 2 clocks per SIMD at most, at the published 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 2.0       # wave64 VALU instructions per second


def _counter_rows(counter_csv: str):
    """Per dispatch: (dispatch id, short kernel name, {counter: value})."""
    by = collections.OrderedDict()
    for r in csv.DictReader(open(counter_csv)):
        did = int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0)
        e = by.setdefault(did, [short_name(r["Kernel_Name"]), {}])
        e[1][r["Counter_Name"]] = e[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [(d, v[0], v[1]) for d, v in sorted(by.items())]


def _steady(rows):
    """The dispatches from the first backward compositing launch on (the
    set-up renders of the training targets come before it)."""
    first = next((i for i, (_, name, _) in enumerate(rows) if name == "composite_bwd"), 0)
    return rows[first:]


def _mean_counters(rows):
    acc = collections.OrderedDict()
    for _, name, vals in rows:
        e = acc.setdefault(name, {"dispatches": 0})
        e["dispatches"] += 1
        for k, v in vals.items():
            e[k] = e.get(k, 0.0) + v
    for e in acc.values():
        n = e["dispatches"]
        for k in list(e):
            if k != "dispatches":
                e[k] /= n
    return acc


def summary(workload: str, trace_csv: str, fetch_csv: str, write_csv: str, sq_csvs, copy_mib: float,
            commands: str, out_json: str):
    """One JSON per workload: for each kernel, over the launches of the
    training steps (from the first backward compositing launch on), the
    average duration (kernel trace), the HBM bytes per launch (FETCH_SIZE and
    WRITE_SIZE in KiB per dispatch, each scaled by what it reads for the
    run's device copy of copy_mib MiB) and the SQ counters per dispatch, with
    the VALU issue share: SQ_INSTS_VALU over the duration at the peak issue
    rate of one wave64 VALU instruction per 2 clocks per SIMD."""
    stats = steady_stats(trace_csv)
    kern = collections.OrderedDict()
    for name, e in stats.items():
        kern[name] = {"calls": e["calls"], "avg_us": round(e["avg_ns"] / 1e3, 3)}
    known = copy_mib * (1 << 20)
    scales = {}
    for label, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _counter_rows(path)
        copies = [v.get("FETCH_SIZE" if label == "fetch" else "WRITE_SIZE", 0.0) * 1024.0
                  for _, n, v in rows if "copyBuffer" in n]
        scale = known / max(copies) if copies else 1.0
        scales[label] = scale
        for name, e in _mean_counters(_steady(rows)).items():
            if name in kern:
                b = e.get("FETCH_SIZE" if label == "fetch" else "WRITE_SIZE", 0.0) * 1024.0 * scale
                kern[name][f"{label}_bytes"] = round(b, 1)
    for k in kern.values():
        if "fetch_bytes" in k or "write_bytes" in k:
            k["bytes_per_launch"] = round(k.get("fetch_bytes", 0.0) + k.get("write_bytes", 0.0), 1)
    for path in sq_csvs:
        for name, e in _mean_counters(_steady(_counter_rows(path))).items():
            if name in kern:
                for c, v in e.items():
                    if c != "dispatches":
                        kern[name][c] = round(v, 1)
    for k in kern.values():
        if "SQ_INSTS_VALU" in k and k["avg_us"] > 0:
            k["valu_issue_pct"] = round(100.0 * k["SQ_INSTS_VALU"] / (k["avg_us"] * 1e-6 * VALU_ISSUE_PEAK), 1)
        if "SQ_INSTS_SALU" in k and "SQ_WAVES" in k and k["SQ_WAVES"] > 0:
            k["salu_per_wave"] = round(k["SQ_INSTS_SALU"] / k["SQ_WAVES"], 1)
    doc = {"workload": workload, "commands": commands, "source_hash": kernel_source_hash(),
           "fetch_scale": scales.get("fetch"), "write_scale": scales.get("write"),
           "scope": "launches from the first backward compositing launch on (the training steps)",
           "kernels": kern}
    json.dump(doc, open(out_json, "w"), indent=1)
    return doc


def main(argv):
    if len(argv) >= 4 and argv[0] == "stats":
        agg = write_stats_txt(argv[1], argv[2], argv[3], argv[4] if len(argv) >= 5 else None)
        print(json.dumps({k: round(v["avg_ns"] / 1e3, 2) for k, v in agg.items()}))
    elif len(argv) >= 6 and argv[0] == "traffic":
        res, fs, ws = pmc_traffic(argv[1], argv[2], float(argv[3]))
        doc = {"command": argv[5], "source_hash": kernel_source_hash(), "fetch_scale": fs, "write_scale": ws,
               "kernels": {k: {kk: round(vv, 1) if isinstance(vv, float) else vv for kk, vv in v.items()}
                           for k, v in res.items()}}
        json.dump(doc, open(argv[4], "w"), indent=1)
        print(f"fetch scale {fs:.3f}, write scale {ws:.3f}")
    elif len(argv) >= 8 and argv[0] == "summary":
        # summary <workload> <trace csv> <fetch csv> <write csv> <copy MiB> <out json> "<commands>" [sq csv ...]
        doc = summary(argv[1], argv[2], argv[3], argv[4], argv[8:], float(argv[5]), argv[7], argv[6])
        for name, k in list(doc["kernels"].items())[:8]:
            print(name, {kk: vv for kk, vv in k.items() if kk in ("avg_us", "bytes_per_launch", "valu_issue_pct",
                                                                  "salu_per_wave")})
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))

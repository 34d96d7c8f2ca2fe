"""Summaries of rocprofv3 output for the profiles/ folder.

  python -m paper_2510_01764_amd.profile_summary stats <rocprof dir> <out.txt> --command "..."
      per-kernel call count and duration statistics (from --kernel-trace --stats), with the
      median dispatch duration from the kernel trace
  python -m paper_2510_01764_amd.profile_summary valu <pmc dir> <out.json> --kernel "..." --command "..."
      vector-ALU instructions per launch of one kernel from an SQ_INSTS_VALU counter run
      (wave-level instructions; each is 64 lane operations).
  python -m paper_2510_01764_amd.profile_summary lanes <pmc dir> <valu.json> --kernel "..." --command "..."
      adds to a valu summary the mean active lanes per VALU instruction, from an
      SQ_THREAD_CYCLES_VALU / SQ_ACTIVE_INST_VALU counter run of the same kernel.
  python -m paper_2510_01764_amd.profile_summary counters <out.json> --kernel "..." --sources a.hip,b.h
      --pass <pmc dir> "<command>" [--pass ...]
      every counter of the runs averaged per dispatch of one kernel, with instructions per wave,
      active lanes per VALU instruction and LDS bank-conflict cycles per LDS-active cycle.
  python -m paper_2510_01764_amd.profile_summary traffic <fetch dir> <write dir> <out.json>
      --calib-bytes N --kernel "step_fused_kernel<256, true, false, false>" --command-fetch "..." --command-write "..."
      HBM bytes per launch of one kernel from FETCH_SIZE and WRITE_SIZE counter runs, each
      scaled by what the same counter reads for the calibration copy kernel of known size.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _find(d, pattern):
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise SystemExit(f"no {pattern} under {d}")
    return hits


def stats(d, out, command):
    rows = []
    for f in _find(d, "*kernel_stats.csv"):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    def short(name):
        # namespace prefix and argument list dropped; template arguments kept
        name = name.replace("void ", "", 1).replace("octax::(anonymous namespace)::", "")
        depth = 0
        for i, ch in enumerate(name):
            depth += (ch == "<") - (ch == ">")
            if ch == "(" and depth == 0:
                return name[:i]
        return name

    # per-dispatch durations from the kernel trace, for the median (the mean
    # also holds the autotuner's and the warm-up's launches of the same kernel)
    durations = defaultdict(list)
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                durations[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))

    def median_us(name):
        v = sorted(durations.get(name, []))
        if not v:
            return float("nan")
        m = len(v) // 2
        return (v[m] if len(v) % 2 else (v[m - 1] + v[m]) / 2) / 1e3

    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}", "",
             f"{'kernel':<56} {'calls':>6} {'avg_us':>10} {'median_us':>10} {'min_us':>10} {'max_us':>10} "
             f"{'total_ms':>10} {'pct':>6}"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"{short(r['Name'])[:56]:<56} {int(r['Calls']):>6} {float(r['AverageNs'])/1e3:>10.1f} "
                     f"{median_us(r['Name']):>10.1f} "
                     f"{float(r['MinNs'])/1e3:>10.1f} {float(r['MaxNs'])/1e3:>10.1f} "
                     f"{float(r['TotalDurationNs'])/1e6:>10.2f} {float(r['Percentage']):>6.2f}")
    text = "\n".join(lines) + "\n"
    with open(out, "w") as fh:
        fh.write(text)
    print(text)


def _counter_means(d, counter):
    per = defaultdict(list)
    for f in _find(d, "*counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in per.items()}


def _pick(means, needle):
    hits = [k for k in means if needle in k]
    if len(hits) != 1:
        raise SystemExit(f"kernel '{needle}' matches {hits}")
    return means[hits[0]]


def traffic(fetch_dir, write_dir, out, calib_bytes, kernel, cmd_f, cmd_w, sources=None):
    sys.path.insert(0, ROOT)
    import bench
    f = _counter_means(fetch_dir, "FETCH_SIZE")
    w = _counter_means(write_dir, "WRITE_SIZE")
    cf, _ = _pick(f, "octax_calib_copy_kernel")
    cw, _ = _pick(w, "octax_calib_copy_kernel")
    kf, nf = _pick(f, kernel)
    kw, nw = _pick(w, kernel)
    scale_f = calib_bytes / (cf * 1024.0)
    scale_w = calib_bytes / (cw * 1024.0)
    fetch_b = kf * 1024.0 * scale_f
    write_b = kw * 1024.0 * scale_w
    d = {
        "kernel": kernel,
        "kernel_source_hash": source_hash(sources) if sources else bench.kernel_source_hash(),
        **({"sources": sources} if sources else {}),
        "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw,
        "dispatches": [nf, nw],
        "calib_copy_bytes": calib_bytes,
        "calib_fetch_kib": cf, "calib_write_kib": cw,
        "scale_fetch": scale_f, "scale_write": scale_w,
        "hbm_fetch_bytes_per_launch": fetch_b,
        "hbm_write_bytes_per_launch": write_b,
        "hbm_bytes_per_launch": fetch_b + write_b,
        "command_fetch": cmd_f, "command_write": cmd_w,
    }
    with open(out, "w") as fh:
        json.dump(d, fh, indent=1)
    print(json.dumps(d, indent=1))


def valu(d, out, kernel, command):
    sys.path.insert(0, ROOT)
    import bench
    v = _counter_means(d, "SQ_INSTS_VALU")
    insts, n = _pick(v, kernel)
    res = {
        "kernel": kernel,
        "kernel_source_hash": bench.kernel_source_hash(),
        "valu_insts_per_dispatch": insts, "dispatches": n,
        "valu_lane_ops_per_launch": insts * 64,
        "command": command,
    }
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


def lanes(d, out, kernel, command):
    """Active lanes per VALU instruction = thread-cycles / instruction-cycles
    (both counted per VALU instruction issue), into the existing summary."""
    sys.path.insert(0, ROOT)
    import bench
    thr, n = _pick(_counter_means(d, "SQ_THREAD_CYCLES_VALU"), kernel)
    ins, _ = _pick(_counter_means(d, "SQ_ACTIVE_INST_VALU"), kernel)
    with open(out) as fh:
        res = json.load(fh)
    if res.get("kernel_source_hash") != bench.kernel_source_hash():
        raise SystemExit(f"{out} was taken on another kernel source; take the VALU counters again first")
    res.update({"thread_cycles_valu_per_dispatch": thr, "active_inst_valu_per_dispatch": ins,
                "lane_dispatches": n, "valu_active_lanes": thr / ins, "active_lane_fraction": thr / ins / 64,
                "command_lanes": command})
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


def source_hash(files):
    """The same digest as bench.kernel_source_hash, over the named csrc files."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2510_01764_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counters(out, kernel, sources, passes):
    """Every counter of the given counter-run directories, averaged per
    dispatch of one kernel, with the ratios the roofline discussion uses:
    instructions of each kind per wave, the mean active lanes per VALU
    instruction, LDS bank-conflict cycles per LDS-active cycle.  `passes` is
    a list of (directory, command) pairs."""
    res = {"kernel": kernel, "kernel_source_hash": source_hash(sources), "sources": sources,
           "per_dispatch": {}, "dispatches": {}, "commands": []}
    for d, cmd in passes:
        res["commands"].append(cmd)
        names = set()
        for f in _find(d, "*counter_collection.csv"):
            with open(f) as fh:
                names |= {r["Counter_Name"] for r in csv.DictReader(fh)}
        for n in sorted(names):
            mean, cnt = _pick(_counter_means(d, n), kernel)
            res["per_dispatch"][n] = mean
            res["dispatches"][n] = cnt
    c = res["per_dispatch"]
    waves = c.get("SQ_WAVES")
    derived = {}
    if waves:
        for n in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_SMEM", "SQ_INSTS_VMEM_RD",
                  "SQ_INSTS_VMEM_WR"):
            if n in c:
                derived[n.replace("SQ_INSTS_", "").lower() + "_per_wave"] = c[n] / waves
    if "SQ_THREAD_CYCLES_VALU" in c and c.get("SQ_ACTIVE_INST_VALU"):
        derived["active_lane_fraction"] = c["SQ_THREAD_CYCLES_VALU"] / c["SQ_ACTIVE_INST_VALU"] / 64
    if c.get("SQ_LDS_IDX_ACTIVE"):
        derived["lds_bank_conflict_per_active_cycle"] = c.get("SQ_LDS_BANK_CONFLICT", 0.0) / c["SQ_LDS_IDX_ACTIVE"]
    if c.get("SQ_INSTS_VALU"):
        derived["valu_lane_ops_per_launch"] = c["SQ_INSTS_VALU"] * 64
    res["derived"] = derived
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("out")
    t.add_argument("--calib-bytes", type=int, required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--sources", default=None,
                   help="comma-separated csrc files the kernel is built from (default: the fused kernel's)")
    v = sub.add_parser("valu")
    v.add_argument("dir")
    v.add_argument("out")
    v.add_argument("--kernel", required=True)
    v.add_argument("--command", required=True)
    ln = sub.add_parser("lanes")
    ln.add_argument("dir")
    ln.add_argument("out")
    ln.add_argument("--kernel", required=True)
    ln.add_argument("--command", required=True)
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("--kernel", required=True)
    c.add_argument("--sources", required=True, help="comma-separated csrc files the kernel is built from")
    c.add_argument("--pass", dest="passes", action="append", nargs=2, metavar=("DIR", "COMMAND"), required=True)
    a = ap.parse_args()
    if a.cmd == "counters":
        counters(a.out, a.kernel, a.sources.split(","), [tuple(x) for x in a.passes])
    elif a.cmd == "stats":
        stats(a.dir, a.out, a.command)
    elif a.cmd == "valu":
        valu(a.dir, a.out, a.kernel, a.command)
    elif a.cmd == "lanes":
        lanes(a.dir, a.out, a.kernel, a.command)
    else:
        traffic(a.fetch_dir, a.write_dir, a.out, a.calib_bytes, a.kernel, a.command_fetch, a.command_write,
                a.sources.split(",") if a.sources else None)


if __name__ == "__main__":
    main()

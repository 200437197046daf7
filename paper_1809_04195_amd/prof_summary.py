"""Summaries of rocprofv3 output for the kernels of this library.

    # HBM bytes per launch from two counter runs of the same command (FETCH_SIZE, then
    # WRITE_SIZE), calibrated on the 1 GiB device copy that `bench.py --copy-probe` makes,
    # optionally over the launches of the n-th interval the library timed
    python -m paper_1809_04195_amd.prof_summary traffic --fetch DIR --write DIR \\
        --workload vol320_256x256_c8_t80_k4 --schedule 0,1 [--window 1] --out profiles/hbm_traffic_<workload>.json

    # per-kernel-family averages and utilisation metrics of one or more counter runs
    python -m paper_1809_04195_amd.prof_summary counters DIR [DIR ...]

    # markdown table of a --kernel-trace --stats run (csv or rocpd database output),
    # optionally from the N-th dispatch of a named kernel on, or only the launches of the
    # n-th interval the library timed (t2s_profile_enable on .. off)
    python -m paper_1809_04195_amd.prof_summary stats DIR [--after k_project:2] [--window 1]

DIR is a rocprofv3 output directory (or the CSV file itself).  Utilisation metrics
follow rocprofv3's own derived-metric definitions on MI355X (256 CUs, 1024 SIMDs,
8 XCDs; GRBM_GUI_ACTIVE is reported summed over the XCDs, so one XCD's active cycles
are a eighth of it).
"""

from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import sys

CU_NUM, SIMD_NUM, XCD_NUM = 256, 1024, 8
COPY_PROBE_BYTES = 1 << 30

FAMILIES = (
    ("k_passA", "pass_a"), ("k_passB_inv", "passB_inv"), ("k_passB", "pass_b"), ("k_llr_finalize", "llr_finalize"), ("k_llr", "llr_admm"), ("k_project", "load_project"),
    ("k_init", "init"), ("k_set_state", "set_state"), ("copyBuffer", "copy"),
    ("k_conv", "unet_conv"), ("k_wgrad_reduce", "unet_wgrad_reduce"), ("k_wgrad", "unet_wgrad"),
    ("k_adam", "unet_adam"), ("k_pool_bwd", "unet_pool_bwd"), ("k_pool", "unet_pool"), ("k_unshuffle", "unet_unshuffle"),
    ("k_unpack", "unet_unpack"), ("k_pack", "unet_pack"), ("k_bias", "unet_bias"), ("k_relu", "unet_relu_bwd"),
    ("k_mse", "unet_mse"), ("k_prep", "unet_prep"), ("k_slice_scale", "unet_scale"),
)


def family(name):
    # k_passC<L, MODE, M>: MODE 1 is the adjoint of the load step, 0 the normal operator
    # of apply_normal / set_initial, 2 the CG step
    if "k_passC<" in name:
        args = name.split("k_passC<", 1)[1].split(">", 1)[0].split(",")
        if len(args) > 1 and args[1].strip() == "1":
            return "passC_adjoint"
        return "pass_c"
    for key, fam in FAMILIES:
        if key in name:
            return fam
    return name.split("(")[0][:48]


def _csv(path, suffix):
    if os.path.isdir(path):
        hits = sorted(glob.glob(os.path.join(path, "**", f"*{suffix}"), recursive=True))
        if not hits:
            raise FileNotFoundError(f"no *{suffix} under {path}")
        return hits[0]
    return path


def dispatches(path):
    """[(dispatch id, family, {counter: value})] in dispatch order."""
    d = collections.OrderedDict()
    for r in csv.DictReader(open(_csv(path, "counter_collection.csv"))):
        i = int(r["Dispatch_Id"])
        if i not in d:
            d[i] = (family(r["Kernel_Name"]), {})
        d[i][1][r["Counter_Name"]] = float(r["Counter_Value"])
    return sorted((i, f, c) for i, (f, c) in d.items())


def copy_probe(fetch_path, write_path):
    """(FETCH_SIZE, WRITE_SIZE) of the copy probe: the device copy whose WRITE_SIZE is
    closest to 1 GiB; both runs execute the same program, so its dispatch id is the
    same in the FETCH_SIZE run."""
    wd = {i: c["WRITE_SIZE"] for i, f, c in dispatches(write_path) if f == "copy"}
    fd = {i: c["FETCH_SIZE"] for i, f, c in dispatches(fetch_path) if f == "copy"}
    i = min(wd, key=lambda j: abs(wd[j] * 1024.0 - COPY_PROBE_BYTES))
    if abs(wd[i] * 1024.0 - COPY_PROBE_BYTES) > 0.05 * COPY_PROBE_BYTES:
        raise RuntimeError("no 1 GiB copy probe in the WRITE_SIZE run")
    return fd[i], wd[i]


def _window_ids(rows, window):
    """Dispatch-id range of the n-th interval between k_profile_mark dispatches (all when
    window is 0)."""
    if not window:
        return 0, 1 << 62
    marks = sorted({int(r["Dispatch_Id"]) for r in rows if "k_profile_mark" in r["Kernel_Name"]})
    if len(marks) < 2 * window:
        raise ValueError(f"fewer than {2 * window} profile marks")
    return marks[2 * window - 2], marks[2 * window - 1]


def read_counters(path, window=0):
    """{family: {"n": dispatches, "dur_ns": mean duration, counter: mean value}}, over the
    dispatches of the n-th timed interval when window = n > 0."""
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    disp = collections.defaultdict(dict)
    rows = list(csv.DictReader(open(_csv(path, "counter_collection.csv"))))
    lo, hi = _window_ids(rows, window)
    for r in rows:
        if not lo < int(r["Dispatch_Id"]) < hi:
            continue
        f = family(r["Kernel_Name"])
        vals[f][r["Counter_Name"]].append(float(r["Counter_Value"]))
        disp[f][r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), r["Kernel_Name"])
    out = {}
    for f, cs in vals.items():
        d = list(disp[f].values())
        e = {"n": len(d), "dur_ns": sum(x[0] for x in d) / len(d), "kernel": d[0][1]}
        for c, v in cs.items():
            e[c] = sum(v) / len(v)
        e["_values"] = cs
        out[f] = e
    return out


def traffic(args):
    fe = read_counters(args.fetch, args.window)
    wr = read_counters(args.write, args.window)
    fcopy, wcopy = copy_probe(args.fetch, args.write)
    fscale = COPY_PROBE_BYTES / (fcopy * 1024.0)
    wscale = COPY_PROBE_BYTES / (wcopy * 1024.0)
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "kernels.hip")
    res = {"kernels_source_sha256_16": hashlib.sha256(open(src, "rb").read()).hexdigest()[:16],
           "workload": args.workload, "schedule": args.schedule, "order": args.order, "window": args.window,
           "fetch_scale": fscale,
           "write_scale": wscale,
           "copy_probe_bytes": COPY_PROBE_BYTES, "traffic": {}}
    alg = {}
    if args.bench:
        # algorithmic bytes per launch of the same run (the bench line it printed; FILE:KEY
        # takes the kernel table of entry KEY, e.g. vol320_fixed)
        path, _, key = args.bench.partition(":")
        line = json.loads([x for x in open(path).read().splitlines() if x.startswith("{")][-1])
        alg = {k: v.get("alg_bytes_per_launch") for k, v in (line[key] if key else line)["kernels"].items()}
    for fam in ("pass_a", "pass_b", "pass_c", "llr_admm"):
        if fam in fe and fam in wr:
            rb = fe[fam]["FETCH_SIZE"] * 1024.0 * fscale
            wb = wr[fam]["WRITE_SIZE"] * 1024.0 * wscale
            e = {"bytes_per_launch": rb + wb, "read_bytes": rb, "write_bytes": wb, "launches": fe[fam]["n"],
                 "avg_ms": fe[fam]["dur_ns"] / 1e6}
            if alg.get(fam):
                e["alg_bytes_per_launch"] = alg[fam]
                e["ratio_to_alg"] = (rb + wb) / alg[fam]
            res["traffic"][fam] = e
    txt = json.dumps(res, indent=1)
    if args.out:
        open(args.out, "w").write(txt + "\n")
    print(txt)


def derived(e):
    """Utilisation metrics of one family (those whose counters were collected)."""
    m = {}
    cyc = e.get("GRBM_GUI_ACTIVE", 0.0) / XCD_NUM          # active cycles of one XCD
    if cyc <= 0:
        return m
    if "SQ_WAVE_CYCLES" in e:
        m["waves_per_cu"] = 4.0 * e["SQ_WAVE_CYCLES"] / (cyc * CU_NUM)
    if "SQ_ACTIVE_INST_VALU" in e:
        m["valu_busy_pct"] = 100.0 * e["SQ_ACTIVE_INST_VALU"] / CU_NUM / cyc
    if "SQ_ACTIVE_INST_LDS" in e:
        m["lds_busy_pct"] = 100.0 * e["SQ_ACTIVE_INST_LDS"] / CU_NUM / cyc
    if "SQ_THREAD_CYCLES_VALU" in e and e.get("SQ_ACTIVE_INST_VALU"):
        m["valu_lanes_active_pct"] = 100.0 * e["SQ_THREAD_CYCLES_VALU"] / (e["SQ_ACTIVE_INST_VALU"] * 64)
    if "SQ_WAIT_ANY" in e and e.get("SQ_WAVE_CYCLES"):
        m["wave_wait_pct"] = 100.0 * e["SQ_WAIT_ANY"] / e["SQ_WAVE_CYCLES"]
    if "SQ_WAIT_INST_ANY" in e and e.get("SQ_WAVE_CYCLES"):
        m["wave_wait_issue_pct"] = 100.0 * e["SQ_WAIT_INST_ANY"] / e["SQ_WAVE_CYCLES"]
    if "SQ_LDS_BANK_CONFLICT" in e:
        m["lds_bank_conflict_pct"] = 100.0 * e["SQ_LDS_BANK_CONFLICT"] / CU_NUM / cyc
    if "SQ_VALU_MFMA_BUSY_CYCLES" in e:
        m["mfma_busy_pct"] = 100.0 * e["SQ_VALU_MFMA_BUSY_CYCLES"] / (cyc * SIMD_NUM)
    if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in e and e["dur_ns"] > 0:
        m["mfma_bf16_tflops"] = e["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512 / e["dur_ns"] / 1e3
    m["clock_ghz"] = cyc / e["dur_ns"]
    return m


def counters(args):
    merged = collections.defaultdict(dict)
    for path in args.dirs:
        for f, e in read_counters(path).items():
            n, dur = e["n"], e["dur_ns"]
            for k, v in e.items():
                if k not in ("_values",):
                    merged[f][k] = v
            merged[f]["n"], merged[f]["dur_ns"] = n, dur
    rows = []
    for f, e in sorted(merged.items(), key=lambda kv: -kv[1]["n"] * kv[1]["dur_ns"]):
        rows.append((f, e["n"], e["dur_ns"] / 1e3, derived(e)))
    keys = sorted({k for _, _, _, m in rows for k in m})
    print("| family | dispatches | avg us | " + " | ".join(keys) + " |")
    print("|---|---|---|" + "---|" * len(keys))
    for f, n, us, m in rows:
        print(f"| {f} | {n} | {us:.1f} | " + " | ".join(f"{m[k]:.2f}" if k in m else "" for k in keys) + " |")


def _stats_rows(path, after="", window=0):
    """[(name, calls, total ns, average ns, percent)] of a --kernel-trace --stats run:
    its kernel_stats.csv (csv output) or its rocpd database (the default output).
    after = "NAME:N" keeps the dispatches from the N-th dispatch of a kernel whose name
    contains NAME on; window = n keeps those of the n-th timed interval of the library
    (between the n-th pair of k_profile_mark dispatches); database output only."""
    dbs = sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True)) if os.path.isdir(path) else (
        [path] if path.endswith(".db") else [])
    if not dbs:
        if after or window:
            raise ValueError("--after / --window need the rocpd database output")
        return [(r["Name"], int(r["Calls"]), int(r["TotalDurationNs"]), float(r["AverageNs"]),
                 float(r["Percentage"])) for r in csv.DictReader(open(_csv(path, "kernel_stats.csv")))]
    import sqlite3
    db = sqlite3.connect(dbs[0])
    t0, t1 = 0, 1 << 62
    if after:
        key, n = after.rsplit(":", 1)
        starts = [r[0] for r in db.execute("select start from kernels where instr(name, ?) > 0 order by start",
                                           (key,))]
        if len(starts) < int(n):
            raise ValueError(f"fewer than {n} dispatches of {key}")
        t0 = starts[int(n) - 1]
    if window:
        # the n-th interval between an enabling and a disabling call of t2s_profile_enable
        marks = [r[0] for r in db.execute("select start from kernels where instr(name, 'k_profile_mark') > 0 "
                                          "order by start")]
        if len(marks) < 2 * window:
            raise ValueError(f"fewer than {2 * window} profile marks")
        t0, t1 = marks[2 * window - 2], marks[2 * window - 1]
    rows = list(db.execute("select name, count(*), sum(end - start) from kernels where start >= ? and start <= ? "
                           "and instr(name, 'k_profile_mark') = 0 group by name order by sum(end - start) desc",
                           (t0, t1)))
    tot = sum(r[2] for r in rows) or 1
    return [(n, c, t, t / c, 100.0 * t / tot) for n, c, t in rows]


def stats(args):
    print("| kernel | calls | total (ns) | average (ns) | % |")
    print("|---|---|---|---|---|")
    for name, calls, total, avg, pct in _stats_rows(args.dir, args.after, args.window):
        print(f"| `{name[:90]}` | {calls} | {total} | {avg:.0f} | {pct:.2f} |")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--schedule", default="0,1")
    t.add_argument("--order", type=int, default=0)
    t.add_argument("--window", type=int, default=0,
                   help="n > 0: only the dispatches of the n-th interval the library timed")
    t.add_argument("--bench", default="",
                   help="bench.py output of the same run, FILE or FILE:KEY (algorithmic bytes per launch)")
    t.add_argument("--out", default="")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--after", default="", help="NAME:N: from the N-th dispatch of a kernel named *NAME* on")
    s.add_argument("--window", type=int, default=0,
                   help="n: the launches of the n-th interval the library timed (t2s_profile_enable on .. off)")
    args = ap.parse_args()
    {"traffic": traffic, "counters": counters, "stats": stats}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())

"""Summaries of rocprofv3 CSV output for the committed profile records.

    python3 -m paper_1412_1953_amd.profiling stats <kernel_stats.csv> <kernel_trace.csv> <out.txt> -- <command>
    python3 -m paper_1412_1953_amd.profiling traffic <kernel> <fetch.csv> <write.csv> <out.txt> [--largest] -- <command>
    python3 -m paper_1412_1953_amd.profiling counters <counters.csv>[,<more.csv>] <out.txt> <kernel>... [--largest] -- <command>
    python3 -m paper_1412_1953_amd.profiling gaps <kernel_trace.csv> <hip_api_trace.csv> <out.txt> -- <command>

`stats` lists the kernels by total time (rocprofv3 --kernel-trace --stats)
and, per kernel, the launch shapes (grid sizes) with their average duration.
`traffic` turns two counter runs (--pmc FETCH_SIZE, then --pmc WRITE_SIZE,
KiB per dispatch) into HBM bytes per launch of one kernel class, each counter
scaled by what it reads for a plain device copy of known size (the 256 MiB
copy that bench.py --copy-probe performs).  The record carries the SHA-256
of the kernel source it was measured on; bench.py reports the traffic only
while that source is unchanged.
`counters` averages every counter of --pmc runs per dispatch of each named
kernel class (a class of the library's timer or a kernel-name pattern):
derived metrics such as VALUBusy, VALUUtilization, OccupancyPercent and
LDSBankConflict, and raw ones such as SQ_WAVES or SQ_INSTS_VALU.
`gaps` reads a kernel trace with the HIP runtime trace (rocprofv3
--kernel-trace --hip-runtime-trace): the idle time of the GPU between one
restart cycle's last kernel (k_cycle_end) and the next kernel, the idle
time between consecutive kernels overall, and the host time spent in each
HIP runtime call.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SRC = os.path.join(ROOT, "paper_1412_1953_amd", "csrc", "kernels.hip")
COPY_BYTES = 1 << 28                       # bench.py --copy-probe
# kernel classes of the library's timer -> kernel-name pattern
CLASS_PATTERN = {
    "apply_dot": r"k_apply_dot<double",
    "axpy": r"k_axpy_pass<\d+>",
    "s1": r"k_s1_zero<double\b|k_s1_pair<double>|k_tail_down<double>",
    "s2": r"k_s2_zero<double\b|k_s2_pair<double>|k_tail_up<double>",
    "cccs_project": r"k_cccs_project<double",
    "cccs_chain": r"k_cccs_chain<double",
    "s1_fine": r"k_s1_zero<double\b",
    "s2_fine": r"k_s2_zero<double\b",
    "cccs_expand": r"k_cccs_expand<double",
}


def short(name: str) -> str:
    return re.sub(r"\(.*", "", name).strip()


def source_sha() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def stats(stats_csv, trace_csv, out, command):
    rows = list(csv.DictReader(open(stats_csv)))
    total = sum(int(r["TotalDurationNs"]) for r in rows)
    shapes = collections.defaultdict(lambda: [0, 0])
    for r in csv.DictReader(open(trace_csv)):
        key = (short(r["Kernel_Name"]), int(r["Grid_Size_X"]), int(r["Grid_Size_Y"]))
        shapes[key][0] += 1
        shapes[key][1] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    lines = [f"command: {command}", f"kernel time: {total / 1e6:.3f} ms", "",
             f"{'share':>6} {'total ms':>9} {'calls':>6} {'avg us':>8}  kernel"]
    for r in sorted(rows, key=lambda r: -int(r["TotalDurationNs"]))[:25]:
        t = int(r["TotalDurationNs"])
        lines.append(f"{100 * t / total:5.1f}% {t / 1e6:9.3f} {int(r['Calls']):6d} "
                     f"{float(r['AverageNs']) / 1e3:8.2f}  {short(r['Name'])}")
    # per timer class: mean kernel duration per launch, and the mean span of
    # its runs of consecutive launches per launch (what one event pair around
    # such a run covers, inter-kernel gaps included)
    trace = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    lines += ["", f"kernels.hip sha256: {source_sha()}",
              "timer classes (mean kernel duration per launch, and the mean span of its runs of consecutive",
              "launches per launch):",
              f"{'class':>13} {'launches':>8} {'kernel us':>10} {'run span us':>12}  kernels"]
    for kc, pat in CLASS_PATTERN.items():
        rx = re.compile(pat)
        n = busy = span = 0
        run = None
        for r in trace:
            if rx.search(r["Kernel_Name"]):
                s, e = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
                n += 1
                busy += e - s
                run = [s, e] if run is None else [run[0], e]
            elif run is not None:
                span += run[1] - run[0]
                run = None
        if run is not None:
            span += run[1] - run[0]
        if n:
            lines.append(f"{kc:>13} {n:8d} {busy / n / 1e3:10.2f} {span / n / 1e3:12.2f}  {pat}")
    lines += ["", "launch shapes (grid x, grid y in work-items):",
              f"{'calls':>6} {'avg us':>8}  kernel [grid]"]
    for (nm, gx, gy), (c, d) in sorted(shapes.items(), key=lambda x: -x[1][1])[:40]:
        lines.append(f"{c:6d} {d / c / 1e3:8.2f}  {nm} [{gx} x {gy}]")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def counter_rows(path):
    out = []
    for r in csv.DictReader(open(path)):
        out.append((short(r["Kernel_Name"]), float(r["Counter_Value"])))
    return out


def counter_rows_sized(path):
    out = []
    for r in csv.DictReader(open(path)):
        out.append((short(r["Kernel_Name"]), float(r["Counter_Value"]), int(r["Grid_Size"])))
    return out


def traffic(kclass, fetch_csv, write_csv, out, command, largest=False, name=None):
    """largest: only the dispatches of the class with the largest grid (the
    finest level of a multigrid kernel that also runs on coarser levels)."""
    pat = re.compile(CLASS_PATTERN[kclass])
    res = {}
    for label, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        sized = counter_rows_sized(path)
        if largest:
            gmax = max((gs for nm, v, gs in sized if pat.search(nm)), default=None)
            sized = [(nm, v, gs) for nm, v, gs in sized if not pat.search(nm) or gs == gmax]
        rows = [(nm, v) for nm, v, gs in sized]
        # the copy probe is the largest single dispatch of a copy kernel
        copies = [v for nm, v in rows if "copy" in nm.lower()]
        if not copies:
            raise SystemExit(f"{path}: no copy dispatch found (run bench.py --copy-probe)")
        kib_copy = max(copies)
        scale = COPY_BYTES / (kib_copy * 1024.0)
        vals = [v for nm, v in rows if pat.search(nm)]
        if not vals:
            raise SystemExit(f"{path}: no dispatch of {kclass}")
        res[label] = (sum(vals) / len(vals), len(vals), kib_copy, scale)
    fetch = res["FETCH_SIZE"][0] * 1024.0 * res["FETCH_SIZE"][3]
    write = res["WRITE_SIZE"][0] * 1024.0 * res["WRITE_SIZE"][3]
    lines = [f"command: {command}",
             f"kernel class: {kclass} ({CLASS_PATTERN[kclass]})" + (", largest grid only" if largest else ""),
             f"kernels.hip sha256: {source_sha()}"]
    for label, (avg, cnt, kib_copy, scale) in res.items():
        lines.append(f"{label}: {avg:.1f} KiB per dispatch over {cnt} dispatches; copy probe of "
                     f"{COPY_BYTES} B read {kib_copy:.1f} KiB -> scale {scale:.4f}")
    lines += [f"fetch bytes per launch: {fetch:.0f}",
              f"write bytes per launch: {write:.0f}",
              f"traffic bytes per launch: {fetch + write:.0f}"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def counters(csv_path, out, classes, command, largest=False):
    """Mean value per dispatch of every counter in csv_path for each class."""
    res = {}                               # kernel -> (VGPRs, AGPRs, SGPRs, LDS bytes, scratch bytes, workgroup)
    rows = []
    for r in (r for path in csv_path.split(",") for r in csv.DictReader(open(path))):
        nm = short(r["Kernel_Name"])
        rows.append((nm, r["Counter_Name"], float(r["Counter_Value"]), int(r["Grid_Size"]), r.get("Dispatch_Id", "")))
        res[nm] = tuple(r.get(k, "?") for k in ("VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "LDS_Block_Size",
                                                  "Scratch_Size", "Workgroup_Size"))
    names = sorted({c for _, c, _, _, _ in rows})
    lines = [f"command: {command}", f"kernels.hip sha256: {source_sha()}",
             "mean per dispatch" + (" (largest grid of each class only)" if largest else ""), ""]
    head = f"{'class':>14} {'dispatches':>10} " + " ".join(f"{c:>22}" for c in names)
    lines.append(head)
    for cl in classes:
        pat = re.compile(CLASS_PATTERN.get(cl, cl))
        sel = [r for r in rows if pat.search(r[0])]
        if largest and sel:
            gmax = max(r[3] for r in sel)
            sel = [r for r in sel if r[3] == gmax]
        if not sel:
            lines.append(f"{cl:>14} {0:>10}")
            continue
        vals = collections.defaultdict(list)
        for r in sel:
            vals[r[1]].append(r[2])
        nd = max(len(v) for v in vals.values())
        cells = [f"{sum(vals[c]) / len(vals[c]):>22.4f}" if vals[c] else f"{'-':>22}" for c in names]
        lines.append(f"{cl:>14} {nd:>10} " + " ".join(cells))
    lines += ["", "resources per kernel (VGPRs, AGPRs, SGPRs, LDS bytes, scratch bytes, workgroup size):"]
    for cl in classes:
        pat = re.compile(CLASS_PATTERN.get(cl, cl))
        for nm in sorted({r[0] for r in rows if pat.search(r[0])}):
            lines.append(f"  {nm}: {', '.join(res[nm])}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def gaps(kernel_csv, api_csv, out, command):
    with open(kernel_csv) as fh:
        ks = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"])
                    for r in csv.DictReader(fh))
    after_cycle = sorted((ks[i + 1][0] - e) / 1e3 for i, (s, e, nm) in enumerate(ks[:-1]) if "k_cycle_end" in nm)
    between = sorted(max(0, ks[i + 1][0] - ks[i][1]) / 1e3 for i in range(len(ks) - 1))
    med = lambda v: v[len(v) // 2] if v else float("nan")
    lines = [f"command: {command}", f"kernels.hip sha256: {source_sha()}",
             f"kernels traced: {len(ks)}, span {(ks[-1][1] - ks[0][0]) / 1e6:.3f} ms, "
             f"busy {sum(e - s for s, e, _ in ks) / 1e6:.3f} ms", "",
             "GPU idle time (us)          count    median       min       max",
             f"after k_cycle_end       {len(after_cycle):10d} {med(after_cycle):9.2f} "
             f"{after_cycle[0] if after_cycle else float('nan'):9.2f} "
             f"{after_cycle[-1] if after_cycle else float('nan'):9.2f}",
             f"between kernels         {len(between):10d} {med(between):9.2f} "
             f"{between[int(0.9 * len(between))] if between else float('nan'):9.2f} (p90) "
             f"{between[-1] if between else float('nan'):9.2f}", "",
             "host time in HIP runtime calls (us)", f"{'call':32s} {'count':>7s} {'total ms':>10s} {'median':>9s}"]
    agg = collections.defaultdict(list)
    with open(api_csv) as fh:
        for r in csv.DictReader(fh):
            agg[r["Function"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    for fn, v in sorted(agg.items(), key=lambda x: -sum(x[1]))[:12]:
        v.sort()
        lines.append(f"{fn:32s} {len(v):7d} {sum(v) / 1e3:10.2f} {med(v):9.2f}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main(argv):
    if "--" not in argv:
        raise SystemExit(__doc__)
    cut = argv.index("--")
    args, command = argv[:cut], " ".join(argv[cut + 1:])
    if args[0] == "stats":
        stats(args[1], args[2], args[3], command)
    elif args[0] == "traffic":
        traffic(args[1], args[2], args[3], args[4], command, largest="--largest" in args)
    elif args[0] == "counters":
        counters(args[1], args[2], [a for a in args[3:] if a != "--largest"], command,
                 largest="--largest" in args)
    elif args[0] == "gaps":
        gaps(args[1], args[2], args[3], command)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])

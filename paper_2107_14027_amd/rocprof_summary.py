"""Condense rocprofv3 CSV output into the short text summaries kept beside the
benchmark: per-kernel launch statistics, and HBM traffic per launch from the
FETCH_SIZE / WRITE_SIZE counters scaled by a plain copy of known size.

    python -m paper_2107_14027_amd.rocprof_summary stats KERNEL_STATS_CSV OUT --command CMD
    python -m paper_2107_14027_amd.rocprof_summary traffic FETCH_CSV WRITE_CSV OUTDIR \
        --calib-bytes NBYTES --command-fetch CMD --command-write CMD
    python -m paper_2107_14027_amd.rocprof_summary counters OUT --points P=N,... \
        --command CMD CSV [CSV ...]

Traffic: each counter is read per dispatch (summed over its dimension entries,
in KiB), averaged over the dispatches of one kernel instantiation, and scaled
by true_bytes / counter for the largest runtime copy dispatch in the same run
(a device-to-device copy of NBYTES reads NBYTES and writes NBYTES).
"""
import argparse
import collections
import csv
import hashlib
import os
import re
import shlex
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fused.hip", "fr_device.h", "fr_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2107_14027_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def short(name):
    m = re.search(r"(k_\w+)<(\d+), (\w+)((?:, \w+)*)>", name)
    if m:
        kern, p, t, extra = m.groups()
        # k_fused<P, T, DIAG, STG[, MF]>: STG selects the stage epilogue;
        # k_lines<P, T, HALO>: HALO forms the neighbour traces from their states
        args = [a.strip() for a in extra.split(",") if a.strip()]
        if kern == "k_fused" and len(args) >= 2 and args[1] == "true":
            kern = "k_fused_stage"
        if kern == "k_lines" and args and args[0] == "true":
            kern = "k_lines_halo"
        return "%s<%s,%s>" % (kern, p, t)
    m = re.search(r"(k_\w+)<([^>]*)>", name)
    if m:
        return "%s<%s>" % (m.group(1), m.group(2).replace(" ", ""))
    m = re.search(r"(k_\w+)\(", name)
    if m:
        return m.group(1)
    m = re.search(r"([A-Za-z_][\w:]*)[<(]", name)
    return (m.group(1) if m else name)[:56]


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))

    def col(r, *names):
        for n in names:
            if n in r and r[n] != "":
                return float(r[n])
        return 0.0
    out = ["# rocprofv3 kernel statistics: %s" % args.workload, "",
           "command: `%s`" % args.command, "",
           "summary: `python3 -m paper_2107_14027_amd.rocprof_summary %s`" % shlex.join(sys.argv[1:]), "",
           "| kernel | calls | total ms | mean us | min us | max us | % |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        pct = col(r, "Percentage", "Percent (Inc)")
        if pct < args.min_percent:
            continue
        out.append("| %s | %d | %.3f | %.1f | %.1f | %.1f | %.1f |" % (
            short(r["Name"]), int(col(r, "Calls")),
            col(r, "TotalDurationNs", "Duration (Nsec)") / 1e6,
            col(r, "AverageNs", "Average (Nsec)") / 1e3,
            col(r, "MinNs", "Min (Nsec)") / 1e3, col(r, "MaxNs", "Max (Nsec)") / 1e3, pct))
    with open(args.out, "w") as f:
        f.write("\n".join(out) + "\n")


def per_dispatch(path, counter):
    val = collections.defaultdict(float)
    name = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        val[d] += float(r["Counter_Value"])
        name[d] = r["Kernel_Name"]
    return val, name


def traffic(args):
    res = {}
    for counter, path in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        val, name = per_dispatch(path, counter)
        copies = [d for d in val if "copyBuffer" in name[d]]
        if not copies:
            raise SystemExit("no runtime copy dispatch in %s" % path)
        cal = max(copies, key=lambda d: val[d])
        scale = args.calib_bytes / (val[cal] * 1024.0)
        per = collections.defaultdict(list)
        for d, v in val.items():
            per[short(name[d])].append(v)
        res[counter] = (scale, val[cal], {k: sum(v) / len(v) for k, v in per.items()},
                        {k: len(v) for k, v in per.items()})
    src = kernel_source_hash()
    os.makedirs(args.outdir, exist_ok=True)
    fs, fcal, fk, fn = res["FETCH_SIZE"]
    ws, wcal, wk, wn = res["WRITE_SIZE"]
    for k in sorted(set(fk) & set(wk)):
        m = re.match(r"(k_fused|k_trace|k_lines|k_lines_halo|k_trace_lines|k_fused_stage)<(\d+),(\w+)>", k)
        if not m:
            continue
        tag = "%s_p%s_%s" % (m.group(1), m.group(2), "f64" if m.group(3) == "double" else "f32")
        fb = fk[k] * 1024.0 * fs
        wb = wk[k] * 1024.0 * ws
        lines = ["# HBM traffic of %s from rocprofv3 counters (%s)" % (k, args.workload),
                 "# fetch pass: %s" % args.command_fetch,
                 "# write pass: %s" % args.command_write,
                 "# summary: python3 -m paper_2107_14027_amd.rocprof_summary %s" % shlex.join(
                     sys.argv[1:]),
                 "# calibration: largest runtime copy of %d bytes read FETCH_SIZE %.1f KiB and "
                 "WRITE_SIZE %.1f KiB" % (args.calib_bytes, fcal, wcal),
                 "kernel: %s" % k,
                 "dispatches: %d fetch, %d write" % (fn[k], wn[k]),
                 "fetch_kib_per_dispatch: %.1f" % fk[k],
                 "write_kib_per_dispatch: %.1f" % wk[k],
                 "fetch_scale: %.4f" % fs,
                 "write_scale: %.4f" % ws,
                 "hbm_read_bytes_per_launch: %.0f" % fb,
                 "hbm_write_bytes_per_launch: %.0f" % wb,
                 "hbm_bytes_per_launch: %.0f" % (fb + wb),
                 "source_sha256_16: %s" % src]
        with open(os.path.join(args.outdir, "traffic_%s.txt" % tag), "w") as f:
            f.write("\n".join(lines) + "\n")


def counters(args):
    """Per-kernel SQ counters of one or more --pmc passes, per solution point
    (wave-level instruction counts x 64 / points) and as ratios."""
    pts = {}
    for kv in args.points.split(","):
        k, v = kv.split("=")
        pts[int(k)] = float(v)
    agg = collections.defaultdict(dict)
    for path in args.csv:
        per = collections.defaultdict(lambda: collections.defaultdict(float))
        for r in csv.DictReader(open(path)):
            k = short(r["Kernel_Name"])
            if not k.startswith("k_"):
                continue
            per[(k, int(r["Dispatch_Id"]))][r["Counter_Name"]] += float(r["Counter_Value"])
        n = collections.Counter(k for k, _ in per)
        for (k, _), cs in per.items():
            for c, v in cs.items():
                agg[k][c] = agg[k].get(c, 0.0) + v / n[k]
    cols = [("SQ_INSTS_VALU", "VALU"), ("SQ_INSTS_VALU_FMA_F64", "FMA64"),
            ("SQ_INSTS_VALU_FMA_F32", "FMA32"), ("SQ_INSTS_VALU_INT32", "INT32"),
            ("SQ_INSTS_SALU", "SALU"), ("SQ_INSTS_LDS", "LDS"), ("SQ_INSTS_VMEM_RD", "VMEM rd")]
    out = ["# rocprofv3 counters per solution point: %s" % args.workload, "",
           "command (one pass per counter group): `%s`" % args.command, "",
           "summary: `python3 -m paper_2107_14027_amd.rocprof_summary %s`" % shlex.join(sys.argv[1:]), "",
           "Instruction counts are per wavefront x 64 / solution points (= per point); "
           "bank conflict = SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS (conflict cycles per LDS instruction); "
           "the last two columns are raw counter ratios SQ_ACTIVE_INST_VALU / SQ_BUSY_CYCLES and "
           "SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES (counters summed as rocprofv3 reports them).", "",
           "| kernel | " + " | ".join(c[1] for c in cols) + " | bank conflict | ACTIVE_INST_VALU / BUSY_CYCLES | WAIT_INST_LDS / WAVE_CYCLES |",
           "|---|" + "---:|" * (len(cols) + 3)]
    for k in sorted(agg):
        m = re.match(r"k_\w+<(\d+),", k)
        if not m or int(m.group(1)) not in pts:
            continue
        a = agg[k]
        w = pts[int(m.group(1))] / 64.0

        def g(c):
            return a.get(c, float("nan"))
        cells = ["%.0f" % (g(c) / w) for c, _ in cols]
        ratio = lambda x, y: "%.2f" % (g(x) / g(y)) if g(y) > 0 else "nan"
        out.append("| %s | %s | %s | %s | %s |" % (k, " | ".join(cells),
                                                   ratio("SQ_LDS_BANK_CONFLICT", "SQ_INSTS_LDS"),
                                                   ratio("SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES"),
                                                   ratio("SQ_WAIT_INST_LDS", "SQ_WAVE_CYCLES")))
    with open(args.out, "w") as f:
        f.write("\n".join(out) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    s.add_argument("--min-percent", type=float, default=0.05)
    s.add_argument("--workload", default="")
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("outdir")
    t.add_argument("--calib-bytes", type=int, required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--workload", default="")
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("csv", nargs="+")
    c.add_argument("--points", required=True, help="order=solution points, comma separated")
    c.add_argument("--command", required=True)
    c.add_argument("--workload", default="")
    a = ap.parse_args()
    {"stats": stats, "traffic": traffic, "counters": counters}[a.cmd](a)


if __name__ == "__main__":
    main()

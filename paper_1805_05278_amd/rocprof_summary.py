"""Turn rocprofv3 CSV output into the short text summaries kept with the
library's measurements.

    python -m paper_1805_05278_amd.rocprof_summary stats DIR --command CMD \
        --workload TEXT -o OUT.md
        Kernel table (calls, average / total duration, share) from the
        ``*kernel_stats.csv`` under DIR, with the library's kernel names.

    python -m paper_1805_05278_amd.rocprof_summary traffic --fetch DIR1 --write DIR2 \
        --command-fetch CMD1 --command-write CMD2 --workload NAME -o OUT.md --json OUT.json
        Per-kernel HBM traffic per dispatch from two ``--pmc`` runs (FETCH_SIZE,
        then WRITE_SIZE, both in KiB per dispatch), each scaled by what the same
        counter reads for a plain elementwise copy of 2^27 doubles (1 GiB read,
        1 GiB written) captured in the same run.  The JSON file keeps one record
        per workload name (other workloads' records are left as they are).

    python -m paper_1805_05278_amd.rocprof_summary counters DIR --command CMD \
        --workload TEXT -o OUT.md
        Per-kernel averages of the counters of one ``--pmc`` run (derived
        counters such as MfmaUtil and VALUBusy as rocprofv3 computes them).

Only reads rocprofv3 output; it runs nothing on the GPU.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 8.0 * (1 << 27)

# Demangled kernel symbol -> the name the library's event timer uses.
_PATTERNS = [
    (r"k_batched_blk<0,", "batched_blk_f64"),
    (r"k_batched_blk<1,", "batched_blk_fp32"),
    (r"k_batched_blk<2,", "batched_blk_bf16"),
    (r"k_batched_refine", "batched_refine"),
    (r"k_batch_reset", "batched_queue_reset"),
    (r"k_zero_block_lower", "zero_block_lower"),
    (r"k_square_last_column", "square_last_column"),
    (r"k_normalize_r", "normalize_r"),
    (r"k_find_zero_diag", "find_zero_diag"),
    (r"k_set_identity", "set_identity"),
    (r"k_copy_matrix", "copy_matrix"),
    (r"k_scale_columns", "scale_columns"),
    (r"k_column_sumsq", "column_sumsq"),
    (r"k_axpy_cols", "axpy_cols"),
    (r"k_xpby_cols", "xpby_cols"),
    (r"k_chain_qr<\d+, true, 2>", "tsqr_chain_qr_leaf_rest"),
    (r"k_chain_qr<\d+, true, \d+>", "tsqr_chain_qr_leaf"),
    (r"k_chain_qr_rest<\d+>", "tsqr_chain_qr_leaf_rest"),
    (r"k_chain_qr<\d+, false, \d+>", "tsqr_chain_qr_tree"),
    (r"k_batched_ls", "batched_ls"),
    (r"k_tsqr_hr\b", "tsqr_hr_root"),
    (r"k_chain_down<\d+, \d+, false, \d+>", "tsqr_down_tree"),
    (r"k_chain_down<\d+, \d+, true, \d+>", "tsqr_down_leaf"),
    (r"k_gemm<\d+, \d+, (true|false), (true|false), 0>", "gemm_f64"),
    (r"k_gemm<\d+, \d+, (true|false), (true|false), 1>", "gemm_f32"),
    (r"k_gemm_bf16<", "gemm_bf16"),
    (r"k_splitk_reduce", "gemm_splitk_reduce"),
    (r"k_trsm_diag<", "trsm_diag"),
    (r"MulFunctor<double>", "copy_calibration"),
]


def library_name(symbol: str) -> str:
    for pat, name in _PATTERNS:
        if re.search(pat, symbol):
            return name
    return ""


# Library kernel name prefix -> the source files its code and launch shapes
# come from. A kernel's traffic record is valid only for those sources.
_KERNEL_SOURCES = [
    ("gemm_", ("gemm.hip", "gemm.h", "common.h")),
    ("tsqr_", ("tsqr.hip", "tsqr.h", "common.h")),
    ("batched_ls", ("batched.hip", "batched.h", "common.h")),
    ("batched_", ("batched_blk.hip", "batched.h", "common.h")),
    ("trsm_diag", ("solve.hip", "solve.h", "common.h")),
]


def source_digest(kernel: str = "") -> str:
    """Digest of the sources a kernel is built from (all HIP/C++ sources when
    the kernel is not named or not known)."""
    files = None
    for prefix, names in _KERNEL_SOURCES:
        if kernel.startswith(prefix):
            files = [os.path.join(HERE, "csrc", n) for n in names]
    if files is None:
        files = sorted(glob.glob(os.path.join(HERE, "csrc", "*")))
    h = hashlib.sha256()
    for p in files:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return hits[-1]


def _rows(path: str):
    with open(path, newline="") as f:
        yield from csv.DictReader(f)


def stats(args):
    path = _find(args.dir, "kernel_stats.csv")
    agg = defaultdict(lambda: [0, 0.0, []])
    for r in _rows(path):
        name = r["Name"]
        key = library_name(name) or name[:70]
        a = agg[key]
        a[0] += int(r["Calls"])
        a[1] += float(r["TotalDurationNs"])
        a[2].append(name)
    total = sum(v[1] for v in agg.values()) or 1.0
    lines = ["# Kernel trace: %s" % args.workload, "",
             "Command (from the repository root on the GPU host):", "", "```",
             args.command, "```", "",
             "| kernel | calls | avg us | total ms | share |", "|---|---:|---:|---:|---:|"]
    for k, (calls, ns, _) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append("| %s | %d | %.2f | %.3f | %.1f%% |" % (k, calls, ns / calls / 1e3, ns / 1e6,
                                                             100 * ns / total))
    lines += ["", "Symbols:", ""]
    for k, (_, _, names) in sorted(agg.items()):
        if library_name(names[0]):
            for n in sorted(set(names)):
                lines.append("- %s: `%s`" % (k, n))
    lines += ["", "source digest: %s" % source_digest(), ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))


def _counter(d: str, counter: str):
    per = defaultdict(list)
    for r in _rows(_find(d, "counter_collection.csv")):
        if r.get("Counter_Name") != counter:
            continue
        key = library_name(r["Kernel_Name"])
        if key:
            per[key].append(float(r["Counter_Value"]))
    return per


def traffic(args):
    fe = _counter(args.fetch, "FETCH_SIZE")
    wr = _counter(args.write, "WRITE_SIZE")
    if "copy_calibration" not in fe or "copy_calibration" not in wr:
        raise SystemExit("calibration copy kernel missing from the counter runs")
    kib = COPY_BYTES / 1024.0
    sf = kib / (sum(fe["copy_calibration"]) / len(fe["copy_calibration"]))
    sw = kib / (sum(wr["copy_calibration"]) / len(wr["copy_calibration"]))
    digest = source_digest()
    out = {"_calibration": {"fetch_scale": sf, "write_scale": sw,
                            "copy_bytes_each_way": COPY_BYTES,
                            "command_fetch": args.command_fetch,
                            "command_write": args.command_write}}
    lines = ["# HBM traffic per dispatch (rocprofv3 PMC)", "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged over dispatches) from two",
             "separate counter runs, scaled by the copy calibration: a 2^27-double elementwise",
             "copy reads and writes 1 GiB; the counters read %.4f and %.4f of that." % (1 / sf, 1 / sw),
             "", "Commands (from the repository root on the GPU host):", "", "```",
             args.command_fetch, args.command_write, "```", "",
             "| kernel | dispatches | FETCH KiB | WRITE KiB | HBM MB / dispatch (scaled) |",
             "|---|---:|---:|---:|---:|"]
    for k in sorted(set(fe) & set(wr)):
        f = sum(fe[k]) / len(fe[k])
        w = sum(wr[k]) / len(wr[k])
        b = (f * sf + w * sw) * 1024.0
        lines.append("| %s | %d | %.1f | %.1f | %.3f |" % (k, len(fe[k]), f, w, b / 1e6))
        if k != "copy_calibration":
            out[k] = {"hbm_bytes_per_launch": b, "fetch_kib": f, "write_kib": w,
                      "dispatches": len(fe[k]), "source_digest": source_digest(k)}
    lines += ["", "source digest: %s" % digest, ""]
    with open(args.out, "w") as fo:
        fo.write("\n".join(lines))
    allrec = {}
    if os.path.exists(args.json):
        with open(args.json) as fo:
            allrec = json.load(fo)
        if "_calibration" in allrec:  # a record without workload keys: replaced
            allrec = {}
    allrec[args.workload] = out
    with open(args.json, "w") as fo:
        json.dump(allrec, fo, indent=1, sort_keys=True)


def counters(args):
    per = defaultdict(lambda: defaultdict(list))
    names = []
    for r in _rows(_find(args.dir, "counter_collection.csv")):
        key = library_name(r["Kernel_Name"]) or r["Kernel_Name"][:50]
        c = r["Counter_Name"]
        if c not in names:
            names.append(c)
        per[key][c].append(float(r["Counter_Value"]))
    lines = ["# Counters per kernel: %s" % args.workload, "",
             "Averages per dispatch over the run (derived counters as rocprofv3 computes",
             "them: MfmaUtil = 100 SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x SIMDs);",
             "VALUBusy = 100 SQ_ACTIVE_INST_VALU / CUs / GRBM_GUI_ACTIVE; MfmaFlopsF64 =",
             "512 SQ_INSTS_VALU_MFMA_MOPS_F64).", "",
             "Command (from the repository root on the GPU host):", "", "```", args.command, "```",
             "", "| kernel | dispatches | " + " | ".join(names) + " |",
             "|---|---:|" + "---:|" * len(names)]
    order = sorted(per, key=lambda k: -len(per[k][names[0]]) if names else 0)
    for k in order:
        n = max(len(v) for v in per[k].values())
        cells = []
        for c in names:
            v = per[k].get(c, [])
            cells.append("%.4g" % (sum(v) / len(v)) if v else "")
        lines.append("| %s | %d | %s |" % (k, n, " | ".join(cells)))
    lines += ["", "source digest: %s" % source_digest(), ""]
    with open(args.out, "w") as fo:
        fo.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--command", required=True)
    s.add_argument("--workload", required=True)
    s.add_argument("-o", "--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("-o", "--out", required=True)
    t.add_argument("--json", required=True)
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--command", required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("-o", "--out", required=True)
    a = ap.parse_args()
    {"stats": stats, "traffic": traffic, "counters": counters}[a.cmd](a)


if __name__ == "__main__":
    main()

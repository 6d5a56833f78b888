"""Measured latency / bandwidth / arithmetic tradeoff of the tall-skinny QR
on one GPU (the paper's alpha-beta-gamma cost terms, Sec. 4 and the TSQR
costs of App. C, turned into measurements).

    python -m paper_1805_05278_amd.tune_sweep [--shapes 262144x256,1048576x64]
        [--reps 6] [-o OUT.md]

For each shape and each tuning (panel width b, leaf height h, chain length
c, tree arity k) it factors a seeded Gaussian matrix with an explicit thin
Q and reports: the time (minimum over the repetitions), the library launches
per factorisation (the alpha term: one launch per tree level and per panel
phase), the algorithmic HBM bytes the launches declare (beta), the flops of
the tree levels (gamma of the reduction tree) and the per-kernel time split.
The library's own per-launch events provide launches, bytes and flops; the
step time is taken on separate repetitions without them.
"""
from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

TUNINGS = [
    dict(),
    dict(leaf_rows=128),
    dict(chain=1),
    dict(chain=2),
    dict(chain=4),
    dict(chain=8),
    dict(arity=2),
    dict(arity=3),
    dict(b=32),
    dict(b=16),
]


def _label(kw):
    return ", ".join("%s=%s" % kv for kv in sorted(kw.items())) or "defaults"


def sweep(shapes, reps):
    import torch
    import synth
    import paper_1805_05278_amd as miqr

    h = miqr.Handle(0)
    rows = []
    for m, n in shapes:
        A = miqr.to_colmajor(synth.gaussian(m, n, 2000))
        T = miqr.colmajor(n, n)
        Q = miqr.colmajor(m, n)
        W = miqr.colmajor(m, n)
        for kw in TUNINGS:
            o = h.opts(Q=Q, **kw)
            times = []
            for r in range(reps):
                W.copy_(A)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                h.factor(W, T, o)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            W.copy_(A)
            torch.cuda.synchronize()
            h.profile(True)
            h.factor(W, T, o)
            torch.cuda.synchronize()
            tot = h.profile_totals()
            h.profile(False)
            launches = sum(v["launches"] for v in tot.values())
            nbytes = sum(v["bytes"] for v in tot.values())
            tree = tot.get("tsqr_chain_qr_tree", {"flops": 0.0, "launches": 0})
            split = {k: v["ms"] for k, v in tot.items()}
            rows.append(dict(shape="%dx%d" % (m, n), tuning=_label(kw), ms=min(times[1:] or times),
                             launches=launches, gbytes=nbytes / 1e9, tree_levels=tree["launches"],
                             tree_gflop=tree["flops"] / 1e9, split=split))
            print("%s %-22s %8.3f ms  launches %4d  bytes %6.2f GB  tree levels %2d" % (
                rows[-1]["shape"], rows[-1]["tuning"], rows[-1]["ms"], launches,
                nbytes / 1e9, tree["launches"]), flush=True)
    return rows


def report(rows, command):
    keys = ["gemm_f64", "tsqr_chain_qr_leaf", "tsqr_chain_qr_leaf_rest", "tsqr_chain_qr_tree",
            "tsqr_hr_root", "tsqr_down_tree", "tsqr_down_leaf"]
    short = ["gemm", "leaf", "leaf rest", "tree", "HR", "down tree", "down leaf"]
    out = ["# TSQR / EG tuning sweep: latency, bandwidth and arithmetic terms measured", "",
           "Command (from the repository root on the GPU host):", "", "```", command, "```", "",
           "ms: factorisation with thin Q, minimum over repetitions without per-launch events. "
           "launches: library launches (alpha). GB: algorithmic HBM bytes the launches declare (beta). "
           "tree: reduction-tree launches (levels, per panel summed) and their flops (gamma of the tree).",
           "", "| shape | tuning | ms | launches | GB | tree levels | tree GFLOP | " +
           " | ".join(short) + " |",
           "|---|---|---:|---:|---:|---:|---:|" + "---:|" * len(short)]
    for r in rows:
        out.append("| %s | %s | %.3f | %d | %.2f | %d | %.3f | %s |" % (
            r["shape"], r["tuning"], r["ms"], r["launches"], r["gbytes"], r["tree_levels"],
            r["tree_gflop"], " | ".join("%.3f" % r["split"].get(k, 0.0) for k in keys)))
    out.append("")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shapes", default="262144x256,1048576x64")
    ap.add_argument("--reps", type=int, default=6)
    ap.add_argument("-o", "--out", default="")
    a = ap.parse_args()
    shapes = [tuple(int(x) for x in s.split("x")) for s in a.shapes.split(",")]
    rows = sweep(shapes, a.reps)
    if a.out:
        cmd = "python -m paper_1805_05278_amd.tune_sweep --shapes %s --reps %d -o %s" % (
            a.shapes, a.reps, a.out)
        with open(a.out, "w") as f:
            f.write(report(rows, cmd))


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Throughput of recursive Householder QR (Elmroth-Gustavson recursion with a
TSQR base case) on one MI355X, FP64, on the square and moderately tall shapes.

One step = factor a 16384 x 16384 and a 65536 x 8192 Gaussian matrix in place
(FP64 MFMA updates, autotuned thresholds, the T-avoiding right-looking top
level with per-panel T and look-ahead).  The two factorisations are
independent and run on two streams with a handle each (--serial: one stream,
one after the other).  Every step works on its own copy of the inputs,
resident in HBM before the timed region.

value = nominal QR flops (2 m n^2 - 2 n^3 / 3, summed over both matrices) per
second over K timed steps.  The roofline of the dominant kernel comes from a
separate pass with every launch on one stream and no look-ahead, so that no
kernel shares the chip with another; --roofline-pass runs only that pass (the
command the rocprofv3 kernel-trace summary is taken of).  Sub-records: the same
step on one stream, the full-T form of Alg. 2, the tall-skinny TSQR /
1D-CAQR-EG step with thin Q and a least-squares solve, the 1024 x 64 TSQR,
mixed-precision least squares, batched and serving; and the CPU oracle timed on
a bounded sample of the headline workload.
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SHAPES = [(16384, 16384), (65536, 8192)]
TS_SHAPES = [(1048576, 64), (262144, 256)]
PEAK = {"hbm": 8.0e12, "fp64": 78.6e12, "fp32": 157.3e12}
# kernel -> arithmetic unit its flops run on
KERNEL_UNIT = {"gemm_f64": ("mfma", "fp64"), "gemm_f32": ("mfma", "fp32"),
               "tsqr_down_leaf": ("mfma", "fp64"), "tsqr_down_tree": ("mfma", "fp64"),
               "tsqr_chain_qr_leaf": ("alu", "fp64"), "tsqr_chain_qr_leaf_rest": ("alu", "fp64"),
               "tsqr_chain_qr_tree": ("alu", "fp64"), "batched_ls": ("alu", "fp64"),
               "tsqr_hr_root": ("alu", "fp64"), "trsm_diag": ("alu", "fp64"),
               "gemm_splitk_reduce": ("alu", "fp64")}
HEADLINE_WORKLOAD = "eg_qr_16384x16384_65536x8192"
TS_WORKLOAD = "tsqr_1048576x64_262144x256"


def nominal_flops(m, n):
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


def nominal_ls_flops(m, n, k):
    """QR of A plus Q^T B and back substitution (nominal)."""
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0 + 4.0 * m * n * k + n * n * k


def dominant(totals):
    return max(totals, key=lambda k: totals[k]["ms"])


def roofline(totals, name, workload):
    t = totals[name]
    sec = t["ms"] * 1e-3 / t["launches"]
    bytes_per = t["bytes"] / t["launches"]
    flops_per = t["flops"] / t["launches"]
    unit, prec = KERNEL_UNIT.get(name, ("alu", "fp64"))
    peak_f = PEAK[prec]
    # The binding roof is the lower of compute and bandwidth at this intensity.
    if flops_per / max(bytes_per, 1.0) < peak_f / PEAK["hbm"]:
        out = dict(bound="hbm", achieved=bytes_per / sec / 1e9, peak=PEAK["hbm"] / 1e9, unit="GB/s")
    else:
        out = dict(bound=unit, achieved=flops_per / sec / 1e12, peak=peak_f / 1e12, unit="TFLOP/s")
    out["frac"] = out["achieved"] / out["peak"]
    out["kernel"] = name
    out["launches"] = t["launches"]
    out["avg_launch_ms"] = t["ms"] / t["launches"]
    out["algorithmic_bytes_per_launch"] = bytes_per
    out["algorithmic_flops_per_launch"] = flops_per
    out["traffic"] = None
    tf = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if os.path.exists(tf):
        from paper_1805_05278_amd.rocprof_summary import source_digest
        with open(tf) as f:
            rec = json.load(f).get(workload, {}).get(name)
        if rec and rec.get("source_digest") == source_digest(name):
            out["traffic"] = rec["hbm_bytes_per_launch"]
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(prefix):
    """The oracle (plain unblocked Householder QR + T, FP64, OpenMP over the
    trailing columns) on a bounded sample of the headline workload: the
    leading 16384 x 1024 block of the 16384^2 input (its QR is the leading
    block of the full QR), on all host threads; and the leading 16384 x 256
    block on one thread."""
    import numpy as np
    import oracle
    m, k = prefix.shape
    A = np.asfortranarray(prefix)
    t0 = time.perf_counter()
    oracle.qr(A)
    dt = time.perf_counter() - t0
    threads = oracle.num_threads()
    k1 = 256
    code = ("import sys, time, numpy as np; sys.path.insert(0, %r); import oracle; "
            "A = np.load(sys.argv[1]); t = time.perf_counter(); oracle.qr(A); "
            "print(time.perf_counter() - t)" % ROOT)
    single = None
    tmp = os.path.join("/tmp", "miqr_cpu_sample_%d.npy" % os.getpid())
    try:
        np.save(tmp, np.asfortranarray(A[:, :k1]))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code, tmp], env=env, capture_output=True,
                           text=True, timeout=600)
        if r.returncode == 0:
            single = float(r.stdout.strip().splitlines()[-1])
    finally:
        if os.path.exists(tmp):
            os.remove(tmp)
    out = {"value": nominal_flops(m, k) / dt / 1e9, "unit": "GFLOP/s", "cores": threads,
           "kind": "oracle",
           "sample": "oracle QR + T of the leading %dx%d block of the %dx%d input (same values), "
                     "%d threads, %.1f s" % (m, k, SHAPES[0][0], SHAPES[0][1], threads, dt),
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    if single is not None:
        out["single_thread"] = {"value": nominal_flops(m, k1) / single / 1e9, "unit": "GFLOP/s",
                                "sample": "leading %dx%d block, 1 thread, %.1f s" % (m, k1, single)}
    return out


def bench_tall_skinny(torch, miqr, synth, steps):
    """The tall-skinny TSQR / 1D-CAQR-EG step (1048576 x 64 and 262144 x 256,
    FP64, explicit thin Q, plus one least-squares right-hand side on the
    262144 x 256 factors), two streams; with the roofline of its dominant
    kernel from a one-stream pass."""
    h1, h2 = miqr.Handle(0), miqr.Handle(0)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    pristine = [synth.gaussian_device(m, n, 2000 + i) for i, (m, n) in enumerate(TS_SHAPES)]
    m2, n2 = TS_SHAPES[1]
    b0 = synth.gaussian_device(m2, 1, 2100)
    Ts = [miqr.colmajor(n, n) for (_, n) in TS_SHAPES]
    Qs = [miqr.colmajor(m, n) for (m, n) in TS_SHAPES]
    opts = [h1.opts(Q=Qs[0]), h2.opts(Q=Qs[1])]

    def fresh():
        As = [miqr.colmajor(*P.shape) for P in pristine]
        for A, P in zip(As, pristine):
            A.copy_(P)
        b = miqr.colmajor(m2, 1)
        b.copy_(b0)
        return As, b

    def step(As, b, sts):
        with torch.cuda.stream(sts[0]):
            h1.factor(As[0], Ts[0], opts[0])
        with torch.cuda.stream(sts[1]):
            h2.factor(As[1], Ts[1], opts[1])
            h2.apply_q("T", As[1], Ts[1], b)
            h2.solve_r(As[1], b[:n2])

    def timed(sts, k, profiled=False):
        batches = [fresh() for _ in range(k)]
        torch.cuda.synchronize()
        if profiled:
            h1.profile(True)
            h2.profile(True)
        main = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(main)
        for st in sts:
            st.wait_stream(main)
        for As, b in batches:
            step(As, b, sts)
        for st in sts:
            main.wait_stream(st)
        e1.record(main)
        torch.cuda.synchronize()
        tot = {}
        if profiled:
            for hh in (h1, h2):
                for kk, v in hh.profile_totals().items():
                    t = tot.setdefault(kk, dict(ms=0.0, launches=0, bytes=0.0, flops=0.0))
                    for f in t:
                        t[f] += v[f]
                hh.profile(False)
        return e0.elapsed_time(e1) / k, tot

    timed(streams, 2)
    ms, _ = timed(streams, steps)
    one = torch.cuda.current_stream()
    sms, _ = timed([one, one], steps)
    _, tot = timed([one, one], 2, profiled=True)
    flops = sum(nominal_flops(m, n) for m, n in TS_SHAPES)
    dom = dominant(tot)
    h1.close()
    h2.close()
    return {"workload": "tall-skinny QR + thin Q: 1048576x64 and 262144x256, plus one LS RHS",
            "ms_per_step": ms, "gflops_nominal": flops / (ms * 1e-3) / 1e9,
            "serial_ms_per_step": sms,
            "roofline_one_stream": roofline(tot, dom, TS_WORKLOAD),
            "kernels_ms_per_step": {k: round(v["ms"] / 2, 3) for k, v in
                                    sorted(tot.items(), key=lambda kv: -kv[1]["ms"])}}


def bench_config1(torch, miqr, synth, h, reps=20):
    """1024 x 64, eight row blocks of 128 and a binary tree, normalised R and
    thin Q: microseconds per factorisation (latency bound)."""
    A0 = synth.gaussian_device(1024, 64, 1000)
    A = miqr.colmajor(1024, 64)
    T = miqr.colmajor(64, 64)
    Q = miqr.colmajor(1024, 64)
    sign = torch.empty(64, dtype=torch.float64, device="cuda")
    o = h.opts(leaf_rows=128, chain=1, arity=2, normalize=True, sign_out=sign, Q=Q)

    def timed():
        times, walls = [], []
        for r in range(reps + 3):
            A.copy_(A0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record()
            h.factor(A, T, o)
            e1.record()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if r >= 3:
                times.append(e0.elapsed_time(e1) * 1e3)
                walls.append((t1 - t0) * 1e6)
        times.sort()
        walls.sort()
        return times, walls

    times, walls = timed()
    # The same calls replayed from one captured launch graph.
    h.graphs(True)
    gtimes, gwalls = timed()
    h.graphs(False)
    return {"us_median": times[len(times) // 2], "us_min": times[0],
            "us_median_wall": walls[len(walls) // 2],
            "graph_us_median": gtimes[len(gtimes) // 2], "graph_us_min": gtimes[0],
            "graph_us_median_wall": gwalls[len(gwalls) // 2],
            "config": "1024x64, 8 blocks of 128 rows, binary tree, R diag >= 0, thin Q"}


def bench_batched(torch, miqr, synth, h, count=10000, seed=4242, precision=None):
    """The serving workload's problems (m in [64, 4096], n in [8, 256], 1-4
    right-hand sides) solved in one batched call, inputs resident in HBM.
    Mixed precisions: refinement iterations per problem (-1: solved again in
    FP64); every result meets backward error <= 1e-13."""
    import numpy as np
    trace = synth.serving_trace(count, 0.0, seed)
    As = [synth.gaussian_device(r.m, r.n, 10 ** 6 + i) for i, r in enumerate(trace)]
    Bs = [synth.gaussian_device(r.m, r.nrhs, 2 * 10 ** 6 + i) for i, r in enumerate(trace)]
    o = h.opts(precision=precision) if precision is not None else None
    mixed = precision not in (None, miqr.FP64)
    warm = 512
    h.lstsq_batched([a.clone() for a in As[:warm]], [b.clone() for b in Bs[:warm]], o)
    torch.cuda.synchronize()
    h.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    res = h.lstsq_batched(As, Bs, o, want_status=False, want_iters=mixed)
    e1.record()
    torch.cuda.synchronize()
    prof = h.profile_totals()
    h.profile(False)
    ms = e0.elapsed_time(e1)
    flops = sum(nominal_ls_flops(r.m, r.n, r.nrhs) for r in trace)
    kms = sum(v["ms"] for k, v in prof.items() if k.startswith("batched"))
    out = {"problems": count, "shapes": "m~U[64,4096], n~U[8,256] (m>=n), nrhs~U[1,4]",
           "ms": ms, "solves_per_s": count / (ms * 1e-3), "gflops_nominal": flops / (ms * 1e-3) / 1e9,
           "kernel_ms": kms, "kernel_tflops": flops / (kms * 1e-3) / 1e12 if kms else None,
           "kernel_frac_fp64_peak": flops / (kms * 1e-3) / PEAK["fp64"] if kms else None,
           "kernels": {k: round(v["ms"], 3) for k, v in prof.items()}}
    if mixed:
        its = np.array(res[2])
        ok = its[its >= 0]
        out["refinement"] = {"iterations_median": float(np.median(ok)) if ok.size else None,
                             "iterations_max": int(ok.max()) if ok.size else None,
                             "fp64_resolves": int((its < 0).sum()),
                             "backward_error_target": 1e-13}
    return out


def bench_batched_all(torch, miqr, synth, h):
    """bench_batched in FP64 and both mixed precisions on the same problems;
    speedup = FP64 kernel time / this precision's kernel time."""
    out = {}
    for name, p in (("fp64", miqr.FP64), ("mixed_fp32", miqr.MIXED_FP32),
                    ("mixed_bf16", miqr.MIXED_BF16)):
        out[name] = bench_batched(torch, miqr, synth, h, precision=p)
        torch.cuda.empty_cache()
    for name in ("mixed_fp32", "mixed_bf16"):
        out[name]["speedup_vs_fp64"] = out["fp64"]["kernel_ms"] / out[name]["kernel_ms"]
    return out


def bench_serving(torch, miqr, synth, h, count=10000, seed=99, rates=(0.25, 0.5, 0.9),
                  precision=0, followup=True):
    """Open-loop Poisson streams through the serving loop with pinned host
    inputs: capacity first (every request submitted at once), then arrival ->
    completion latency at 25, 50 and 90 % of it; and follow-up right-hand
    sides against kept factors."""
    import numpy as np
    P = 32
    g = torch.Generator().manual_seed(seed)
    # Each request's A (m x n) and B (m x nrhs) are contiguous column-major
    # blocks (lda = m), as a client would send them: the leading m n values of
    # a pooled pinned buffer.
    poolA = [torch.randn(4096 * 256, generator=g, dtype=torch.float64).pin_memory()
             for _ in range(P)]
    poolB = [torch.randn(4096 * 4, generator=g, dtype=torch.float64).pin_memory()
             for _ in range(P)]

    def req_views(i, r, nrhs=None):
        k = r.nrhs if nrhs is None else nrhs
        a = poolA[i % P][: r.m * r.n].view(r.n, r.m).t()
        b = poolB[i % P][: r.m * k].view(k, r.m).t()
        return a, b

    def run(rate, keep=False):
        trace = synth.serving_trace(count, rate, seed)
        X = [np.zeros((r.n, r.nrhs), order="F") for r in trace]
        srv = miqr.Server(h, hbm_budget=16 << 30, max_batch=1024, keep_factors=keep,
                          precision=precision)
        warm = 8
        for i in range(warm):
            srv.submit(*req_views(i, trace[i]), X[i])
        got = 0
        while got < warm:
            got += len(srv.poll(wait=True))
        recs = []
        t0 = srv.clock()
        idx = 0
        while len(recs) < count:
            now = srv.clock() - t0
            if now > 300.0:
                raise RuntimeError("serving run did not finish (%d of %d done)" % (len(recs), count))
            while idx < count and trace[idx].arrival_s <= now:
                srv.submit(*req_views(idx, trace[idx]), X[idx])
                idx += 1
            recs.extend(srv.poll())
        srv.close()
        lat = np.array([d["end_s"] - d["submit_s"] for d in recs])
        span = max(d["end_s"] for d in recs) - min(d["submit_s"] for d in recs)
        return trace, recs, lat, span

    trace, recs, lat, span = run(0.0)
    h2d = sum(8.0 * r.m * (r.n + r.nrhs) for r in trace)
    cap = count / span
    out = {"requests": count, "capacity": {
        "solves_per_s": cap, "h2d_gb_per_s": h2d / span / 1e9,
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_batch": float(np.mean([d["batch_size"] for d in recs])),
        "note": "all requests submitted at t = 0"},
        "inputs": "pinned host memory: each request's A and B contiguous (lda = m), "
                  "taken from 32 pooled N(0,1) buffers", "rates": []}
    for frac in rates:
        qps = frac * cap
        _, recs, lat, span = run(qps)
        out["rates"].append({"fraction_of_capacity": frac, "qps_offered": qps,
                             "solves_per_s": count / span,
                             "p50_ms": float(np.percentile(lat, 50) * 1e3),
                             "p99_ms": float(np.percentile(lat, 99) * 1e3),
                             "mean_batch": float(np.mean([d["batch_size"] for d in recs]))})
    if not followup:
        return out
    # Follow-up right-hand sides against kept factors: 2000 requests factored
    # with keep_factors, then one more right-hand side each.
    sub = synth.serving_trace(2000, 0.0, seed + 1)
    srv = miqr.Server(h, hbm_budget=16 << 30, max_batch=1024, keep_factors=True)
    X = [np.zeros((r.n, r.nrhs), order="F") for r in sub]
    ids = [srv.submit(*req_views(i, r), X[i]) for i, r in enumerate(sub)]
    done = 0
    while done < len(sub):
        done += len(srv.poll(wait=True))
    X2 = [np.zeros((r.n, 1), order="F") for r in sub]
    t0 = srv.clock()
    sub_t = {}
    for i, r in enumerate(sub):
        _, b = req_views(i + 7, r, 1)
        rid = srv.resolve(ids[i], b, X2[i])
        sub_t[rid] = srv.clock()
    lat2 = []
    while len(lat2) < len(sub):
        for d in srv.poll(wait=True):
            lat2.append(d["end_s"] - d["submit_s"])
    span2 = srv.clock() - t0
    srv.close()
    lat2 = np.array(lat2)
    out["followup_rhs"] = {"requests": len(sub), "solves_per_s": len(sub) / span2,
                           "p50_ms": float(np.percentile(lat2, 50) * 1e3),
                           "p99_ms": float(np.percentile(lat2, 99) * 1e3),
                           "note": "one new right-hand side per request against its kept factors"}
    return out


def bench_mixed(torch, miqr, synth, h, m=65536, n=2048, conds=(1e2, 1e6)):
    """Least squares on the conditioned 65536 x 2048 workload: FP64 against the
    mixed forms, each to backward error <= 1e-13."""
    out = {"shape": [m, n]}
    for cond in conds:
        seed = 34000 + int(round(__import__("math").log10(cond)))
        A = synth.conditioned(m, n, cond, seed)
        _, B = synth.ls_rhs(A, seed + 100, noise=1e-6, nrhs=1)
        A0, B0 = miqr.to_colmajor(A), miqr.to_colmajor(B)
        cell = {}
        for name, prec in (("fp64", miqr.FP64), ("fp32", miqr.MIXED_FP32),
                           ("bf16", miqr.MIXED_BF16)):
            times = []
            for rep in range(3):
                Ad = miqr.colmajor(m, n)
                Bd = miqr.colmajor(m, 1)
                Ad.copy_(A0)
                Bd.copy_(B0)
                torch.cuda.synchronize()
                t = time.perf_counter()
                st, info = h.lstsq(Ad, Bd, h.opts(precision=prec))
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t)
            best = min(times[1:])
            cell[name] = {"ms": best * 1e3, "solves_per_s": 1.0 / best, "status": st,
                          "backward_error": info.backward_error, "iterations": info.iterations,
                          "fallback": info.fallback}
        cell["speedup_fp32_vs_fp64"] = cell["fp64"]["ms"] / cell["fp32"]["ms"]
        cell["speedup_bf16_vs_fp64"] = cell["fp64"]["ms"] / cell["bf16"]["ms"]
        out["cond_%g" % cond] = cell
    return out


# Sub-records of the bench line, in the order they run.
EXTRAS = {
    "tall_skinny": lambda torch, miqr, synth, h: bench_tall_skinny(torch, miqr, synth, 5),
    "tsqr_1024x64": bench_config1,
    "mixed_ls": bench_mixed,
    "batched": bench_batched_all,
    "serving": bench_serving,
    "serving_mixed_fp32": lambda torch, miqr, synth, h: bench_serving(
        torch, miqr, synth, h, precision=miqr.MIXED_FP32, followup=False),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-profile", action="store_true", help="no roofline pass")
    ap.add_argument("--roofline-pass", action="store_true",
                    help="run only the one-stream, no-look-ahead pass with kernel events")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="the roofline pass's two factorisations without the per-kernel "
                         "event timer (for rocprofv3 counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (PMC byte-counter scale)")
    ap.add_argument("--serial", action="store_true",
                    help="run the step's two factorisations one after the other on one stream")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the sub-records other than the one-stream step")
    ap.add_argument("--only", choices=sorted(EXTRAS),
                    help="run one sub-record alone and print it (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1805_05278_amd as miqr
    import synth

    dev = torch.device("cuda:0")
    hs = [miqr.Handle(0), miqr.Handle(0)]
    blk = [hs[i].opts(t_layout=miqr.T_BLOCKED) for i in range(2)]
    pristine = [synth.gaussian_device(m, n, 31000 + n) for (m, n) in SHAPES]
    # The oracle's sample: the leading 1024 columns of the square input.
    prefix = None if args.no_cpu or args.roofline_pass else pristine[0][:, :1024].cpu().numpy()
    Ts = [miqr.colmajor(hs[0].t_rows(m, n, blk[0]), n) for (m, n) in SHAPES]
    flops = sum(nominal_flops(m, n) for m, n in SHAPES)

    def fresh():
        out = []
        for P in pristine:
            A = miqr.colmajor(*P.shape)
            A.copy_(P)
            out.append(A)
        return out

    if args.copy_calibration:
        # A plain elementwise copy of 2^27 doubles (1 GiB each way): the scale
        # for the PMC byte counters.
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y

    def roofline_pass():
        """Both factorisations on the current stream, no look-ahead, one event
        pair around every kernel; returns (per-kernel totals, ms per matrix)."""
        nola = [hs[i].opts(t_layout=miqr.T_BLOCKED, lookahead=False) for i in range(2)]
        As = fresh()
        torch.cuda.synchronize()
        # warm the path once (tuning cache, workspace)
        for i in range(2):
            hs[i].factor(As[i], Ts[i], nola[i])
        As = fresh()
        torch.cuda.synchronize()
        tot, per = {}, []
        for i in range(2):
            hs[i].profile(True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            hs[i].factor(As[i], Ts[i], nola[i])
            e1.record()
            torch.cuda.synchronize()
            per.append(e0.elapsed_time(e1))
            for k, v in hs[i].profile_totals().items():
                t = tot.setdefault(k, dict(ms=0.0, launches=0, bytes=0.0, flops=0.0))
                for f in t:
                    t[f] += v[f]
            hs[i].profile(False)
        return tot, per

    if args.only:
        print(json.dumps({args.only: EXTRAS[args.only](torch, miqr, synth, hs[0])}))
        return

    if args.pmc_pass:
        # One factorisation of each matrix (counter collection serialises
        # every dispatch, so a repeat would double a long run).
        nola = [hs[i].opts(t_layout=miqr.T_BLOCKED, lookahead=False) for i in range(2)]
        As = fresh()
        torch.cuda.synchronize()
        for i in range(2):
            hs[i].factor(As[i], Ts[i], nola[i])
            torch.cuda.synchronize()
            print(json.dumps({"pmc_pass_done": list(SHAPES[i])}), flush=True)
        return

    if args.roofline_pass:
        tot, per = roofline_pass()
        dom = dominant(tot)
        print(json.dumps({"roofline_pass": roofline(tot, dom, HEADLINE_WORKLOAD),
                          "ms_per_matrix": per,
                          "kernels": {k: {"ms": v["ms"], "launches": v["launches"]}
                                      for k, v in sorted(tot.items(), key=lambda kv: -kv[1]["ms"])}}))
        return

    one = torch.cuda.current_stream()
    two = [torch.cuda.Stream(), torch.cuda.Stream()]

    def timed(streams, k):
        """k steps on `streams`; returns (ms per step, wall s, per-matrix ms of
        the last step when both run on one stream, outputs of the last step)."""
        batches = [fresh() for _ in range(k)]
        main = torch.cuda.current_stream()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(main)
        for st in streams:
            st.wait_stream(main)
        for bi, As in enumerate(batches):
            for i in range(2):
                with torch.cuda.stream(streams[i]):
                    if bi == k - 1 and streams[0] is streams[1]:
                        ev[i].record(streams[i])
                    hs[i].factor(As[i], Ts[i], blk[i])
            if bi == k - 1 and streams[0] is streams[1]:
                ev[2].record(streams[1])
        for st in streams:
            main.wait_stream(st)
        e1.record(main)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = None
        if streams[0] is streams[1]:
            per = [ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])]
        return e0.elapsed_time(e1) / k, wall, per, batches[-1]

    streams = [one, one] if args.serial else two
    for _ in range(args.warmup):
        timed(streams, 1)
    ms, wall, per, last = timed(streams, args.steps)
    value = flops / (ms * 1e-3) / 1e9

    # Spot check of the last step (not timed): ||A z - Q (R z)|| / (||A|| ||z||)
    # for a random z, through the library's blocked Q application.
    checks = {}
    for i, (m, n) in enumerate(SHAPES):
        z = torch.randn(n, 1, dtype=torch.float64, device=dev)
        y = miqr.colmajor(m, 1)
        y.zero_()
        y[:n] = torch.triu(last[i][:n, :n]) @ z
        nb = Ts[i].shape[0]
        hs[i].apply_q_blocked("N", last[i], Ts[i], nb, y)
        ref = pristine[i] @ z
        checks["%dx%d" % (m, n)] = float(torch.linalg.norm(ref - y) /
                                        (torch.linalg.norm(pristine[i]) * torch.linalg.norm(z)))
    del last

    line = {
        "metric": "QR GFLOP/s (nominal 2mn^2-2n^3/3, FP64 on FP64 MFMA, recursive EG QR)",
        "value": value,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: i.i.d. N(0,1) drawn on the device from torch's seeded generator "
                "(seeds 47384 and 39192)",
        "config": {"workload": "recursive EG QR of a 16384x16384 and a 65536x8192 matrix, "
                               "FP64, T-avoiding right-looking top level with look-ahead, "
                               "autotuned thresholds; two streams",
                   "streams": 1 if args.serial else 2,
                   "fraction_of_fp64_peak": value * 1e9 / PEAK["fp64"],
                   "wall_s": wall, "probe_g1": checks,
                   "tuning": {"%dx%d" % s: hs[i].plan(s[0], s[1], blk[i])["tuning"]
                              for i, s in enumerate(SHAPES)}},
    }
    if not args.serial:
        sms, swall, sper, _ = timed([one, one], args.steps)
        line["serial"] = {"ms_per_step": sms, "value": flops / (sms * 1e-3) / 1e9,
                          "ms_per_matrix_last_step": {"%dx%d" % s: sper[i]
                                                      for i, s in enumerate(SHAPES)},
                          "note": "same step on one stream, the two factorisations in turn"}
    if not args.no_profile:
        tot, rper = roofline_pass()
        dom = dominant(tot)
        rl = roofline(tot, dom, HEADLINE_WORKLOAD)
        rl["pass"] = ("one stream, no look-ahead, both factorisations in turn, an event pair "
                      "around every kernel (bench.py --roofline-pass)")
        line["roofline"] = rl
        line["roofline_pass_ms_per_matrix"] = {"%dx%d" % s: rper[i] for i, s in enumerate(SHAPES)}
        line["kernels"] = {k: {"ms": round(v["ms"], 3), "launches": v["launches"],
                               "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 2)}
                           for k, v in sorted(tot.items(), key=lambda kv: -kv[1]["ms"])}
    if not args.no_extras:
        # The full-T form of Alg. 2 (every superdiagonal block of T formed).
        full = {}
        for i, (m, n) in enumerate(SHAPES):
            T = miqr.colmajor(n, n)
            best = None
            for r in range(2):
                A = fresh()[i]
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                hs[i].factor(A, T, hs[i].opts(t_layout=miqr.T_FULL))
                e1.record()
                torch.cuda.synchronize()
                best = e0.elapsed_time(e1) if best is None else min(best, e0.elapsed_time(e1))
                del A
            full["%dx%d" % (m, n)] = {
                "ms": best, "gflops_nominal": nominal_flops(m, n) / (best * 1e-3) / 1e9,
                "algorithmic_gemm_flops": hs[i].last_gemm_flops,
                "gemm_flops_over_nominal": hs[i].last_gemm_flops / nominal_flops(m, n)}
            del T
            torch.cuda.empty_cache()
        line["full_t"] = full
        blk_fl = {}
        for i, (m, n) in enumerate(SHAPES):
            A = fresh()[i]
            hs[i].factor(A, Ts[i], blk[i])
            torch.cuda.synchronize()
            blk_fl["%dx%d" % (m, n)] = hs[i].last_gemm_flops / nominal_flops(m, n)
            del A
        line["config"]["gemm_flops_over_nominal"] = blk_fl
        del pristine[:]
        torch.cuda.empty_cache()
        for key, fn in EXTRAS.items():
            try:
                line[key] = fn(torch, miqr, synth, hs[0])
            except Exception as exc:  # reported, never hidden
                line[key] = {"error": "%s: %s" % (type(exc).__name__, exc)}
            torch.cuda.empty_cache()
    if prefix is not None:
        line["cpu_baseline"] = cpu_baseline(prefix)
    print(json.dumps(line))
    for hh in hs:
        hh.close()


if __name__ == "__main__":
    main()

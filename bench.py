#!/usr/bin/env python3
"""Throughput of the tall-skinny QR hot path (TSQR / 1D-CAQR-EG base case with
EG recursion above it) on one MI355X, FP64, with explicit thin Q and a
least-squares solve on the factors.

One step = factor a 1,048,576 x 64 and a 262,144 x 256 Gaussian matrix in place
(each with its explicit thin Q), then solve one least-squares right-hand side
with the 262,144 x 256 factors (apply Q^T, back substitution).  Every step works
on its own copy of the inputs, prepared in HBM before the timed region.  The two
factorisations are independent and run on two streams with a handle each
(--serial: one stream, one after the other).

value = nominal QR flops (2 m n^2 - 2 n^3 / 3, summed over both matrices) per
second, from a timed region of K steps with no instrumentation.  A second
timed region of K more steps records HIP events around every library launch
(on the stream it runs on); the roofline of the dominant kernel (per-launch
algorithmic bytes or flops over its average duration) comes from those.  The
JSON line also carries the CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SHAPES = [(1048576, 64), (262144, 256)]
PEAK = {"hbm": 8.0e12, "fp64": 78.6e12, "fp32": 157.3e12}
# kernel -> arithmetic unit its flops run on
KERNEL_UNIT = {"gemm_f64": ("mfma", "fp64"), "gemm_f32": ("mfma", "fp32"),
               "tsqr_down_leaf": ("mfma", "fp64"), "tsqr_down_tree": ("mfma", "fp64"),
               "tsqr_chain_qr_leaf": ("alu", "fp64"), "tsqr_chain_qr_leaf_rest": ("alu", "fp64"),
               "tsqr_chain_qr_tree": ("alu", "fp64"), "batched_ls": ("alu", "fp64"),
               "tsqr_hr_root": ("alu", "fp64"), "trsm_diag": ("alu", "fp64"),
               "gemm_splitk_reduce": ("alu", "fp64")}


def nominal_flops(m, n):
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


def dominant(totals):
    return max(totals, key=lambda k: totals[k]["ms"])


def roofline(totals, steps, name):
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
    out["launches_per_step"] = t["launches"] / steps
    out["avg_launch_ms"] = t["ms"] / t["launches"]
    out["algorithmic_bytes_per_launch"] = bytes_per
    out["algorithmic_flops_per_launch"] = flops_per
    out["traffic"] = None
    tf = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if os.path.exists(tf):
        from paper_1805_05278_amd.rocprof_summary import source_digest
        with open(tf) as f:
            rec = json.load(f).get(name)
        if rec and rec.get("source_digest") == source_digest(name):
            out["traffic"] = rec["hbm_bytes_per_launch"]
    return out


def cpu_baseline(inputs):
    """The oracle (plain unblocked Householder QR + T + thin Q, FP64, OpenMP over
    trailing columns) on the same two matrices (about 10 s of host time)."""
    import numpy as np
    import oracle
    sample = list(SHAPES)
    flops = 0.0
    t0 = time.perf_counter()
    for (ms, ns), A in zip(sample, inputs):
        f = oracle.qr(np.asfortranarray(A[:ms, :ns]))
        oracle.thin_q(f)
        flops += nominal_flops(ms, ns)
    dt = time.perf_counter() - t0
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "oracle QR + T + thin Q of the full 1048576x64 and 262144x256 "
                      "matrices of one step, without the LS solve (%.1f s)" % dt}


def nominal_ls_flops(m, n, k):
    """QR of A plus Q^T B and back substitution (nominal)."""
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0 + 4.0 * m * n * k + n * n * k


def bench_batched(torch, miqr, synth, h, count=10000, seed=4242):
    """The serving workload's problems (m in [64, 4096], n in [8, 256], 1-4
    right-hand sides) solved in one batched call, inputs resident in HBM."""
    trace = synth.serving_trace(count, 0.0, seed)
    As = [synth.gaussian_device(r.m, r.n, 10 ** 6 + i) for i, r in enumerate(trace)]
    Bs = [synth.gaussian_device(r.m, r.nrhs, 2 * 10 ** 6 + i) for i, r in enumerate(trace)]
    warm = 512
    h.lstsq_batched([a.clone() for a in As[:warm]], [b.clone() for b in Bs[:warm]])
    torch.cuda.synchronize()
    h.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    st, _ = h.lstsq_batched(As, Bs, want_status=False)
    e1.record()
    torch.cuda.synchronize()
    tot = h.profile_totals().get("batched_ls", {})
    h.profile(False)
    ms = e0.elapsed_time(e1)
    flops = sum(nominal_ls_flops(r.m, r.n, r.nrhs) for r in trace)
    kms = tot.get("ms", float("nan"))
    return {"problems": count, "shapes": "m~U[64,4096], n~U[8,256] (m>=n), nrhs~U[1,4]",
            "ms": ms, "solves_per_s": count / (ms * 1e-3), "gflops_nominal": flops / (ms * 1e-3) / 1e9,
            "kernel_ms": kms, "kernel_tflops": flops / (kms * 1e-3) / 1e12 if kms == kms else None,
            "kernel_frac_fp64_alu_peak": flops / (kms * 1e-3) / PEAK["fp64"] if kms == kms else None}


def bench_serving(torch, miqr, synth, h, count=10000, qps=4000.0, seed=99):
    """Open-loop Poisson stream through the serving loop with pinned host
    inputs: arrival -> completion latency at an offered rate the server
    sustains, then capacity with every request submitted at once."""
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

    def req_views(i, r):
        a = poolA[i % P][: r.m * r.n].view(r.n, r.m).t()
        b = poolB[i % P][: r.m * r.nrhs].view(r.nrhs, r.m).t()
        return a, b

    def run(rate):
        trace = synth.serving_trace(count, rate, seed)
        X = [np.zeros((r.n, r.nrhs), order="F") for r in trace]
        srv = miqr.Server(h, hbm_budget=16 << 30, max_batch=1024)
        # Warm the path (graphs, pools) with a few requests first.
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

    trace, recs, lat, span = run(qps)
    flops = sum(nominal_ls_flops(r.m, r.n, r.nrhs) for r in trace)
    h2d = sum(8.0 * r.m * (r.n + r.nrhs) for r in trace)
    out = {"requests": count, "qps_offered": qps, "solves_per_s": count / span,
           "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "mean_batch": float(np.mean([d["batch_size"] for d in recs])),
           "gflops_nominal": flops / span / 1e9, "h2d_gb": h2d / 1e9,
           "inputs": "pinned host memory: each request's A and B contiguous (lda = m), "
                     "taken from 32 pooled N(0,1) buffers"}
    _, recs2, lat2, span2 = run(0.0)
    out["capacity"] = {"solves_per_s": count / span2, "h2d_gb_per_s": h2d / span2 / 1e9,
                       "p50_ms": float(np.percentile(lat2, 50) * 1e3),
                       "p99_ms": float(np.percentile(lat2, 99) * 1e3),
                       "mean_batch": float(np.mean([d["batch_size"] for d in recs2])),
                       "note": "all requests submitted at t = 0"}
    return out


def bench_eg(torch, miqr, synth, h, shapes=((16384, 16384), (65536, 8192)), reps=3):
    """Square and moderately tall recursive EG QR (FP64): QR GFLOP/s per shape,
    inputs resident, best of `reps` after one warm-up, with the GEMMs' share."""
    out = {}
    for (m, n) in shapes:
        A0 = synth.gaussian_device(m, n, 31000 + n)
        T = miqr.colmajor(n, n)
        A = miqr.colmajor(m, n)
        best, tot = None, None
        for r in range(reps + 1):
            A.copy_(A0)
            torch.cuda.synchronize()
            if r == reps:
                h.profile(True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            h.factor(A, T)
            e1.record()
            torch.cuda.synchronize()
            if r == reps:
                tot = h.profile_totals()
                h.profile(False)
            elif r > 0:
                ms = e0.elapsed_time(e1)
                best = ms if best is None else min(best, ms)
        gemm_ms = sum(v["ms"] for k, v in tot.items() if k.startswith("gemm"))
        gemm_fl = sum(v["flops"] for k, v in tot.items() if k.startswith("gemm"))
        out["%dx%d" % (m, n)] = {
            "ms": best, "gflops_nominal": nominal_flops(m, n) / (best * 1e-3) / 1e9,
            "frac_fp64_peak": nominal_flops(m, n) / (best * 1e-3) / PEAK["fp64"],
            "gemm_tflops": gemm_fl / (gemm_ms * 1e-3) / 1e12 if gemm_ms else None,
            "gemm_share": gemm_ms / sum(v["ms"] for v in tot.values()),
            "algorithmic_gemm_flops": gemm_fl}
        del A0, A, T
        torch.cuda.empty_cache()
    return out


def bench_mixed(torch, miqr, synth, h, m=65536, n=2048, cond=1e2, seed=34001):
    """Least squares on the conditioned 65536 x 2048 workload: FP64 against the
    mixed forms, each to backward error <= 1e-13."""
    A = synth.conditioned(m, n, cond, seed)
    _, B = synth.ls_rhs(A, seed + 1, noise=1e-6, nrhs=1)
    A0, B0 = miqr.to_colmajor(A), miqr.to_colmajor(B)
    out = {"shape": [m, n], "cond": cond}
    for name, prec in (("fp64", miqr.FP64), ("fp32", miqr.MIXED_FP32), ("bf16", miqr.MIXED_BF16)):
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
        # One more solve with per-kernel event timing (not part of the best time).
        Ad.copy_(A0)
        Bd.copy_(B0)
        torch.cuda.synchronize()
        h.profile(True)
        h.lstsq(Ad, Bd, h.opts(precision=prec))
        torch.cuda.synchronize()
        tot = h.profile_totals()
        h.profile(False)
        out[name] = {"ms": best * 1e3, "solves_per_s": 1.0 / best, "status": st,
                     "backward_error": info.backward_error, "iterations": info.iterations,
                     "fallback": info.fallback,
                     "kernels_ms": {k: round(v["ms"], 3) for k, v in
                                    sorted(tot.items(), key=lambda kv: -kv[1]["ms"])}}
    out["speedup_fp32_vs_fp64"] = out["fp64"]["ms"] / out["fp32"]["ms"]
    out["speedup_bf16_vs_fp64"] = out["fp64"]["ms"] / out["bf16"]["ms"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-profile", action="store_true", help="no per-kernel event timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (PMC byte-counter scale)")
    ap.add_argument("--serial", action="store_true",
                    help="run the step's two factorisations one after the other on one stream")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched, serving and mixed-precision sections")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1805_05278_amd as miqr
    import synth

    dev = torch.device("cuda:0")
    # The two factorisations of a step are independent: each gets its own
    # handle (workspace) and stream, so one's latency-bound phases (tree
    # levels, reconstruction root) overlap the other's wide kernels.
    h1, h = miqr.Handle(0), miqr.Handle(0)
    if args.serial:
        streams = [torch.cuda.current_stream()] * 2
    else:
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    host = [synth.gaussian(m, n, 2000 + i) for i, (m, n) in enumerate(SHAPES)]
    pristine = [miqr.to_colmajor(A) for A in host]
    m2, n2 = SHAPES[1]
    xt = synth.rng(2100).standard_normal(n2)
    b_host = host[1] @ xt + 1e-6 * synth.rng(2101).standard_normal(m2)
    b_pristine = miqr.to_colmajor(b_host.reshape(-1, 1))

    def fresh():
        As = []
        for P in pristine:
            A = miqr.colmajor(*P.shape)
            A.copy_(P)
            As.append(A)
        b = miqr.colmajor(m2, 1)
        b.copy_(b_pristine)
        return As, b

    Ts = [miqr.colmajor(n, n) for (_, n) in SHAPES]
    Qs = [miqr.colmajor(m, n) for (m, n) in SHAPES]
    opts = [h.opts(Q=Q) for Q in Qs]

    def step(As, b):
        with torch.cuda.stream(streams[0]):
            h1.factor(As[0], Ts[0], opts[0])
        with torch.cuda.stream(streams[1]):
            h.factor(As[1], Ts[1], opts[1])
            h.apply_q("T", As[1], Ts[1], b)
            h.solve_r(As[1], b[:n2])

    work = fresh()
    for _ in range(args.warmup):
        for A, P in zip(work[0], pristine):
            A.copy_(P)
        work[1].copy_(b_pristine)
        torch.cuda.synchronize()
        step(*work)
        torch.cuda.synchronize()
    def measure(streams):
        """Time args.steps steps on `streams`, then (unless --no-profile) the
        same number of steps again with an event pair around every kernel.
        Returns (ms per step of the clean pass, its wall s, per-kernel totals
        of the instrumented pass, ms per step of the instrumented pass, last
        step's outputs).  The per-kernel events add a gap between launches, so
        the step time is taken from the pass without them."""
        def step(As, b):
            with torch.cuda.stream(streams[0]):
                h1.factor(As[0], Ts[0], opts[0])
            with torch.cuda.stream(streams[1]):
                h.factor(As[1], Ts[1], opts[1])
                h.apply_q("T", As[1], Ts[1], b)
                h.solve_r(As[1], b[:n2])

        def timed(profiled):
            batches = [fresh() for _ in range(args.steps)]
            torch.cuda.synchronize()
            if profiled:
                h1.profile(True)
                h.profile(True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            main = torch.cuda.current_stream()
            t0 = time.perf_counter()
            e0.record(main)
            for st in streams:
                st.wait_stream(main)
            for As, b in batches:
                step(As, b)
            for st in streams:
                main.wait_stream(st)
            e1.record(main)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            totals = {}
            if profiled:
                for hh in (h1, h):
                    for k, v in hh.profile_totals().items():
                        t = totals.setdefault(k, dict(ms=0.0, launches=0, bytes=0.0, flops=0.0))
                        for f in t:
                            t[f] += v[f]
                h1.profile(False)
                h.profile(False)
            return e0.elapsed_time(e1) / args.steps, wall, totals, batches[-1]

        ms, wall, _, last = timed(False)
        totals, pms = {}, None
        if not args.no_profile:
            pms, _, totals, _ = timed(True)
        return ms, wall, totals, pms, last

    ms, wall, totals, pms, last = measure(streams)
    serial = None
    if not args.serial:
        one = torch.cuda.current_stream()
        serial = measure([one, one])

    # Spot check of the last step against simple invariants (not timed).
    As, b = last
    R1 = torch.triu(As[0][:64, :64])
    Qr = Qs[0]
    rec = float(torch.linalg.norm(Qr[:4096] @ R1 - pristine[0][:4096]) /
                torch.linalg.norm(pristine[0][:4096]))

    if args.copy_calibration:
        # A plain elementwise copy of 2^27 doubles (1 GiB each way): the scale
        # for the PMC byte counters.
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()

    flops = sum(nominal_flops(m, n) for m, n in SHAPES)
    value = flops / (ms * 1e-3) / 1e9
    line = {
        "metric": "QR GFLOP/s (nominal 2mn^2-2n^3/3, FP64, tall-skinny TSQR/1D-CAQR-EG with thin Q + LS solve)",
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
        "data": "synthetic: i.i.d. N(0,1) from numpy PCG64 seeds 2000/2001",
        "config": {"workload": "tall-skinny QR + thin Q: 1048576x64 and 262144x256, "
                               "plus one least-squares RHS on the 262144x256 factors",
                   "streams": 1 if args.serial else 2,
                   "fraction_of_fp64_peak": value * 1e9 / PEAK["fp64"],
                   "wall_s": wall, "recon_err_top4096": rec,
                   "ms_per_step_with_kernel_events": pms},
    }
    # The dominant kernel is the one with the most time in the one-stream step,
    # where launches do not share the chip; on two streams overlapping launches
    # stretch each other's durations and the ranking of close kernels can flip.
    dom = None
    if serial is not None:
        sms, swall, stot, spms, _ = serial
        line["serial"] = {"ms_per_step": sms, "value": flops / (sms * 1e-3) / 1e9,
                          "ms_per_step_with_kernel_events": spms,
                          "note": "same step on one stream, the two factorisations in turn"}
        if stot:
            dom = dominant(stot)
            line["serial"]["roofline"] = roofline(stot, args.steps, dom)
    if totals:
        if dom is None or dom not in totals:
            dom = dominant(totals)
        line["roofline"] = roofline(totals, args.steps, dom)
        line["kernels"] = {k: {"ms_per_step": v["ms"] / args.steps,
                               "launches_per_step": v["launches"] / args.steps}
                           for k, v in sorted(totals.items(), key=lambda kv: -kv[1]["ms"])}
    if not args.no_extras:
        for key, fn in (("eg_square_tall", bench_eg), ("batched", bench_batched),
                        ("serving", bench_serving), ("mixed_ls", bench_mixed)):
            try:
                line[key] = fn(torch, miqr, synth, h)
            except Exception as exc:  # reported, never hidden
                line[key] = {"error": "%s: %s" % (type(exc).__name__, exc)}
            torch.cuda.empty_cache()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(host)
    print(json.dumps(line))
    h.close()
    h1.close()


if __name__ == "__main__":
    main()

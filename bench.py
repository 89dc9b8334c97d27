"""Benchmark: compressed vs uncompressed FFT-based FMM translation on one MI355X.

One step = one tfmm_translate call: for every plane-wave direction and every
right-hand side, restore the FFT'ed operator from its compressed form, FFT the
zero-padded patterns, multiply, inverse-FFT and crop (Eq. (5)).  Inputs are
resident in device memory before the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload plain|batching|precision]

Prints one JSON line (rank 0).  The metric is translated grid points x
directions per second (boxes x directions x RHS / step time) of the
compressed operator; the uncompressed (FULL) operator is timed the same way
and reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP32_VALU_TFLOPS = 157.3  # packed; non-packed issue is half of it
PEAK_BF16_MFMA_TFLOPS = 2500.0  # dense


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="plain", choices=["plain", "batching", "precision", "tiny", "serving"])
    ap.add_argument("--requests", type=int, default=2000, help="serving: number of requests in the stream")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run 10 plain device copies of MIB MiB (reference for HBM byte counters)")
    ap.add_argument("--fmt", default=None, help="override the compressed format")
    ap.add_argument("--prec", default=None, choices=["fp32", "bf16x3"],
                    help="override the restoration arithmetic")
    ap.add_argument("--autotune", action="store_true",
                    help="run tfmm_autotune for the workload's RHS count before timing "
                         "(always on for the batching and precision workloads)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    return ap.parse_args()


def workload(name):
    return {"plain": synth.PLAIN, "batching": synth.BATCHING, "precision": synth.PRECISION,
            "tiny": synth.TINY}[name]


def restore_flops(fmt, ranks, n, ndir):
    """Real flops of the restoration contractions per launch (8 per complex MAC), shared over RHS."""
    n1, n2, n3 = n
    N = n1 * n2 * n3
    cm = 0
    if fmt == "tucker3d":
        r = np.asarray(ranks).reshape(-1, 3)
        for r1, r2, r3 in r:
            cm += n1 * r1 * r2 * r3 + n1 * n2 * r2 * r3 + N * r3
    elif fmt == "tt3d":
        r = np.asarray(ranks).reshape(-1, 2)
        for r1, r2 in r:
            cm += n1 * r1 * n2 * r2 + N * r2
    elif fmt == "tucker4d":
        r1, r2, r3, r4 = ranks
        cm += ndir * (r1 * r2 * r3 * r4 + n1 * r1 * r2 * r3 + n1 * n2 * r2 * r3 + N * r3)
    elif fmt == "htucker4d":
        r1, r2, r3, r4, r12, r34 = ranks
        cm += ndir * (r3 * r4 * r34 + r3 * r34 * r12 + r1 * r2 * r12 * r3 + n1 * r1 * r2 * r3 + n1 * n2 * r2 * r3
                      + N * r3)
    elif fmt == "tt4d":
        r1, r2, r3 = ranks
        cm += n1 * r1 * n2 * r2 + ndir * (r2 * n3 * r3 + N * r2)
    return 8.0 * cm


def fft_flops(K, n, ndir, nrhs):
    """Real flops of the pruned forward + inverse 3-D FFTs (5 m log2 m per line of length m)."""
    (K1, K2, K3), (n1, n2, n3) = K, n
    f = lambda m: 5.0 * m * math.log2(m)
    lines = (K2 * K3 * f(n1) + n1 * K3 * f(n2) + n1 * n2 * f(n3)) * 2
    return nrhs * ndir * (lines + 6.0 * n1 * n2 * n3)


def time_steps(ctx, op, A, B, steps, warmup, torch):
    """Time `steps` translations as the library runs them (a captured hipGraph per
    (op, nrhs, A, B) replayed on torch's current stream) between two
    synchronisations; then per-step latencies from HIP events around each step
    in a pass of their own (an event pair costs GPU time of its own, so it stays
    out of the timed loop); then, in an eager pass with the library's HIP-event
    profiling on, the per-kernel durations on the stream the kernels run on."""
    st = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.translate(op, A, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.translate(op, A, B)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nl = min(steps, 200)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nl)]
    for i in range(nl):
        evs[i][0].record(st)
        ctx.translate(op, A, B)
        evs[i][1].record(st)
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    ctx.set_profiling(True)
    ctx.kernel_times(reset=True)
    for _ in range(min(steps, 100)):
        ctx.translate(op, A, B)
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    kt = ctx.kernel_times(reset=True)
    return (t1 - t0) / steps * 1e3, lat, kt


def cpu_baseline(w, fmt, gpu_Bs, A_np, target_s):
    """The FP64 oracle on a bounded sample of directions: restoration + FFT convolution timed
    on the host; also the reference each GPU result (one per precision) is checked against
    on that sample: relative L2 error per direction, max and median."""
    import oracle as O

    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    khat, _ = O.directions(w.L, w.grid)
    ndir = khat.shape[0]
    rng = np.random.default_rng(12345)
    # grow the sample until it costs about target_s seconds
    sample = []
    t_total = 0.0
    errs = {p: [] for p in gpu_Bs}
    errs_exact = []
    order = rng.permutation(ndir)
    ctxm = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        for p in order:
            T = O.sample_operator(w.K, w.box, w.k, w.L, khat[p:p + 1])
            Th = O.fft_operator(T)
            comp = O.compress(Th, fmt, w.tol) if fmt != "full" else {"fmt": "full", "T": Th}
            Ap = A_np[:, p:p + 1].astype(np.complex128)
            t0 = time.perf_counter()
            Bc = O.translate_compressed(Ap, comp)
            t_total += time.perf_counter() - t0
            Bex = O.translate_fft(Ap, Th)
            for prec, gB in gpu_Bs.items():
                errs[prec].append(O.rel_l2(gB[:, p:p + 1], Bex))
            errs_exact.append(O.rel_l2(Bc, Bex))
            sample.append(int(p))
            if t_total >= target_s or len(sample) >= ndir:
                break
    finally:
        if ctxm is not None:
            ctxm.__exit__(None, None, None)
    units = w.boxes * len(sample) * A_np.shape[0]
    return {
        "value": units / t_total,
        "unit": "grid-pts*dirs/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{len(sample)} of {ndir} directions x {A_np.shape[0]} RHS of the {w.name} workload "
                  f"({fmt} restore + FFT convolution, FP64 numpy, 1 thread); {t_total:.1f} s",
        "cpu": platform.processor() or platform.machine(),
        "gpu_rel_err_max": {p: float(max(e)) for p, e in errs.items()},
        "gpu_rel_err_median": {p: float(np.median(e)) for p, e in errs.items()},
        "oracle_compressed_rel_err_max": float(max(errs_exact)),
    }


SERVING_SKIP = {
    # (grid, format) pairs left out of the stream, with the reason
    ((32, 32, 32), "tt4d"): "host TT-SVD of the 64^3 x 450 operator (Gram of a 2560-row unfolding) takes too long",
    ((24, 24, 24), "tt4d"): "host TT-SVD of the 48^3 x 450 operator takes too long",
    ((64, 16, 16), "tt4d"): "host TT-SVD of the 128 x 32 x 32 x 450 operator takes too long",
}


SERVING_BUDGET_BYTES = 1536 << 20


def bench_serving(args):
    """Poisson stream of translation requests through tfmm_submit / tfmm_poll."""
    import threading

    import torch

    import paper_2010_00520_amd as P

    # args.requests requests of the served operators (the stream is drawn long
    # enough that the ones of operators left out do not reduce the count)
    reqs = [r for r in synth.serving_requests(3 * args.requests) if (r["grid"], r["fmt"]) not in SERVING_SKIP]
    reqs = reqs[:args.requests]
    L = 14  # ceil rule at 0.5 lambda boxes and 4 digits (450 directions)
    keys = sorted({(r["grid"], r["fmt"]) for r in reqs})
    out = {}
    # HBM budget: every compressed operator plus translation scratch fits, the
    # uncompressed operators of the same grids (about 2 GB) would not
    budget = SERVING_BUDGET_BYTES
    with P.Context(0, budget_bytes=budget) as ctx:
        ops, setup_s, stored = {}, {}, {}
        bytes_stored, bytes_full = 0, 0
        for key in keys:
            grid, fmt = key
            t0 = time.perf_counter()
            ops[key] = ctx.setup(K=grid, box=0.5, k=synth.K0, L=L, fmt=fmt, tol=1e-4)
            setup_s[f"{grid}-{fmt}"] = time.perf_counter() - t0
            inf = ops[key].info()
            stored[f"{grid}-{fmt}"] = inf["bytes_stored"] / inf["bytes_full"]
            bytes_stored += inf["bytes_stored"]
        bytes_full = sum(8 * 8 * g[0] * g[1] * g[2] * (L + 1) * 2 * (L + 1) for g in {k[0] for k in keys})
        ndir = (L + 1) * 2 * (L + 1)
        # per grid: one seeded input buffer of 16 RHS and a ring of output buffers
        inputs, rings, ring_pos = {}, {}, {}
        for grid in sorted({k[0] for k in keys}):
            inputs[grid] = torch.from_numpy(synth.gaussian_patterns((16, ndir) + grid, 77)).cuda()
            rings[grid] = [torch.empty_like(inputs[grid]) for _ in range(8)]
            ring_pos[grid] = 0
        torch.cuda.synchronize()
        # warm-up: one job per operator
        for key, op in ops.items():
            g = key[0]
            ctx.wait(ctx.submit(op, inputs[g][:1], rings[g][0][:1]))
        lock = threading.Lock()
        busy = {g: [0] * 8 for g in rings}
        pending, lat, units_done = [], [], [0]
        waits, wait_s = 0, 0.0  # requests that found every output slot of their grid busy
        t_start = time.perf_counter()
        for r in reqs:
            now = time.perf_counter() - t_start
            if r["arrival_s"] > now:
                time.sleep(r["arrival_s"] - now)
            g, nr = r["grid"], r["nrhs"]
            # reclaim finished output slots, wait if every slot of this grid is in use
            tw = None
            while True:
                for item in list(pending):
                    done, st, l = ctx.poll(item[0])
                    if done:
                        lat.append(l)
                        units_done[0] += item[3]
                        busy[item[1]][item[2]] = 0
                        pending.remove(item)
                free = [i for i, b in enumerate(busy[g]) if not b]
                if free:
                    break
                if tw is None:
                    tw = time.perf_counter()
                    waits += 1
                time.sleep(0.0002)
            if tw is not None:
                wait_s += time.perf_counter() - tw
            slot = free[0]
            busy[g][slot] = 1
            t = ctx.submit(ops[(g, r["fmt"])], inputs[g][:nr], rings[g][slot][:nr])
            pending.append((t, g, slot, nr * ndir * g[0] * g[1] * g[2]))
        for item in pending:
            st, l = ctx.wait(item[0])
            lat.append(l)
            units_done[0] += item[3]
        wall = time.perf_counter() - t_start
        for op in ops.values():
            op.release()
    lat = np.array(lat) / 1e3  # ms
    out = {
        "metric": "translated grid-pts*dirs/s under a Poisson request stream; p50/p99 latency",
        "value": units_done[0] / wall,
        "unit": "grid-pts*dirs/s",
        "n_gpus": 1,
        "requests": len(reqs),
        "rate_hz": synth.SERVING_RATE_HZ,
        "wall_s": wall,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "admission_waits": {"requests": waits, "total_ms": wait_s * 1e3},
        "config": {"workload": "serving", "L": L, "n_dir": ndir, "tol": 1e-4, "hbm_budget_bytes": budget,
                   "operators_stored_bytes": bytes_stored, "uncompressed_operators_bytes": bytes_full,
                   "operators": [f"{g}-{f}" for g, f in keys],
                   "skipped": {f"{g}-{f}": why for (g, f), why in SERVING_SKIP.items()}},
        "setup_s": setup_s,
        "memory_fraction": stored,
    }
    print(json.dumps(out))


def bench_precision(args):
    """Precision workload (128 x 8 x 8 boxes, 338 directions, 4 RHS): TT-4D and H-Tucker-4D
    at gamma = 1e-4 and 1e-6, each restored in FP32 and in bf16x3; throughput, and the error of
    every RHS against the exact FP64 translation (the oracle's operator sampled for a bounded
    set of directions)."""
    import torch

    import oracle as O
    import paper_2010_00520_amd as P

    w = synth.PRECISION
    A_np = synth.patterns_for(w)
    A = torch.from_numpy(A_np).cuda()
    ndir, nrhs = w.n_dir, w.nrhs
    units = w.boxes * ndir * nrhs
    khat, _ = O.directions(w.L, w.grid)
    rng = np.random.default_rng(2024)
    sample = sorted(int(p) for p in rng.choice(ndir, size=12, replace=False))
    exact = {}
    for p in sample:
        Th = O.fft_operator(O.sample_operator(w.K, w.box, w.k, w.L, khat[p:p + 1]))
        exact[p] = O.translate_fft(A_np[:, p:p + 1].astype(np.complex128), Th)
    rows = []
    with P.Context(0) as ctx:
        full = ctx.setup(K=w.K, box=w.box, k=w.k, L=w.L, fmt="full")
        ctx.autotune(full, nrhs=nrhs, reps=10)  # tiles autotuned on both sides of the comparison
        Bf = torch.zeros_like(A)
        ms_f, _, _ = time_steps(ctx, full, A, Bf, args.steps, args.warmup, torch)
        bytes_full = full.info()["bytes_stored"]
        full.release()
        for fmt in ("htucker4d", "tt4d"):
            for tol in (1e-4, 1e-6):
                t0 = time.perf_counter()
                op = ctx.setup(K=w.K, box=w.box, k=w.k, L=w.L, fmt=fmt, tol=tol, prec="fp32")
                setup_s = time.perf_counter() - t0
                info = op.info()
                nr = 6 if fmt == "htucker4d" else 3
                ranks, data = list(info["ranks"][:nr]), op.export()
                for prec in ("fp32", "bf16x3"):
                    o = op if prec == "fp32" else ctx.import_factors(w.K, w.L, fmt, ranks, data, prec=prec)
                    plan, _ = ctx.autotune(o, nrhs=nrhs, reps=10)
                    B = torch.zeros_like(A)
                    ms, lat, kt = time_steps(ctx, o, A, B, args.steps, args.warmup, torch)
                    Bn = B.cpu().numpy().astype(np.complex128)
                    per_rhs = [max(O.rel_l2(Bn[s, p], exact[p][s, 0]) for p in sample) for s in range(nrhs)]
                    rows.append({"fmt": fmt, "tol": tol, "precision": prec, "ms_per_step": ms,
                                 "value": units / (ms * 1e-3), "time_ratio_compressed_over_full": ms / ms_f,
                                 "memory_fraction": info["bytes_stored"] / bytes_full, "ranks": ranks,
                                 "rel_err_fro_setup": info["rel_err_fro"], "setup_s": setup_s,
                                 "rel_err_per_rhs_max_over_sample": per_rhs,
                                 "within_10gamma": bool(max(per_rhs) <= 10 * tol + 1e-6), "kernels": kt,
                                 "plan": plan})
                    if o is not op:
                        o.release()
                op.release()
    head = next(r for r in rows if r["fmt"] == "htucker4d" and r["tol"] == 1e-4 and r["precision"] == "bf16x3")
    print(json.dumps({
        "metric": "translated grid-pts*dirs/s, compressed operator (vs uncompressed), rel err <= 1e-4",
        "value": head["value"], "unit": "grid-pts*dirs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3 (split-bf16 MFMA, f32 accumulate; FFTs f32)", "data": "synthetic",
        "config": {"workload": w.name, "K": list(w.K), "box": w.box, "L": w.L, "n_dir": ndir, "nrhs": nrhs,
                   "error_sample_directions": sample},
        "uncompressed": {"ms_per_step": ms_f, "value": units / (ms_f * 1e-3)},
        "results": rows,
    }))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "precision":
        return bench_precision(args)
    import torch

    import paper_2010_00520_amd as P

    w = workload(args.workload)
    fmt = args.fmt or w.fmt
    # the compressed path is timed in both restoration arithmetics; the headline
    # is split-BF16 (bf16x3, FP32 accumulation), FP32 is reported beside it
    precs = [args.prec] if args.prec else ["bf16x3", "fp32"]
    A_np = synth.patterns_for(w)
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = args.calibrate_copy << 18  # MiB -> float32 count
        src = torch.ones(n, device=dev)
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    A = torch.from_numpy(A_np).to(dev)
    res = {}
    with P.Context(0) as ctx:
        for prec in precs:
            B = torch.zeros_like(A)
            t0 = time.perf_counter()
            op = ctx.setup(K=w.K, box=w.box, k=w.k, L=w.L, fmt=fmt, tol=w.tol, prec=prec)
            setup_s = time.perf_counter() - t0
            tune = args.autotune or args.workload == "batching"
            tuned = ctx.autotune(op, nrhs=w.nrhs, reps=10) if tune else None
            ms, lat, kt = time_steps(ctx, op, A, B, args.steps, args.warmup, torch)
            res[prec] = {"ms": ms, "lat": lat, "kt": kt, "info": op.info(), "ranks": op.ranks(), "setup_s": setup_s,
                         "plan": op.plan(), "autotune": tuned, "B": B.cpu().numpy().astype(np.complex128)}
            op.release()
        # the batching grid is also run with Tucker-4D (per-call core contraction
        # + register-chained restoration, the format with the smallest operator there)
        extra = {}
        for xf in (["tucker4d"] if args.workload == "batching" and not args.fmt else []):
            t0 = time.perf_counter()
            op = ctx.setup(K=w.K, box=w.box, k=w.k, L=w.L, fmt=xf, tol=w.tol, prec=precs[0])
            setup_s = time.perf_counter() - t0
            ctx.autotune(op, nrhs=w.nrhs, reps=10)
            B = torch.zeros_like(A)
            ms_x, lat_x, kt_x = time_steps(ctx, op, A, B, args.steps, args.warmup, torch)
            extra[xf] = {"ms": ms_x, "kt": kt_x, "info": op.info(), "setup_s": setup_s, "plan": op.plan()}
            op.release()
        full = ctx.setup(K=w.K, box=w.box, k=w.k, L=w.L, fmt="full")
        if args.autotune or args.workload == "batching":
            ctx.autotune(full, nrhs=w.nrhs, reps=10)
        Bf = torch.zeros_like(A)
        ms_f, lat_f, kt_f = time_steps(ctx, full, A, Bf, args.steps, args.warmup, torch)
        finfo = full.info()
        full.release()

    ndir, nrhs = w.n_dir, w.nrhs
    units = w.boxes * ndir * nrhs
    n = w.n
    prof_steps = min(args.steps, 100)

    def roofline(prec, r):
        kt, info = r["kt"], r["info"]
        # dominant kernel of the compressed path (largest total time)
        zname = max(kt, key=lambda k: kt[k]["avg_ms"] * kt[k]["launches"])
        zms = kt[zname]["avg_ms"] * kt[zname]["launches"] / prof_steps  # per step
        flops = restore_flops(fmt, r["ranks"], n, ndir)
        io = 2 * 8 * units  # A read + B written, complex64
        # the fused kernel moves A and B as well; the three-pass z-stage only reads the operator
        alg_bytes = info["bytes_stored"] + (io if zname.startswith("fused") else 0)
        valu_flops = fft_flops(w.K, n, ndir, nrhs) if zname.startswith("fused") else 0.0
        mfma_tfs = flops / (zms * 1e-3) / 1e12
        if prec == "bf16x3":
            # each FP32 product is three bf16 products (hi*hi + hi*lo + lo*hi) on the bf16 matrix cores
            cand = [("mfma", 3 * mfma_tfs, PEAK_BF16_MFMA_TFLOPS, "TFLOP/s")]
        else:
            cand = [("mfma", mfma_tfs, PEAK_FP32_MFMA_TFLOPS, "TFLOP/s")]
        cand.append(("hbm", alg_bytes / (zms * 1e-3) / 1e9, PEAK_HBM_GBS, "GB/s"))
        if valu_flops:
            cand.append(("alu", valu_flops / (zms * 1e-3) / 1e12, PEAK_FP32_VALU_TFLOPS, "TFLOP/s"))
        bound = max(cand, key=lambda c: c[1] / c[2])
        traffic = None
        tpath = os.path.join(ROOT, "profiles", "traffic.json")
        if os.path.exists(tpath):
            try:
                tr = json.load(open(tpath))
                key = f"{args.workload}:{fmt}:{prec}:{zname}"
                if key in tr and tr[key].get("kernel_sha") == _kernel_sha():
                    traffic = tr[key]["bytes_per_launch"]
            except Exception:
                traffic = None
        return {"bound": bound[0], "achieved": round(bound[1], 3), "peak": bound[2], "unit": bound[3],
                "frac": round(bound[1] / bound[2], 4), "traffic": traffic, "kernel": zname,
                "kernel_avg_ms": zms, "algorithmic_flops": flops, "algorithmic_bytes": alg_bytes,
                "fft_flops": valu_flops,
                "other_bound": {c[0]: {"achieved": round(c[1], 3), "peak": c[2], "unit": c[3],
                                       "frac": round(c[1] / c[2], 4)} for c in cand if c[0] != bound[0]}}

    head = precs[0]
    r = res[head]
    ms = r["ms"]
    out = {
        "metric": "translated grid-pts*dirs/s, compressed operator (vs uncompressed), rel err <= 1e-4",
        "value": units / (ms * 1e-3),
        "unit": "grid-pts*dirs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32" else "bf16x3 (split-bf16 MFMA, f32 accumulate; FFTs f32)",
        "data": "synthetic",
        "config": {"workload": w.name, "K": list(w.K), "box": w.box, "L": w.L, "n_dir": ndir, "fmt": fmt,
                   "tol": w.tol, "nrhs": nrhs, "precision": head},
        "p50_ms": float(np.percentile(r["lat"], 50)),
        "p99_ms": float(np.percentile(r["lat"], 99)),
        "uncompressed": {"value": units / (ms_f * 1e-3), "ms_per_step": ms_f,
                         "p50_ms": float(np.percentile(lat_f, 50)), "p99_ms": float(np.percentile(lat_f, 99)),
                         "kernels": kt_f},
        "time_ratio_compressed_over_full": ms / ms_f,
        "memory_fraction": r["info"]["bytes_stored"] / finfo["bytes_stored"],
        "op": {"ranks_max": r["info"]["ranks"], "rel_err_fro": r["info"]["rel_err_fro"], "setup_s": r["setup_s"],
               "bytes_stored": r["info"]["bytes_stored"], "bytes_full": finfo["bytes_stored"], "plan": r["plan"],
               "autotune": r["autotune"]},
        "kernels": r["kt"],
        "fft_flops_per_step": fft_flops(w.K, n, ndir, nrhs),
        "roofline": roofline(head, r),
        "cpu_baseline": None,
    }
    for prec in precs[1:]:
        q = res[prec]
        out[prec] = {"value": units / (q["ms"] * 1e-3), "ms_per_step": q["ms"],
                     "p50_ms": float(np.percentile(q["lat"], 50)), "p99_ms": float(np.percentile(q["lat"], 99)),
                     "time_ratio_compressed_over_full": q["ms"] / ms_f, "kernels": q["kt"],
                     "roofline": roofline(prec, q)}
    if extra:
        out["other_formats"] = {
            xf: {"precision": precs[0], "value": units / (x["ms"] * 1e-3), "ms_per_step": x["ms"],
                 "time_ratio_compressed_over_full": x["ms"] / ms_f,
                 "memory_fraction": x["info"]["bytes_stored"] / finfo["bytes_stored"],
                 "ranks": x["info"]["ranks"], "rel_err_fro": x["info"]["rel_err_fro"], "setup_s": x["setup_s"],
                 "plan": x["plan"], "kernels": x["kt"]}
            for xf, x in extra.items()}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, fmt, {p: res[p]["B"] for p in precs}, A_np, args.cpu_seconds)
        out["rel_err_vs_fp64"] = out["cpu_baseline"]["gpu_rel_err_max"][head]
    print(json.dumps(out))


def _kernel_sha():
    import hashlib

    h = hashlib.sha256()
    for f in ("device_common.h", "gen_dft.py", "kernels.hip", "stages.h", "tucker_restore.h", "xy_stages.h",
              "zstage_full.hip", "zstage_tt3d.hip", "zstage_tt4d.hip", "zstage_tucker.hip"):
        with open(os.path.join(ROOT, "paper_2010_00520_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()

"""Throughput of the FC^2T^2 explicit layer, forward + backward, on one MI355X.

One step = expansion of the sources (bin + sort, P2M, M2M, M2L at every level, L2L),
evaluation at the queries (L2P), and the backward pass (L2P^T, L2L^T, M2L^T, M2M^T, P2M^T
and the query gradient): y, w_bar, p_bar, q_bar for the 2-D workload N = M = 2^20
sources/queries, 256^2 grid, K = 6, Gaussian sigma = 0.01, FP32 IO.  Inputs are resident
in HBM before the timed region.

Prints one JSON line with the throughput, the roofline of the dominant kernel (timed live
with HIP events on the stream it runs on) and the CPU checker's throughput on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "queries/sec fwd+bwd at fixed rel-L2 err vs FP64 direct sum; M2L MFMA util"
PEAKS = {  # MI355X published peaks
    "hbm_GBps": 8000.0,
    "fp32_vector_TFLOPs": 157.3,
    "bf16_mfma_TFLOPs": 2500.0,
    "fp64_TFLOPs": 78.6,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="explicit2d")
    ap.add_argument("--m2l", default="bf16x3", help="f32 | bf16 | bf16x2 | bf16x3")
    ap.add_argument("--compare-f32", type=int, default=1,
                    help="also time the same step with the plain FP32 M2L (same accuracy class)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=256, help="queries in the CPU sample")
    ap.add_argument("--kernel-reps", type=int, default=20)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2111_00110_amd import accounting, fc2t2, workloads

    torch.cuda.set_device(0)
    wl = workloads.workload(args.workload)
    x = workloads.make(wl, seed=0)
    dev = torch.device("cuda", 0)
    t = {k: torch.from_numpy(v).to(dev) for k, v in x.items()}
    def make_plan(m2l):
        return fc2t2.Plan(wl.dim, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K, m2l=m2l, io=wl.io)

    p, w = t["p"], t["w"]
    q, gy = t.get("q"), t.get("gy")

    layer = wl.layer
    if layer != "explicit":
        o, r = t["o"], t["r"]

    def time_steps(plan, steps, warmup):
        Lt = plan.new_local()
        gL = plan.new_local()
        gp = torch.zeros_like(p)
        gw = torch.zeros_like(w)
        if layer == "explicit":
            gq = torch.zeros_like(q)

            def step():
                plan.expand(p, w, out=Lt)
                y, _, _ = plan.eval(Lt, q)
                gL.zero_()
                gq.zero_()
                gp.zero_()
                gw.zero_()
                plan.eval_backward(Lt, q, gy, gL, gq)
                plan.expand_backward(gL, p, w, gp, gw)
                return y
        elif layer == "ray_integral":
            def step():
                plan.expand(p, w, out=Lt)
                y = plan.ray_integral(Lt, o, r, wl.t0, wl.t1)
                gL.zero_()
                gp.zero_()
                gw.zero_()
                plan.ray_integral_backward(o, r, wl.t0, wl.t1, gy, gL)
                plan.expand_backward(gL, p, w, gp, gw)
                return y
        else:
            gt, gn = t["gt"], t["gn"]

            def step():
                plan.expand(p, w, out=Lt)
                tt, nrm, hit, saved = plan.ray_root(Lt, o, r, wl.t0, wl.t1, 0.5)
                gL.zero_()
                gp.zero_()
                gw.zero_()
                plan.ray_root_backward(saved, hit, gt, gn, gL)
                plan.expand_backward(gL, p, w, gp, gw)
                return tt

        for _ in range(warmup):
            y = step()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):
            y = step()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps, y

    t_plan0 = time.perf_counter()
    plan = make_plan(args.m2l)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t_plan0) * 1e3
    ms, y = time_steps(plan, args.steps, args.warmup)
    units = wl.M if wl.layer == "explicit" else wl.R
    value = units / (ms * 1e-3)
    f32_ms = None
    if args.compare_f32 and args.m2l != "f32":
        f32_ms, _ = time_steps(make_plan("f32"), max(3, args.steps // 4), 1)

    # ---- dominant kernel: the finest-level M2L launch, timed alone with events on the
    # current stream (the stream the library launches on)
    shp = plan.level_shape(0)
    Mg = torch.randn(shp, dtype=plan.dtype, device=dev)
    Lg = torch.empty(shp, dtype=plan.dtype, device=dev)
    plan.m2l(0, Mg, Lg)
    torch.cuda.synchronize()
    k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k0.record()
    for _ in range(args.kernel_reps):
        plan.m2l(0, Mg, Lg)
    k1.record()
    torch.cuda.synchronize()
    m2l_ms = k0.elapsed_time(k1) / args.kernel_reps
    flops = accounting.m2l_flops(wl.dim, wl.n, wl.K, level=0)
    if args.m2l == "f32":
        bound, peak = "alu", PEAKS["fp32_vector_TFLOPs"]
    else:
        bound, peak = "mfma", PEAKS["bf16_mfma_TFLOPs"]
    achieved = flops / (m2l_ms * 1e-3) / 1e12
    passes = {"f32": 1, "bf16": 1, "bf16x2": 2, "bf16x3": 3}[args.m2l]
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None,
                "kernel": "m2l level 0 (finest), forward, %s" % args.m2l, "kernel_us": round(m2l_ms * 1e3, 2),
                "flops_per_launch": flops, "mfma_passes": passes,
                "mfma_issue_frac": round(achieved * passes * accounting.mfma_padding(wl.dim, wl.K) / peak, 4)
                if bound == "mfma" else None}

    unit = "queries/s" if wl.layer == "explicit" else "rays/s"
    outputs = {"explicit": "y, w_bar, p_bar, q_bar", "ray_integral": "y (ray integrals), w_bar, p_bar",
               "ray_root": "t*, grad f(q*), w_bar, p_bar"}[wl.layer]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": unit, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded %s sources, Gaussian weights)" % wl.sources,
        "config": {"workload": wl.name, "dim": wl.dim, "N": wl.N, "M": wl.M, "R": wl.R,
                   "grid": "%d^%d" % (wl.n, wl.dim), "K": wl.K, "kernel": "%s %g" % (wl.kernel, wl.param),
                   "m2l": args.m2l, "outputs": outputs},
        "roofline": roofline,
        "plan_ms": round(plan_ms, 1),
    }
    if f32_ms is not None:
        out["m2l_f32_comparison"] = {"value": round(units / (f32_ms * 1e-3), 1), "unit": unit,
                                     "ms_per_step": round(f32_ms, 4)}

    # ---- CPU baseline: the FP64 direct-sum checker on a bounded sample of queries (all N
    # sources), timed on this host; the same values give the GPU's error against it.
    if not args.no_cpu_baseline and wl.layer == "explicit":
        from oracle import direct, kernels
        idx = workloads.subsample(123, args.cpu_sample, wl.M)
        ker = kernels.make_kernel(wl.kernel, wl.param, wl.dim)
        threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        threads = min(threads, 16)
        c0 = time.perf_counter()
        yd = direct.explicit_y(ker, x["p"], x["w"], x["q"][idx], chunk=4, threads=threads)
        direct.explicit_grads(ker, x["p"], x["w"], x["q"][idx], x["gy"][idx], chunk=4, threads=threads)
        cpu_s = time.perf_counter() - c0
        yg = y.detach().cpu().numpy()[idx]
        err = float(np.linalg.norm(yg - yd) / np.linalg.norm(yd))
        out["cpu_baseline"] = {"value": round(len(idx) / cpu_s, 2), "unit": "queries/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "%d seeded queries x all %d sources, FP64 direct sum: y and the "
                                         "per-query gradient terms (q_bar and the w_bar/p_bar contributions); "
                                         "%.1f s" % (len(idx), wl.N, cpu_s)}
        out["rel_l2_vs_direct"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

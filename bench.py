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
    ap.add_argument("--m2l", default="bf16x3",
                    help="f32 | bf16 | bf16x2 | bf16x3 | separable (Gaussian kernels only)")
    ap.add_argument("--compare-f32", type=int, default=1,
                    help="also time the same step with the plain FP32 M2L (same accuracy class)")
    ap.add_argument("--fit", default="taylor", help="M2L tensor: taylor | lsq (least-squares fit)")
    ap.add_argument("--compare-fit", type=int, default=1,
                    help="explicit layers: also report the error of the other M2L tensor fit "
                         "against the same direct-sum sample")
    ap.add_argument("--compare-separable", type=int, default=1,
                    help="Gaussian kernels: also time the same step with the separable M2L")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1536, help="queries in the CPU sample")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device-to-device copies of MIB MiB (the reference "
                         "kernel for scaling HBM byte counters) and exit")
    return ap.parse_args()


def copy_calibration(mib):
    """Five device-to-device copies of a known size; each reads and writes mib MiB."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 5}), flush=True)


def source_hash():
    """sha256 over the library's kernel sources (names and contents, sorted by name)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2111_00110_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        with open(os.path.join(ROOT, "include", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, stage):
    """HBM bytes per launch of a stage's kernel from the committed counter summary
    profiles/<workload>_<stage>_hbm_counters.md, whose 'traffic-json:' line holds the scaled
    FETCH_SIZE + WRITE_SIZE bytes and the source hash they were taken at; None when there is
    no such summary or the kernels have changed since."""
    path = os.path.join(ROOT, "profiles", "%s_%s_hbm_counters.md" % (workload, stage))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic-json:"):
                rec = json.loads(line.split(":", 1)[1])
                if rec.get("source_hash") == source_hash():
                    return rec.get("bytes_per_launch")
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import torch
    from paper_2111_00110_amd import accounting, fc2t2, workloads

    torch.cuda.set_device(0)
    wl = workloads.workload(args.workload)
    x = workloads.make(wl, seed=0)
    dev = torch.device("cuda", 0)
    t = {k: torch.from_numpy(v).to(dev) for k, v in x.items()}
    def make_plan(m2l, fit=None):
        return fc2t2.Plan(wl.dim, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K, m2l=m2l, io=wl.io,
                          fit=fit or args.fit)

    p, w = t["p"], t["w"]
    q, gy = t.get("q"), t.get("gy")

    layer = wl.layer
    if layer != "explicit":
        o, r = t["o"], t["r"]

    def make_step(plan):
        Lt = plan.new_local()
        gL = plan.new_local()
        gp = torch.zeros_like(p)
        gw = torch.zeros_like(w)
        if layer == "explicit":
            gq = torch.zeros_like(q)

            def step():   # the backward calls overwrite the gradient buffers (no fills)
                plan.expand(p, w, out=Lt)
                y, _, _ = plan.eval(Lt, q)
                plan.eval_backward(Lt, q, gy, gL, gq, accumulate=False)
                plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
                return y
        elif layer == "ray_integral":
            def step():
                plan.expand(p, w, out=Lt)
                y = plan.ray_integral(Lt, o, r, wl.t0, wl.t1)
                gL.zero_()
                plan.ray_integral_backward(o, r, wl.t0, wl.t1, gy, gL)
                plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
                return y
        else:
            gt, gn = t["gt"], t["gn"]

            def step():
                plan.expand(p, w, out=Lt)
                tt, nrm, hit, saved = plan.ray_root(Lt, o, r, wl.t0, wl.t1, 0.5)
                gL.zero_()
                plan.ray_root_backward(saved, hit, gt, gn, gL)
                plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
                return tt
        return step

    def run(step, steps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
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
    step = make_step(plan)
    for _ in range(args.warmup):
        step()

    # ---- stage breakdown: the same steps with every stage bracketed by events on the
    # stream the library launches on (the current stream)
    plan.stage_timing(fc2t2.STAGES)
    run(step, args.steps)
    stages = {}
    for name in fc2t2.STAGES:
        st_ms, calls = plan.stage_time(name)
        if calls:
            stages[name] = {"ms_per_step": round(st_ms / args.steps, 4), "calls_per_step": calls // args.steps,
                            "ms_per_call": st_ms / calls}

    # ---- dominant kernel: the slowest single-kernel stage with a roofline model; the timed
    # region brackets only that stage's launches
    es = 8 if wl.io == "f64" else 4
    modelled = [n for n in ("m2l", "m2l_T", "p2m", "l2p", "l2p_T", "qgrad", "p2m_T") if n in stages]
    dom = max(modelled, key=lambda n: stages[n]["ms_per_step"])
    plan.stage_timing([dom])
    ms, y = run(step, args.steps)
    dom_ms, dom_calls = plan.stage_time(dom)
    plan.stage_timing([])
    kernel_ms = dom_ms / max(dom_calls, 1)
    units = wl.M if wl.layer == "explicit" else wl.R
    value = units / (ms * 1e-3)
    f32_ms = None
    if args.compare_f32 and args.m2l != "f32":
        plan32 = make_plan("f32")
        step32 = make_step(plan32)
        step32()
        f32_ms, _ = run(step32, max(3, args.steps // 4))

    sep_cmp = None
    if args.compare_separable and wl.kernel == "gaussian" and args.m2l != "separable":
        plan_s = make_plan("separable")
        step_s = make_step(plan_s)
        step_s()
        plan_s.stage_timing(["m2l", "m2l_T"])
        reps = max(3, args.steps // 4)
        sep_ms, _ = run(step_s, reps)
        sep_cmp = {"value": round((wl.M if wl.layer == "explicit" else wl.R) / (sep_ms * 1e-3), 1),
                   "ms_per_step": round(sep_ms, 4)}
        for name in ("m2l", "m2l_T"):
            st_ms, calls = plan_s.stage_time(name)
            sep_cmp[name + "_us_per_call"] = round(st_ms / max(calls, 1) * 1e3, 2)
        plan_s.stage_timing([])

    passes = {"f32": 1, "bf16": 1, "bf16x2": 2, "bf16x3": 3, "separable": None}[args.m2l]
    flops_dense = accounting.m2l_flops(wl.dim, wl.n, wl.K)
    separable = args.m2l == "separable"
    mfma = passes is not None and args.m2l != "f32"
    m2l_peak = PEAKS["bf16_mfma_TFLOPs"] if mfma else PEAKS["fp32_vector_TFLOPs"]
    # the MFMA path skips tiles with nothing to contribute: count the useful flops of the
    # tiles that run (source occupancy from the same FP32 cell index as the kernels)
    if mfma:
        occ = accounting.occupancy_pyramid(x["p"], wl.lo, wl.hi, wl.n, wl.dim)
        flops_run = {"m2l": accounting.m2l_flops_executed(wl.dim, wl.K, occ, False),
                     "m2l_T": accounting.m2l_flops_executed(wl.dim, wl.K, occ, True)}
    elif separable:
        f = accounting.m2l_flops_separable(wl.dim, wl.n, wl.K)
        flops_run = {"m2l": f, "m2l_T": f}
    else:
        flops_run = {"m2l": flops_dense, "m2l_T": flops_dense}

    def m2l_line(name):
        if name not in stages:
            return None
        kt = stages[name]["ms_per_call"]
        ach = flops_run[name] / (kt * 1e-3) / 1e12
        return {"kernel_us": round(kt * 1e3, 2), "achieved_TFLOPs": round(ach, 3), "peak_TFLOPs": m2l_peak,
                "frac": round(ach / m2l_peak, 4),
                "mfma_issue_frac": round(ach * passes * accounting.mfma_padding(wl.dim, wl.K) / m2l_peak, 4)
                if mfma else None,
                "flops_run": flops_run[name], "flops_dense": flops_dense,
                "dense_equivalent_TFLOPs": round(flops_dense / (kt * 1e-3) / 1e12, 3)}

    if dom in ("m2l", "m2l_T") and separable:
        # one launch per dimension (all levels, window and hole chains in each); the stage is
        # bound by its intermediate rows in HBM
        nbytes = accounting.m2l_bytes_separable(wl.dim, wl.n, wl.K, itemsize=es)
        achieved = nbytes / (kernel_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAKS["hbm_GBps"], "unit": "GB/s",
                    "frac": round(achieved / PEAKS["hbm_GBps"], 4), "traffic": None,
                    "kernel": "%s, separable: %d one-dimensional passes" % (dom, wl.dim),
                    "kernel_us": round(kernel_ms * 1e3, 2), "launches": dom_calls * wl.dim,
                    "bytes_per_launch": nbytes, "flops_per_launch": flops_run[dom], "flops_dense": flops_dense}
    elif dom in ("m2l", "m2l_T"):
        achieved = flops_run[dom] / (kernel_ms * 1e-3) / 1e12
        roofline = {"bound": "mfma" if mfma else "alu", "achieved": round(achieved, 3), "peak": m2l_peak,
                    "unit": "TFLOP/s", "frac": round(achieved / m2l_peak, 4), "traffic": None,
                    "kernel": "%s, all levels in one launch, %s" % (dom, args.m2l),
                    "kernel_us": round(kernel_ms * 1e3, 2), "launches": dom_calls,
                    "flops_per_launch": flops_run[dom], "flops_dense": flops_dense, "mfma_passes": passes}
    else:
        nbytes = accounting.stage_bytes(dom, wl.dim, wl.n, wl.K, N=wl.N, M=wl.M, itemsize=es)
        achieved = nbytes / (kernel_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAKS["hbm_GBps"], "unit": "GB/s",
                    "frac": round(achieved / PEAKS["hbm_GBps"], 4), "traffic": None,
                    "kernel": dom, "kernel_us": round(kernel_ms * 1e3, 2), "launches": dom_calls,
                    "bytes_per_launch": nbytes}
    traffic_key = dom + "_separable" if separable and dom in ("m2l", "m2l_T") else dom
    roofline["traffic"] = measured_traffic(wl.name, traffic_key)

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
                   "m2l": args.m2l, "fit": args.fit, "outputs": outputs},
        "roofline": roofline,
        ("m2l_separable" if separable else "m2l_mfma"): {"forward": m2l_line("m2l"),
                                                         "transpose": m2l_line("m2l_T")},
        "stages_ms_per_step": {k: v["ms_per_step"] for k, v in stages.items()},
        "plan_ms": round(plan_ms, 1),
    }
    if sep_cmp is not None:
        sep_cmp["unit"] = unit
        out["m2l_separable_comparison"] = sep_cmp
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
        if args.compare_fit and args.m2l != "separable":
            other = "lsq" if args.fit == "taylor" else "taylor"
            t0 = time.perf_counter()
            plan_o = make_plan(args.m2l, other)
            torch.cuda.synchronize()
            plan_o_ms = (time.perf_counter() - t0) * 1e3
            y_o, _, _ = plan_o.eval(plan_o.expand(p, w), q)
            yo = y_o.detach().cpu().numpy()[idx]
            out["fit_comparison"] = {"fit": other, "rel_l2_vs_direct": float(np.linalg.norm(yo - yd) / np.linalg.norm(yd)),
                                     "plan_ms": round(plan_o_ms, 1),
                                     "note": "same kernels and step time; only the plan's M2L tensor differs"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

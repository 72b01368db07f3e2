"""Throughput of the FC^2T^2 layers, forward + backward, on one MI355X.

Headline (the default run): the 3-D explicit layer, N = 2^21 shell sources, M = 10^7 uniform
queries, 64^3 grid on [-1, 1]^3, K = 4, inverse multiquadric eps = 0.02, FP32 IO, M2L on the
FP16 matrix cores with the hi/lo split (three passes).  One step = expansion of the sources
(bin + sort, P2M, M2M, M2L at every level, L2L), evaluation at the queries (L2P), and the
backward pass (sort of the queries, L2P^T, q_bar, L2L^T, M2L^T, M2M^T, P2M^T): y, w_bar,
p_bar, q_bar.  Inputs are resident in HBM before the timed region.

Prints one JSON line with
  * the throughput (queries/s) and the roofline of the dominant stage, timed live with HIP
    events on the stream the library launches on;
  * the whole-step roofline: sum over stages of max(bytes / HBM peak, flops / MFMA peak)
    against the measured step;
  * the accuracy on a seeded sample: eps_cfg = rel-L2(step-by-step FP64 checker, FP64 direct
    sum), the GPU's error against each, and the contract check;
  * the same step with the other M2L forms (BF16x3, plain FP32 on the matrix cores) with their
    errors, i.e. FP16x3 against FP32 at equal accuracy;
  * the FP64 direct-sum checker timed on the host's cores on a bounded sample (cpu_baseline);
  * the other workloads (2-D explicit, line integral, ray root, volumetric rendering, small
    FP64 case) under "other_workloads".
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
    "fp32_matrix_TFLOPs": 157.3,
    "bf16_mfma_TFLOPs": 2500.0,
    "fp16_mfma_TFLOPs": 2500.0,
    "fp64_TFLOPs": 78.6,
}
EPS_IMPL = 1e-5          # error contract against the step-by-step checker (values, w_bar)
PASSES = {"f32": 1, "f32_mfma": 1, "bf16": 1, "bf16x2": 2, "bf16x3": 3, "f16x3": 3, "separable": None}
MODELLED = ("sort", "p2m", "shift_up", "m2l", "shift_down", "l2p", "l2p_T", "qgrad", "m2l_T", "p2m_T")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="explicit3d_imq")
    ap.add_argument("--m2l", default="f16x3",
                    help="f16x3 | bf16x3 | bf16x2 | bf16 | f32_mfma | f32 | separable (Gaussian kernels only)")
    ap.add_argument("--fit", default="taylor", help="M2L tensor: taylor | lsq (least-squares fit)")
    ap.add_argument("--compare", type=int, default=1,
                    help="also time the step with the other M2L forms and report their errors")
    ap.add_argument("--others", type=int, default=1, help="also run the other workloads (extra key)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=768, help="queries in the CPU sample")
    ap.add_argument("--acc-sample", type=int, default=256, help="queries in the accuracy sample")
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


def host_threads():
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


class Runner:
    """One workload's inputs on the GPU and its step for a given M2L form."""

    def __init__(self, name, fit="taylor"):
        import torch
        from paper_2111_00110_amd import workloads
        self.torch = torch
        self.wl = workloads.workload(name)
        self.x = workloads.make(self.wl, seed=0)
        dev = torch.device("cuda", 0)
        self.t = {k: torch.from_numpy(v).to(dev) for k, v in self.x.items()}
        self.fit = fit
        self.unit = "queries/s" if self.wl.layer == "explicit" else "rays/s"
        self.units = self.wl.M if self.wl.layer == "explicit" else self.wl.R

    def plan(self, m2l):
        from paper_2111_00110_amd import fc2t2
        wl = self.wl
        return fc2t2.Plan(wl.dim, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K, m2l=m2l, io=wl.io, fit=self.fit,
                          channels=4 if wl.layer == "volume" else 1)

    def step_fn(self, plan):
        torch, wl, t = self.torch, self.wl, self.t
        p, w = t["p"], t["w"]
        Lt = plan.new_local()
        gL = plan.new_local()
        gp = torch.zeros_like(p)
        gw = torch.zeros_like(w)
        if wl.layer == "explicit" and wl.io == "f64":
            q = t["q"]

            def step():   # the small FP64 case: forward only
                plan.expand(p, w, out=Lt)
                y, _, _ = plan.eval(Lt, q)
                return y
        elif wl.layer == "explicit":
            q, gy = t["q"], t["gy"]
            gq = torch.zeros_like(q)

            ws = plan.workspace("eval_sorted", q.shape[0])
            side = torch.cuda.Stream()   # default priority

            def step():
                # queries sorted once per step, on a second stream while the expansion is built
                # (after the previous step's backward has read the records); the backward calls
                # overwrite their outputs
                main = torch.cuda.current_stream()
                side.wait_stream(main)
                with torch.cuda.stream(side):
                    plan.sort_queries(q, ws)
                plan.expand(p, w, out=Lt)
                main.wait_stream(side)
                y = plan.eval_presorted(Lt, q.shape[0], ws)
                plan.eval_backward_sorted(Lt, q.shape[0], gy, ws, gL, gq, accumulate=False)
                plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
                return y
        elif wl.layer == "ray_integral":
            o, r, gy = t["o"], t["r"], t["gy"]

            def step():
                plan.expand(p, w, out=Lt)
                y = plan.ray_integral(Lt, o, r, wl.t0, wl.t1)
                gL.zero_()
                plan.ray_integral_backward(o, r, wl.t0, wl.t1, gy, gL)
                plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
                return y
        elif wl.layer == "volume":
            o, r, gy = t["o"], t["r"], t["gy"]
            bg = tuple(float(v) for v in self.x["bg"])

            def step():
                plan.expand(p, w, out=Lt)
                y = plan.ray_volume(Lt, o, r, wl.t0, wl.t1, bg)
                gL.zero_()
                plan.ray_volume_backward(Lt, o, r, wl.t0, wl.t1, gy, gL, bg)
                plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
                return y
        else:
            o, r, gt, gn = t["o"], t["r"], t["gt"], t["gn"]

            def step():
                plan.expand(p, w, out=Lt)
                tt, nrm, hit, saved = plan.ray_root(Lt, o, r, wl.t0, wl.t1, 0.5)
                gL.zero_()
                plan.ray_root_backward(saved, hit, gt, gn, gL)
                plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
                return tt
        return step

    def run(self, step, steps):
        torch = self.torch
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(steps):
            y = step()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps, y

    def stages(self, plan, step, steps):
        """Per-stage event timing over `steps` steps: {stage: (ms per step, calls per step, ms per call)}."""
        from paper_2111_00110_amd import fc2t2
        plan.stage_timing(fc2t2.STAGES)
        self.run(step, steps)
        out = {}
        for name in fc2t2.STAGES:
            st_ms, calls = plan.stage_time(name)
            if calls:
                out[name] = (st_ms / steps, calls // steps, st_ms / calls)
        plan.stage_timing([])
        return out


def m2l_flops_run(wl, x, m2l):
    """Useful M2L flops of the tiles that run (forward, transpose)."""
    from paper_2111_00110_amd import accounting
    if m2l == "separable":
        f = accounting.m2l_flops_separable(wl.dim, wl.n, wl.K)
        return f, f
    if m2l in ("f32", "f64"):
        f = accounting.m2l_flops(wl.dim, wl.n, wl.K)
        return f, f
    occ = accounting.occupancy_pyramid(x["p"], wl.lo, wl.hi, wl.n, wl.dim)
    return (accounting.m2l_flops_executed(wl.dim, wl.K, occ, False),
            accounting.m2l_flops_executed(wl.dim, wl.K, occ, True))


def m2l_peak(m2l):
    if m2l in ("bf16", "bf16x2", "bf16x3"):
        return PEAKS["bf16_mfma_TFLOPs"], "mfma"
    if m2l == "f16x3":
        return PEAKS["fp16_mfma_TFLOPs"], "mfma"
    if m2l == "f32_mfma":
        return PEAKS["fp32_matrix_TFLOPs"], "mfma"
    return PEAKS["fp32_vector_TFLOPs"], "alu"


def m2l_lines(wl, st, m2l, flops):
    from paper_2111_00110_amd import accounting
    peak, _ = m2l_peak(m2l)
    dense = accounting.m2l_flops(wl.dim, wl.n, wl.K)
    out = {}
    for name, fl in (("forward", flops[0]), ("transpose", flops[1])):
        key = "m2l" if name == "forward" else "m2l_T"
        if key not in st:
            continue
        kt = st[key][2]
        ach = fl / (kt * 1e-3) / 1e12
        line = {"kernel_us": round(kt * 1e3, 2), "achieved_TFLOPs": round(ach, 3), "peak_TFLOPs": peak,
                "frac": round(ach / peak, 4), "flops_run": fl, "flops_dense": dense}
        if PASSES.get(m2l) and m2l not in ("f32", "f32_mfma"):
            line["mfma_issue_frac"] = round(ach * PASSES[m2l] * accounting.mfma_padding(wl.dim, wl.K) / peak, 4)
        out[name] = line
    return out


def whole_step(wl, st, ms, m2l, flops):
    """Sum over stages of max(bytes / HBM peak, flops / peak) against the measured step."""
    from paper_2111_00110_amd import accounting
    if wl.layer != "explicit" or wl.io != "f32":
        return None
    model = accounting.explicit_step_model(wl.dim, wl.n, wl.K, wl.N, wl.M, flops[0], flops[1])
    peak, _ = m2l_peak(m2l)
    stages = {}
    t_roof = 0.0
    for name, v in model.items():
        roof = accounting.stage_roof_us(v, PEAKS["hbm_GBps"], peak)
        t_roof += roof
        meas = st[name][0] * 1e3 if name in st else None
        stages[name] = {"roof_us": round(roof, 2), "measured_us": None if meas is None else round(meas, 2),
                        "bytes": v["bytes"], "flops": v["flops"],
                        "bound": "mfma" if v["flops"] / (peak * 1e6) > v["bytes"] / (PEAKS["hbm_GBps"] * 1e3) else "hbm"}
    return {"t_roof_us": round(t_roof, 1), "ms_per_step": round(ms, 4), "frac": round(t_roof * 1e-3 / ms, 4),
            "note": "M2L priced at useful flops of the tiles that run over the %s peak; other stages at their "
                    "algorithmic bytes over 8 TB/s" % m2l, "stages": stages}


def dominant_roofline(r, plan, step, st, steps, m2l, flops):
    """The slowest modelled single stage: timed again with only its launches bracketed."""
    from paper_2111_00110_amd import accounting
    wl = r.wl
    cands = [n for n in MODELLED if n in st and (n != "sort" or wl.layer == "explicit")]
    dom = max(cands, key=lambda n: st[n][0])
    plan.stage_timing([dom])
    ms, y = r.run(step, steps)
    dom_ms, dom_calls = plan.stage_time(dom)
    plan.stage_timing([])
    kernel_ms = dom_ms / max(dom_calls, 1)
    es = 8 if wl.io == "f64" else 4
    if dom in ("m2l", "m2l_T") and m2l == "separable":
        nbytes = accounting.m2l_bytes_separable(wl.dim, wl.n, wl.K, itemsize=es)
        ach = nbytes / (kernel_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAKS["hbm_GBps"], "unit": "GB/s",
                "frac": round(ach / PEAKS["hbm_GBps"], 4), "kernel": "%s, separable, %d one-dimensional passes"
                % (dom, wl.dim), "bytes_per_launch": nbytes}
    elif dom in ("m2l", "m2l_T"):
        fl = flops[0] if dom == "m2l" else flops[1]
        peak, bound = m2l_peak(m2l)
        ach = fl / (kernel_ms * 1e-3) / 1e12
        roof = {"bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4), "kernel": "%s, all levels in one launch, %s" % (dom, m2l),
                "flops_per_launch": fl, "mfma_passes": PASSES.get(m2l)}
    else:
        model = accounting.explicit_step_model(wl.dim, wl.n, wl.K, wl.N, wl.M, 0, 0, itemsize=es)
        nbytes = model[dom]["bytes"]
        if dom == "sort":
            # the stage's calls differ (sources, queries, source occupancy): priced per step
            kernel_ms, dom_calls = dom_ms / steps, dom_calls // steps
        ach = nbytes / (kernel_ms * 1e-3) / 1e9
        label = dom if dom != "sort" else ("sort stage per step: sources and queries by cell (keys and digit "
                                          "histograms, %d one-sweep passes, cell starts each) and the sources' "
                                          "occupancy; several launches" % accounting.key_passes(wl.n ** wl.dim))
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAKS["hbm_GBps"], "unit": "GB/s",
                "frac": round(ach / PEAKS["hbm_GBps"], 4), "kernel": label, "bytes_per_launch": nbytes}
    roof["kernel_us"] = round(kernel_ms * 1e3, 2)
    roof["launches"] = dom_calls
    key = dom + "_separable" if m2l == "separable" and dom in ("m2l", "m2l_T") else dom
    roof["traffic"] = measured_traffic(wl.name, key) if m2l != "separable" or dom.startswith("m2l") else None
    return dom, ms, y, roof


def checker_sample(wl, x, idx, fit="taylor"):
    """Step-by-step FP64 checker (locals cell by cell from the full moment pyramid) at sampled
    queries: y [S, C]."""
    from oracle import fmm, kernels
    geo = fmm.Geometry(wl.dim, wl.n, wl.lo, wl.hi, wl.K, np.float32 if wl.io == "f32" else np.float64, fit)
    ker = kernels.make_kernel(wl.kernel, wl.param, wl.dim)
    qs = x["q"][idx]
    cells = geo.cell_index(qs)
    Lc = fmm.locals_at_cells(geo, ker, fmm.moments_all_levels(geo, x["p"], x["w"]), cells)
    dvec = qs.astype(np.float64) - geo.centre(0, cells)
    return np.einsum("csp,sp->sc", Lc, fmm.monomials(dvec, geo.idx))


def accuracy(r, y_gpu, sample, threads):
    """eps_cfg, the GPU's errors, and the contract check on a seeded query sample."""
    from oracle import direct, kernels
    from paper_2111_00110_amd import workloads
    wl, x = r.wl, r.x
    idx = workloads.subsample(321, sample, wl.M)
    ker = kernels.make_kernel(wl.kernel, wl.param, wl.dim)
    yd = direct.explicit_y(ker, x["p"], x["w"], x["q"][idx], chunk=4, threads=threads)
    yf = checker_sample(wl, x, idx, r.fit)
    yg = y_gpu[idx]
    eps_cfg = rel(yf, yd)
    vs_direct = rel(yg, yd)
    return idx, yd, yf, {
        "eps_cfg": eps_cfg, "eps_impl": rel(yg, yf), "rel_l2_vs_direct": vs_direct,
        "bound": 1.05 * eps_cfg + EPS_IMPL, "holds": bool(vs_direct <= 1.05 * eps_cfg + EPS_IMPL),
        "sample": "%d seeded queries; eps_cfg = rel-L2(FP64 step-by-step checker, FP64 direct sum), "
                  "eps_impl = rel-L2(GPU, checker) with contract %g" % (len(idx), EPS_IMPL)}


def cpu_baseline(r, sample, threads):
    """The FP64 direct-sum checker on a bounded query sample against all sources, on the host."""
    from oracle import direct, kernels
    from paper_2111_00110_amd import workloads
    wl, x = r.wl, r.x
    idx = workloads.subsample(123, sample, wl.M)
    ker = kernels.make_kernel(wl.kernel, wl.param, wl.dim)
    c0 = time.perf_counter()
    direct.explicit_y(ker, x["p"], x["w"], x["q"][idx], chunk=4, threads=threads)
    if wl.io == "f32":
        direct.explicit_grads(ker, x["p"], x["w"], x["q"][idx], x["gy"][idx], chunk=4, threads=threads)
    cpu_s = time.perf_counter() - c0
    what = "y and the per-query gradient terms (q_bar and the w_bar/p_bar contributions)" if wl.io == "f32" else "y"
    return {"value": round(len(idx) / cpu_s, 2), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "host_cpu_count": os.cpu_count(),
            "sample": "%d seeded queries x all %d sources, FP64 direct sum: %s; %.1f s on %d threads"
                      % (len(idx), wl.N, what, cpu_s, threads)}


def cpu_baseline_rays(r, rays, threads):
    """Ray integrals of the Gaussian direct sum in closed form (erf per source) for a bounded ray
    sample, on the host."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import direct
    from paper_2111_00110_amd import workloads
    wl, x = r.wl, r.x
    idx = workloads.subsample(124, rays, wl.R)

    def one(i):
        ta, tb = direct.clip_ray(x["o"][i], x["r"][i], wl.t0, wl.t1, wl.lo, wl.hi)
        return direct.ray_integral_gaussian(wl.param, x["p"], x["w"], x["o"][i], x["r"][i], ta, tb)
    c0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, idx))
    cpu_s = time.perf_counter() - c0
    return {"value": round(len(idx) / cpu_s, 2), "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded rays x all %d sources, FP64 closed-form Gaussian line integrals (forward only); "
                      "%.1f s" % (len(idx), wl.N, cpu_s)}


def other_workload(name, m2l, steps, warmup, threads):
    r = Runner(name)
    wl = r.wl
    form = m2l if wl.io == "f32" else "f64"
    if wl.kernel != "gaussian" and form == "separable":
        form = "f16x3"
    plan = r.plan(form)
    step = r.step_fn(plan)
    for _ in range(warmup):
        step()
    st = r.stages(plan, step, max(2, steps // 2))
    ms, y = r.run(step, steps)
    flops = m2l_flops_run(wl, r.x, form) if form != "f64" else (0, 0)
    out = {"value": round(r.units / (ms * 1e-3), 1), "unit": r.unit, "ms_per_step": round(ms, 4), "m2l": form,
           "config": {"dim": wl.dim, "N": wl.N, "M": wl.M, "R": wl.R, "grid": "%d^%d" % (wl.n, wl.dim), "K": wl.K,
                      "kernel": "%s %g" % (wl.kernel, wl.param), "io": wl.io,
                      "outputs": {"explicit": "y, w_bar, p_bar, q_bar" if wl.io == "f32" else "y (forward only)",
                                  "ray_integral": "y, w_bar, p_bar", "ray_root": "t*, grad f(q*), w_bar, p_bar",
                                  "volume": "colour y, w_bar, p_bar (four channels)"}[wl.layer]},
           "stages_ms_per_step": {k: round(v[0], 4) for k, v in st.items()}}
    if form != "f64":
        out["m2l_mfma"] = m2l_lines(wl, st, form, flops)
        ws = whole_step(wl, st, ms, form, flops)
        if ws is not None:
            out["whole_step"] = {k: ws[k] for k in ("t_roof_us", "ms_per_step", "frac")}
    if wl.layer == "explicit":
        yg = y.detach().cpu().numpy()
        _, _, _, acc = accuracy(r, yg, 128 if wl.M > 4096 else wl.M, threads)
        out["accuracy"] = acc
        if wl.io == "f32":
            out["cpu_baseline"] = cpu_baseline(r, 128, threads)
    elif wl.layer == "ray_integral":
        out["cpu_baseline"] = cpu_baseline_rays(r, 32, threads)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library is single-GPU (no collectives), so --gpus %d is not "
              "supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import torch
    torch.cuda.set_device(0)
    threads = host_threads()
    r = Runner(args.workload, fit=args.fit)
    wl = r.wl

    t_plan0 = time.perf_counter()
    plan = r.plan(args.m2l)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t_plan0) * 1e3
    step = r.step_fn(plan)
    for _ in range(args.warmup):
        step()
    st = r.stages(plan, step, args.steps)
    flops = m2l_flops_run(wl, r.x, args.m2l)
    dom, ms, y, roofline = dominant_roofline(r, plan, step, st, args.steps, args.m2l, flops)
    value = r.units / (ms * 1e-3)

    outputs = {"explicit": "y, w_bar, p_bar, q_bar", "ray_integral": "y (ray integrals), w_bar, p_bar",
               "ray_root": "t*, grad f(q*), w_bar, p_bar", "volume": "colour y, w_bar, p_bar (four channels)"}[wl.layer]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": r.unit, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded %s sources, Gaussian weights and cotangents)" % wl.sources,
        "config": {"workload": wl.name, "dim": wl.dim, "N": wl.N, "M": wl.M, "R": wl.R,
                   "grid": "%d^%d" % (wl.n, wl.dim), "K": wl.K, "kernel": "%s %g" % (wl.kernel, wl.param),
                   "m2l": args.m2l, "fit": args.fit, "outputs": outputs},
        "roofline": roofline,
        "whole_step": whole_step(wl, st, ms, args.m2l, flops),
        ("m2l_separable" if args.m2l == "separable" else "m2l_mfma"): m2l_lines(wl, st, args.m2l, flops),
        "stages_ms_per_step": {k: round(v[0], 4) for k, v in st.items()},
        "plan_ms": round(plan_ms, 1),
    }

    acc_idx = None
    if wl.layer == "explicit":
        yg = y.detach().cpu().numpy()
        acc_idx, yd, yf, out["accuracy"] = accuracy(r, yg, args.acc_sample, threads)

    if args.compare and wl.io == "f32":
        forms = {}
        for form in ("f16x3", "bf16x3", "f32_mfma") + (("separable",) if wl.kernel == "gaussian" else ()):
            if form == args.m2l:
                continue
            pl = r.plan(form)
            stp = r.step_fn(pl)
            stp()
            reps = max(3, args.steps // 4)
            fms, fy = r.run(stp, reps)
            rec = {"value": round(r.units / (fms * 1e-3), 1), "unit": r.unit, "ms_per_step": round(fms, 4)}
            if acc_idx is not None:
                fyg = fy.detach().cpu().numpy()[acc_idx]
                rec["eps_impl"] = rel(fyg, yf)
                rec["rel_l2_vs_direct"] = rel(fyg, yd)
            forms[form] = rec
            del pl
        out["m2l_forms"] = forms

    if not args.no_cpu_baseline:
        if wl.layer == "explicit":
            out["cpu_baseline"] = cpu_baseline(r, args.cpu_sample, threads)
        elif wl.layer == "ray_integral":
            out["cpu_baseline"] = cpu_baseline_rays(r, 64, threads)

    if args.others:
        del r, plan
        torch.cuda.empty_cache()
        others = {}
        for name in ("explicit2d", "ray_integral3d", "ray_root3d", "volume3d", "explicit2d_small"):
            if name == args.workload:
                continue
            others[name] = other_workload(name, args.m2l,
                                          args.steps, args.warmup, threads)
            torch.cuda.empty_cache()
        out["other_workloads"] = others
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

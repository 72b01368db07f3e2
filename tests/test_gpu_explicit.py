"""GPU parity of the explicit layer (expansion, evaluation, backward) against the FP64
checker, through the C-ABI.  Tolerances: FP64 path 1e-12 relative L2 against the
step-by-step checker; FP32 path 1e-5 on values and w_bar, 1e-4 on the gradient-derived
p_bar and q_bar (one order of the expansion is lost by differentiating)."""
import numpy as np
import pytest

from oracle import direct, fmm, kernels
from paper_2111_00110_amd import workloads as W

from helpers import oracle_geometry, oracle_kernel, poly_coef_list, rel, scaled_locals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_00110_amd import fc2t2
    return fc2t2


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _plan(F, wl, m2l=None, coef=None, channels=1):
    m2l = m2l or ("f64" if wl.io == "f64" else "f32")
    return F.Plan(wl.dim, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K, m2l=m2l, io=wl.io,
                  channels=channels, coef=coef)


def _run_gpu(F, plan, x):
    p, w, q, gy = (_dev(x[k]) for k in ("p", "w", "q", "gy"))
    Lt = plan.expand(p, w)
    y, g, _ = plan.eval(Lt, q, grad=True)
    gL = plan.new_local()
    gq = torch.zeros_like(q)
    plan.eval_backward(Lt, q, gy, gL, gq)
    gp = torch.zeros_like(p)
    gw = torch.zeros_like(w)
    plan.expand_backward(gL, p, w, gp, gw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in dict(L=Lt, y=y, g=g, gL=gL, gq=gq, gp=gp, gw=gw).items()}


def test_small_2d_fp64_matches_checker(F):
    wl = W.workload("explicit2d_small")
    x = W.make(wl)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    got = _run_gpu(F, plan, x)
    L0 = fmm.expand(geo, ker, x["p"], x["w"])
    assert rel(got["L"], scaled_locals(geo, L0, plan.P_pad)) < 1e-12
    y, gw, gp, gq = fmm.explicit_forward_backward(geo, ker, x["p"], x["w"], x["q"], x["gy"])
    assert rel(got["y"], y) < 1e-12
    assert rel(got["gw"], gw) < 1e-12
    assert rel(got["gp"], gp) < 1e-12
    assert rel(got["gq"], gq) < 1e-12
    gdir = fmm.l2p_grad(geo, L0, x["q"])
    assert rel(got["g"], gdir) < 1e-12


@pytest.mark.parametrize("d,n,K", [(2, 8, 4), (2, 32, 6), (3, 8, 3), (3, 16, 5)])
def test_polynomial_kernel_fp64_equals_direct_sum(F, d, n, K):
    rng = np.random.default_rng(7 * n + K)
    deg = min(K, 4)
    coef = {a: rng.standard_normal() for a in fmm.multi_indices(d, deg)}
    ker = kernels.Polynomial(coef, d)
    wl = W.Workload("poly", d, n, -1.0, 1.0, K, "poly", 0.0, 700, 500, 0, "f64", "explicit", "uniform")
    p = rng.uniform(-1, 1, (700, d))
    q = rng.uniform(-1, 1, (500, d))
    w = rng.standard_normal((700, 2))
    gy = rng.standard_normal((500, 2))
    plan = _plan(F, wl, coef=poly_coef_list(ker, d, deg), channels=2)
    got = _run_gpu(F, plan, dict(p=p, q=q, w=w, gy=gy))
    assert rel(got["y"], direct.explicit_y(ker, p, w, q)) < 1e-11
    gwd, gpd, gqd = direct.explicit_grads(ker, p, w, q, gy)
    assert rel(got["gw"], gwd) < 1e-11
    assert rel(got["gp"], gpd) < 1e-10
    assert rel(got["gq"], gqd) < 1e-10


@pytest.mark.parametrize("name,N,M,n", [("explicit2d", 1 << 15, 1 << 14, 256), ("explicit2d", 3001, 2999, 64)])
def test_2d_fp32_matches_checker(F, name, N, M, n):
    wl = W.workload(name, N=N, M=M, n=n)
    x = W.make(wl, seed=1)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    got = _run_gpu(F, plan, x)
    y, gw, gp, gq = fmm.explicit_forward_backward(geo, ker, x["p"], x["w"], x["q"], x["gy"])
    assert rel(got["y"], y) < 1e-5
    assert rel(got["gw"], gw) < 1e-5
    assert rel(got["gp"], gp) < 1e-4
    assert rel(got["gq"], gq) < 1e-4


@pytest.mark.parametrize("kind,param,K", [("gaussian", 0.05, 4), ("imq", 0.1, 3), ("gaussian", 0.06, 5)])
@pytest.mark.parametrize("io", ["f64", "f32"])
def test_3d_small_matches_checker(F, kind, param, K, io):
    wl = W.Workload("t3", 3, 16, -1.0, 1.0, K, kind, param, 4000, 3000, 0, io, "explicit", "shell")
    x = W.make(wl, seed=2)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    got = _run_gpu(F, plan, x)
    y, gw, gp, gq = fmm.explicit_forward_backward(geo, ker, x["p"], x["w"], x["q"], x["gy"])
    tol, tolg = (1e-12, 1e-12) if io == "f64" else (1e-5, 1e-4)
    assert rel(got["y"], y) < tol
    assert rel(got["gw"], gw) < tol
    assert rel(got["gp"], gp) < tolg
    assert rel(got["gq"], gq) < tolg


def test_bitwise_deterministic(F):
    wl = W.workload("explicit2d", N=1 << 16, M=1 << 15, n=128)
    x = W.make(wl, seed=3)
    plan = _plan(F, wl)
    a = _run_gpu(F, plan, x)
    b = _run_gpu(F, plan, x)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_edge_cases(F):
    wl = W.Workload("e", 2, 16, 0.0, 1.0, 4, "gaussian", 0.05, 0, 0, 0, "f64", "explicit", "uniform")
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    # no sources: zero expansion, zero output
    Lt = plan.expand(_dev(np.zeros((0, 2))), _dev(np.zeros((0, 1))))
    q = np.random.default_rng(0).uniform(0, 1, (37, 2))
    y, _, _ = plan.eval(Lt, _dev(q))
    assert float(torch.abs(Lt).max()) == 0.0 and float(torch.abs(y).max()) == 0.0
    # no queries
    y0, _, _ = plan.eval(Lt, _dev(np.zeros((0, 2))))
    assert y0.shape == (0, 1)
    # all sources in one cell, points on faces and outside the domain (clamped)
    p = np.array([[0.51, 0.52]] * 50 + [[0.0, 0.0], [1.0, 1.0], [0.5, 0.25], [-0.01, 0.3], [1.02, 0.7]])
    w = np.random.default_rng(1).standard_normal((len(p), 1))
    qq = np.array([[0.5, 0.5], [0.0, 1.0], [0.999, 0.001], [0.3, 0.7]])
    got = _run_gpu(F, plan, dict(p=p, w=w, q=qq, gy=np.ones((4, 1))))
    y, gw, gp, gq = fmm.explicit_forward_backward(geo, ker, p, w, qq, np.ones((4, 1)))
    assert rel(got["y"], y) < 1e-12 and rel(got["gw"], gw) < 1e-12 and rel(got["gp"], gp) < 1e-12


def test_stage_timing_records_each_stage(F):
    """The library's event bracketing: every stage of one explicit step is timed once per call
    (two sorts: sources and queries), and turning timing off records nothing further."""
    wl = W.workload("explicit2d", N=1 << 15, M=1 << 14, n=64)
    x = W.make(wl, seed=5)
    plan = _plan(F, wl, m2l="bf16x3")
    plan.stage_timing(F.STAGES)
    _run_gpu(F, plan, x)
    want = {"sort": 3, "p2m": 1, "shift_up": 2, "m2l": 1, "shift_down": 2, "l2p": 1, "l2p_T": 1,
            "m2l_T": 1, "p2m_T": 1, "qgrad": 1}
    for name, calls in want.items():
        ms, n = plan.stage_time(name)
        assert n == calls, (name, n)
        assert ms > 0.0, name
    assert plan.stage_time("ray") == (0.0, 0)
    plan.stage_timing([])
    _run_gpu(F, plan, x)
    assert plan.stage_time("m2l") == (0.0, 0)


@pytest.mark.parametrize("case", ["2d_gauss", "3d_imq", "2d_poly"])
def test_lsq_fitted_tensors_match_checker(F, case):
    """Least-squares fitted M2L tensors (section 3.1), FP64 IO against the checker with the same
    fit (the fit's normal equations limit agreement to about 1e-10), and for a polynomial kernel
    of degree K against the Taylor plan (the fit is exact there)."""
    coef = None
    if case == "2d_gauss":
        wl = W.Workload("l", 2, 32, 0.0, 1.0, 4, "gaussian", 0.02, 3000, 2000, 0, "f64", "explicit", "uniform")
    elif case == "3d_imq":
        wl = W.Workload("l", 3, 8, -1.0, 1.0, 3, "imq", 0.3, 1500, 1000, 0, "f64", "explicit", "uniform")
    else:
        wl = W.Workload("l", 2, 16, -1.0, 1.0, 4, "poly", 0.0, 700, 500, 0, "f64", "explicit", "uniform")
        rng = np.random.default_rng(4)
        c = {a: rng.standard_normal() for a in fmm.multi_indices(2, 4)}
        ker_p = kernels.Polynomial(c, 2)
        coef = poly_coef_list(ker_p, 2, 4)
    x = W.make(wl, seed=6)
    plan = F.Plan(wl.dim, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K, m2l="f64", io="f64", coef=coef, fit="lsq")
    got = _run_gpu(F, plan, x)
    if case == "2d_poly":
        ref = _run_gpu(F, _plan(F, wl, coef=coef), x)
        for k in ("y", "gw", "gp", "gq"):
            assert rel(got[k], ref[k]) < 1e-9, k
        return
    geo = fmm.Geometry(wl.dim, wl.n, wl.lo, wl.hi, wl.K, fit="lsq")
    y, gw, gp, gq = fmm.explicit_forward_backward(geo, oracle_kernel(wl), x["p"], x["w"], x["q"], x["gy"])
    assert rel(got["y"], y) < 1e-10
    assert rel(got["gw"], gw) < 1e-10
    assert rel(got["gp"], gp) < 1e-9
    assert rel(got["gq"], gq) < 1e-9


def test_lsq_fitted_tensors_bf16x3(F):
    """The fitted tensors feed the MFMA tables too: BF16x3 against the checker's fitted layer."""
    wl = W.Workload("l", 2, 64, 0.0, 1.0, 6, "gaussian", 0.01, 1 << 14, 1 << 12, 0, "f32", "explicit", "uniform")
    x = W.make(wl, seed=8)
    plan = F.Plan(wl.dim, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K, m2l="bf16x3", io="f32", fit="lsq")
    got = _run_gpu(F, plan, x)
    geo = fmm.Geometry(wl.dim, wl.n, wl.lo, wl.hi, wl.K, np.float32, fit="lsq")
    y, gw, gp, gq = fmm.explicit_forward_backward(geo, oracle_kernel(wl), x["p"], x["w"], x["q"], x["gy"])
    assert rel(got["y"], y) < 3e-5
    assert rel(got["gw"], gw) < 3e-5
    assert rel(got["gp"], gp) < 5e-5
    assert rel(got["gq"], gq) < 5e-5


@pytest.mark.parametrize("io,C", [("f32", 1), ("f64", 1), ("f32", 2)])
def test_backward_overwrite_equals_zero_then_accumulate(F, io, C):
    """accumulate=False writes the gradients over whatever the buffers held: the same values as
    zeroed buffers accumulated into (every backward path: sorted records with carried data,
    the fused FP64 pass, several channels), and an empty query set zeroes gL."""
    wl = W.Workload("o", 2, 32, 0.0, 1.0, 4, "gaussian", 0.03, 3000, 2000, 0, io, "explicit", "uniform")
    x = W.make(wl, seed=12)
    rng = np.random.default_rng(13)
    x["w"] = rng.standard_normal((wl.N, C)).astype(x["p"].dtype)
    x["gy"] = rng.standard_normal((wl.M, C)).astype(x["p"].dtype)
    plan = _plan(F, wl, channels=C)
    p, w, q, gy = (_dev(x[k]) for k in ("p", "w", "q", "gy"))
    Lt = plan.expand(p, w)
    res = {}
    for acc in (True, False):
        fill = (lambda t: t.zero_()) if acc else (lambda t: t.fill_(7.5))
        gL = fill(plan.new_local())
        gq, gp, gw = fill(torch.empty_like(q)), fill(torch.empty_like(p)), fill(torch.empty_like(w))
        plan.eval_backward(Lt, q, gy, gL, gq, accumulate=acc)
        plan.expand_backward(gL, p, w, gp, gw, accumulate=acc)
        torch.cuda.synchronize()
        res[acc] = [t.cpu().numpy() for t in (gL, gq, gp, gw)]
    for a, b in zip(res[True], res[False]):
        assert np.array_equal(a, b)
    gL = plan.new_local().fill_(3.0)
    plan.eval_backward(Lt, q[:0], gy[:0], gL, None, accumulate=False)
    torch.cuda.synchronize()
    assert float(gL.abs().max()) == 0.0


def test_out_of_domain_points_are_counted(F, monkeypatch):
    """Sources and queries outside the domain (and NaN) are counted on the device; reset zeroes
    the count; in debug mode the call that met them raises."""
    plan = F.Plan(2, 16, 0.0, 1.0, "gaussian", 0.05, 3, m2l="f32", io="f32")
    rng = np.random.default_rng(3)
    p = rng.uniform(0, 1, (5000, 2)).astype(np.float32)
    p[:37, 0] = 1.5
    p[37:40, 1] = -0.25
    p[40, 0] = np.nan
    q = rng.uniform(0, 1, (3000, 2)).astype(np.float32)
    q[-5:, 1] = 2.0
    w = np.ones((5000, 1), np.float32)
    Lt = plan.expand(_dev(p), _dev(w))
    assert plan.out_of_domain() == 41
    plan.eval(Lt, _dev(q))
    assert plan.out_of_domain(reset=True) == 46
    assert plan.out_of_domain() == 0
    plan.eval(Lt, _dev(q[:-5]))
    assert plan.out_of_domain() == 0
    monkeypatch.setenv("FC2T2_DEBUG", "1")
    with pytest.raises(F.FC2T2Error):
        plan.eval(Lt, _dev(q))
    plan.eval(Lt, _dev(q[:-5]))


@pytest.mark.parametrize("d,io", [(2, "f64"), (3, "f64"), (2, "f32"), (3, "f32")])
def test_eval_hessian_matches_checker(F, d, io):
    """The Hessian output of fc2t2_eval (upper triangle row by row) against the checker's L2P
    Hessian, with the value and gradient outputs of the same call."""
    lo, hi = (0.0, 1.0) if d == 2 else (-1.0, 1.0)
    K = 5 if d == 2 else 4
    wl = W.Workload("h", d, 16, lo, hi, K, "gaussian", 0.06, 3000, 2000, 0, io, "explicit",
                    "uniform" if d == 2 else "shell")
    x = W.make(wl, seed=9)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    Lt = plan.expand(_dev(x["p"]), _dev(x["w"]))
    y, g, hs = plan.eval(Lt, _dev(x["q"]), grad=True, hess=True)
    L0 = fmm.expand(geo, ker, x["p"], x["w"])
    H = fmm.l2p_hess(geo, L0, x["q"])                        # [M, C, d, d]
    iu = np.triu_indices(d)
    want = H[:, :, iu[0], iu[1]]
    tol = 1e-12 if io == "f64" else 1e-4
    assert rel(hs.cpu().numpy(), want) < tol
    assert rel(g.cpu().numpy(), fmm.l2p_grad(geo, L0, x["q"])) < tol
    assert rel(y.cpu().numpy(), fmm.l2p(geo, L0, x["q"])) < (1e-12 if io == "f64" else 1e-5)


@pytest.mark.parametrize("d,io_kernel", [(2, ("gaussian", 0.03)), (3, ("imq", 0.1))])
def test_sorted_query_path_matches_checker_and_unsorted(F, d, io_kernel):
    """fc2t2_eval_sorted + fc2t2_eval_backward_sorted (queries sorted once, q_bar fused into the
    transpose of L2P) against the checker at the contract, and bitwise equal to the unsorted
    calls (same formulas, same per-cell summation order); overwrite and accumulate; M = 0."""
    kern, par = io_kernel
    lo, hi = (0.0, 1.0) if d == 2 else (-1.0, 1.0)
    wl = W.Workload("s", d, 32 if d == 2 else 16, lo, hi, 4, kern, par, 5000, 7001, 0, "f32", "explicit", "uniform")
    x = W.make(wl, seed=14)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    p, w, q, gy = (_dev(x[k]) for k in ("p", "w", "q", "gy"))
    Lt = plan.expand(p, w)
    y_s, ws = plan.eval_sorted(Lt, q)
    gL_s, gq_s = plan.new_local().fill_(5.0), torch.empty_like(q).fill_(5.0)
    plan.eval_backward_sorted(Lt, wl.M, gy, ws, gL_s, gq_s, accumulate=False)
    y_u, _, _ = plan.eval(Lt, q)
    gL_u, gq_u = plan.new_local(), torch.zeros_like(q)
    plan.eval_backward(Lt, q, gy, gL_u, gq_u)
    torch.cuda.synchronize()
    assert torch.equal(y_s, y_u)
    assert torch.equal(gL_s, gL_u)
    assert torch.equal(gq_s, gq_u)
    plan.eval_backward_sorted(Lt, wl.M, gy, ws, gL_s, gq_s, accumulate=True)
    assert torch.allclose(gL_s, 2 * gL_u, rtol=1e-6, atol=0) and torch.allclose(gq_s, 2 * gq_u, rtol=1e-6, atol=0)
    L0 = fmm.expand(geo, ker, x["p"], x["w"])
    assert rel(y_s.cpu().numpy(), fmm.l2p(geo, L0, x["q"])) < 1e-5
    gq_ref = np.einsum("mc,mcj->mj", x["gy"].astype(np.float64), fmm.l2p_grad(geo, L0, x["q"]))
    assert rel(gq_u.cpu().numpy(), gq_ref) < 1e-4
    G = fmm.l2p_T(geo, x["q"], x["gy"])
    from helpers import scaled_cotangent
    assert rel(gL_u.cpu().numpy(), scaled_cotangent(geo, G, plan.P_pad)) < 1e-5
    # no queries: overwrite zeroes gL
    y0, ws0 = plan.eval_sorted(Lt, q[:0])
    gL0 = plan.new_local().fill_(1.0)
    plan.eval_backward_sorted(Lt, 0, gy[:0], ws0, gL0, None, accumulate=False)
    assert y0.shape == (0, 1) and float(gL0.abs().max()) == 0.0


def test_query_sort_on_a_side_stream_matches_eval_sorted(F):
    """fc2t2_sort_queries on a second stream while the expansion runs on the first, then
    fc2t2_eval_presorted after the streams join: y and the backward from the sorted records are
    bitwise those of fc2t2_eval_sorted, over three steps reusing one workspace."""
    wl = W.workload("explicit3d_imq", N=1 << 15, M=50_001, n=32)
    x = W.make(wl, seed=23)
    plan = _plan(F, wl)
    p, w, q, gy = (_dev(x[k]) for k in ("p", "w", "q", "gy"))
    Lt = plan.expand(p, w)
    y_ref, ws_ref = plan.eval_sorted(Lt, q)
    gL_ref, gq_ref = plan.new_local(), torch.empty_like(q)
    plan.eval_backward_sorted(Lt, wl.M, gy, ws_ref, gL_ref, gq_ref, accumulate=False)
    ws = plan.workspace("eval_sorted", wl.M)
    L2 = plan.new_local()
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    for _ in range(3):
        side.wait_stream(main)
        with torch.cuda.stream(side):
            plan.sort_queries(q, ws)
        plan.expand(p, w, out=L2)
        main.wait_stream(side)
        y = plan.eval_presorted(L2, wl.M, ws)
        gL, gq = plan.new_local().fill_(3.0), torch.empty_like(q).fill_(3.0)
        plan.eval_backward_sorted(L2, wl.M, gy, ws, gL, gq, accumulate=False)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        assert torch.equal(gL, gL_ref) and torch.equal(gq, gq_ref)
    assert plan.sort_failures() == 0
    e = plan.sort_queries(q[:0])
    assert plan.eval_presorted(Lt, 0, e).shape == (0, 1)


def test_explicit_autograd_uses_sorted_queries(F):
    """The autograd wrapper (sorted-query path for FP32, one channel) against the unsorted calls."""
    wl = W.workload("explicit2d", N=1 << 14, M=1 << 13, n=64)
    x = W.make(wl, seed=15)
    plan = _plan(F, wl)
    assert plan.sorted_queries
    p, w, q = (_dev(x[k]).requires_grad_(True) for k in ("p", "w", "q"))
    y = F.Explicit.apply(plan, p, w, q)
    (y * _dev(x["gy"])).sum().backward()
    got = _run_gpu(F, plan, x)
    assert np.array_equal(y.detach().cpu().numpy(), got["y"])
    assert rel(w.grad.cpu().numpy(), got["gw"]) < 1e-6
    assert rel(p.grad.cpu().numpy(), got["gp"]) < 1e-6
    assert np.array_equal(q.grad.cpu().numpy(), got["gq"])

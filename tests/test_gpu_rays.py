"""GPU parity of the ray layers (line integral, ray insertion, first level crossing and
its implicit-function-theorem backward) against the FP64 checker, through the C-ABI.

Stage tests feed both sides the same expansion (rounded to the IO type first) so that the
ray stage is compared on its own; end-to-end tests compare the GPU's expansion + ray stage
with the checker's."""
import numpy as np
import pytest

from oracle import fmm, rays
from paper_2111_00110_amd import workloads as W

from helpers import (oracle_geometry, oracle_kernel, physical_locals, rays_toward_origin, rel,
                     scaled_cotangent, scaled_locals)

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


def _wl(n=16, K=4, sigma=0.06, N=3000, io="f32", R=96, layer="ray_root"):
    return W.Workload("r", 3, n, -1.0, 1.0, K, "gaussian", sigma, N, 0, R, io, layer, "shell")


def _plan(F, wl, channels=1):
    return F.Plan(3, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K,
                  m2l="f64" if wl.io == "f64" else "f32", io=wl.io, channels=channels)


def _shared_locals(wl, x, plan, channels=1):
    """The checker's expansion rounded to the IO type in the library layout, and the same
    values back in physical units for the checker."""
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    w = x["w"] if channels == 1 else np.concatenate([x["w"], 0.5 * x["w"] ** 2], axis=1)
    L0 = fmm.expand(geo, ker, x["p"], w)
    dt = np.float64 if wl.io == "f64" else np.float32
    Lt = scaled_locals(geo, L0, plan.P_pad).astype(dt)
    return geo, Lt, physical_locals(geo, Lt)


@pytest.mark.parametrize("io,K", [("f64", 4), ("f32", 4), ("f32", 5), ("f64", 2)])
def test_ray_integral_stage(F, io, K):
    wl = _wl(K=K, io=io, R=80)
    x = W.make(wl, seed=21)
    plan = _plan(F, wl, channels=2)
    geo, Lt, Lphys = _shared_locals(wl, x, plan, channels=2)
    o, r = x["o"], x["r"]
    y = plan.ray_integral(_dev(Lt), _dev(o), _dev(r), 0.0, 4.0).cpu().numpy()
    want = rays.ray_integral(geo, Lphys, o, r, 0.0, 4.0)
    assert rel(y, want) < (1e-12 if io == "f64" else 1e-6)
    # ray insertion: gL against the checker's transpose, and the adjoint identity
    gy = np.random.default_rng(3).standard_normal((len(o), 2)).astype(Lt.dtype)
    gL = plan.new_local()
    plan.ray_integral_backward(_dev(o), _dev(r), 0.0, 4.0, _dev(gy), gL)
    gL = gL.cpu().numpy()
    G = rays.ray_integral_T(geo, o, r, 0.0, 4.0, gy, 2)
    assert rel(gL, scaled_cotangent(geo, G, plan.P_pad)) < (1e-12 if io == "f64" else 1e-6)
    assert abs(np.sum(gL * Lt) - np.sum(gy * y)) < 1e-5 * np.abs(gy * y).sum()


def test_ray_integral_end_to_end_and_gradients(F):
    wl = _wl(n=16, K=4, sigma=0.06, N=4000, io="f32", R=128, layer="ray_integral")
    x = W.make(wl, seed=22)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    p = _dev(x["p"]).requires_grad_(True)
    w = _dev(x["w"]).requires_grad_(True)
    y = F.RayIntegral.apply(plan, p, w, _dev(x["o"]), _dev(x["r"]), 0.0, 4.0)
    (y * _dev(x["gy"])).sum().backward()
    L0 = fmm.expand(geo, ker, x["p"], x["w"])
    yr = rays.ray_integral(geo, L0, x["o"], x["r"], 0.0, 4.0)
    assert rel(y.detach().cpu().numpy(), yr) < 1e-5
    G = rays.ray_integral_T(geo, x["o"], x["r"], 0.0, 4.0, x["gy"], 1)
    gw, gp = fmm.p2m_T(geo, fmm.expand_T(geo, ker, G), x["p"], x["w"])
    assert rel(w.grad.cpu().numpy(), gw) < 1e-5
    assert rel(p.grad.cpu().numpy(), gp) < 1e-4


@pytest.mark.parametrize("io,K,n", [("f64", 4, 16), ("f32", 5, 16), ("f64", 5, 32), ("f32", 3, 8)])
def test_ray_root_stage(F, io, K, n):
    wl = _wl(n=n, K=K, io=io, R=200, sigma=0.08 if n <= 16 else 0.05)
    x = W.make(wl, seed=23)
    plan = _plan(F, wl)
    geo, Lt, Lphys = _shared_locals(wl, x, plan)
    o, r = x["o"], x["r"]
    t, nrm, hit, saved = plan.ray_root(_dev(Lt), _dev(o), _dev(r), 0.0, 4.0, 0.5)
    t, nrm, hit, saved = (a.cpu().numpy() for a in (t, nrm, hit, saved))
    ref = rays.ray_root(geo, Lphys, o, r, 0.0, 4.0)
    assert hit.sum() > 0.8 * len(o)
    assert np.array_equal(hit, ref["hit"])
    h = hit == 1
    tol = 1e-10 if io == "f64" else 1e-6
    assert np.max(np.abs(t[h] - ref["t"][h])) < tol
    assert np.all(np.isnan(t[~h]))
    assert rel(nrm[h], ref["normal"][h]) < (1e-9 if io == "f64" else 1e-5)
    assert rel(saved[:, 8], ref["tau"]) < (1e-12 if io == "f64" else 1e-6)
    # backward: IFT insertion against the checker's
    rng = np.random.default_rng(5)
    gt = rng.standard_normal(len(o)).astype(Lt.dtype)
    gn = rng.standard_normal((len(o), 3)).astype(Lt.dtype)
    gL = plan.new_local()
    plan.ray_root_backward(_dev(saved), _dev(hit), _dev(gt), _dev(gn), gL)
    G = rays.ray_root_T(geo, o, r, ref, gt, gn)
    assert rel(gL.cpu().numpy(), scaled_cotangent(geo, G, plan.P_pad)) < (1e-8 if io == "f64" else 1e-4)


@pytest.mark.parametrize("io,K", [("f64", 4), ("f64", 3), ("f32", 4), ("f64", 2), ("f64", 5), ("f32", 5)])
def test_ray_root_closed_forms_match_the_cascade(F, io, K):
    """For K <= 4 the roots, and for K <= 5 the critical points, come from the closed forms
    (Ferrari, Cardano, the quadratic formula; section 5.1).  On the same rays the derivative
    cascade gives the same hits and levels and the same roots to rounding, and the closed-form
    hits match the checker's."""
    wl = _wl(n=16, K=K, io=io, R=256, sigma=0.08)
    x = W.make(wl, seed=31)
    plan = _plan(F, wl)
    geo, Lt, Lphys = _shared_locals(wl, x, plan)
    o, r, L = _dev(x["o"]), _dev(x["r"]), _dev(Lt)
    t1, n1, h1, s1 = (a.cpu().numpy() for a in plan.ray_root(L, o, r, 0.0, 4.0, 0.5))
    F.lib().fc2t2_debug_root_cascade(1)
    try:
        t2, n2, h2, s2 = (a.cpu().numpy() for a in plan.ray_root(L, o, r, 0.0, 4.0, 0.5))
    finally:
        F.lib().fc2t2_debug_root_cascade(0)
    assert np.array_equal(h1, h2) and h1.sum() > 0.8 * len(h1)
    h = h1 == 1
    tol = 1e-10 if io == "f64" else 1e-6
    assert np.max(np.abs(t1[h] - t2[h])) < tol
    assert np.max(np.abs(s1[:, 8] - s2[:, 8]) / np.abs(s2[:, 8])) < (1e-12 if io == "f64" else 1e-6)
    ref = rays.ray_root(geo, Lphys, x["o"], x["r"], 0.0, 4.0)
    assert np.array_equal(h1, ref["hit"])
    assert np.max(np.abs(t1[h] - ref["t"][h])) < tol


def test_ray_root_end_to_end(F):
    """Expansion + ray root + IFT backward through the autograd wrapper against the checker.
    The cotangents are zeroed on the few rays where the two sides disagree on the hit or its
    kind (a rounding-level difference at a threshold), so both backward passes sum over the
    same rays; the gradients must be finite and match."""
    wl = _wl(n=16, K=5, sigma=0.08, N=3000, io="f32", R=256)
    x = W.make(wl, seed=24)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    o, r = _dev(x["o"]), _dev(x["r"])
    L0 = fmm.expand(geo, ker, x["p"], x["w"])
    ref = rays.ray_root(geo, L0, x["o"], x["r"], 0.0, 4.0)
    Lt = plan.expand(_dev(x["p"]), _dev(x["w"]))
    _, _, hit0, saved0 = plan.ray_root(Lt, o, r, 0.0, 4.0, 0.5)
    kind0 = F.Plan.root_kind(saved0).cpu().numpy()
    hit0 = hit0.cpu().numpy()
    same = (hit0 == ref["hit"]) & ((hit0 == 0) | (kind0 == ref["kind"]))
    assert same.sum() >= 0.97 * len(same)
    gt = np.where(same, x["gt"], 0.0).astype(np.float32)
    gn = np.where(same[:, None], x["gn"], 0.0).astype(np.float32)
    p = _dev(x["p"]).requires_grad_(True)
    w = _dev(x["w"]).requires_grad_(True)
    t, nrm, hit = F.RayRoot.apply(plan, p, w, o, r, 0.0, 4.0, 0.5)
    ((t.nan_to_num() * _dev(gt)).sum() + (nrm * _dev(gn)).sum()).backward()
    both = (hit.cpu().numpy() == 1) & (ref["hit"] == 1)
    assert np.median(np.abs(t.detach().cpu().numpy()[both] - ref["t"][both])) < 1e-5
    gw_gpu, gp_gpu = w.grad.cpu().numpy(), p.grad.cpu().numpy()
    assert np.all(np.isfinite(gw_gpu)) and np.all(np.isfinite(gp_gpu))
    G = rays.ray_root_T(geo, x["o"], x["r"], ref, gt, gn)
    gw, gp = fmm.p2m_T(geo, fmm.expand_T(geo, ker, G), x["p"], x["w"])
    assert rel(gw_gpu, gw) < 1e-4
    assert rel(gp_gpu, gp) < 1e-4


def _face_field(plan, geo, dt, rng):
    """Library-layout locals with a jump across the face x = 0: about 0.2 in the cells with x
    index 3, about 1 beyond, zero before; small random higher terms (cell-scaled units)."""
    n = plan.n
    Lt = np.zeros((1, n, n, n, plan.P_pad))
    Lt[0, 3, :, :, :plan.P] = 0.05 * rng.standard_normal((n, n, plan.P))
    Lt[0, 3, :, :, 0] += 0.2
    Lt[0, 4:, :, :, :plan.P] = 0.05 * rng.standard_normal((n - 4, n, n, plan.P))
    Lt[0, 4:, :, :, 0] += 1.0
    Lt = Lt.reshape(1, n ** 3, plan.P_pad).astype(dt)
    return Lt, physical_locals(geo, Lt)


def _grazing_field(plan, geo, dt):
    """f = A + B u_x^3 + C u_y in cell (4, 4, 4) (u = (q - c)/h), A - 0.5 before it along x and
    2A beyond it, so that tau = A on rays along +x through that cell, crossed at the centre with
    zero slope along an untilted ray."""
    n = plan.n
    A, B, C = 0.5, 0.5, 0.3
    idx = fmm.multi_indices(3, plan.K)
    Lt = np.zeros((1, n, n, n, plan.P_pad))
    Lt[0, :4, :, :, 0] = A - 0.5
    Lt[0, 5:, :, :, 0] = 2 * A
    Lt[0, 4, 4, 4, idx.index((0, 0, 0))] = A
    Lt[0, 4, 4, 4, idx.index((3, 0, 0))] = 6 * B
    Lt[0, 4, 4, 4, idx.index((0, 1, 0))] = C
    Lt = Lt.reshape(1, n ** 3, plan.P_pad).astype(dt)
    return Lt, physical_locals(geo, Lt)


def _root_stage_compare(F, plan, geo, Lt, Lphys, o, r, io, tol_t, tol_g):
    t, nrm, hit, saved = plan.ray_root(_dev(Lt), _dev(o), _dev(r), 0.0, 4.0, 0.5)
    kind = F.Plan.root_kind(saved).cpu().numpy()
    t, nrm, hit, saved = (a.cpu().numpy() for a in (t, nrm, hit, saved))
    ref = rays.ray_root(geo, Lphys, o, r, 0.0, 4.0)
    assert np.array_equal(hit, ref["hit"])
    h = hit == 1
    assert np.array_equal(kind[h], ref["kind"][h])
    assert np.max(np.abs(t[h] - ref["t"][h])) < tol_t
    assert rel(nrm[h], ref["normal"][h]) < tol_g
    rng = np.random.default_rng(7)
    dt = Lt.dtype
    gt = rng.standard_normal(len(o)).astype(dt)
    gn = rng.standard_normal((len(o), 3)).astype(dt)
    gL = plan.new_local()
    plan.ray_root_backward(_dev(saved), _dev(hit), _dev(gt), _dev(gn), gL)
    gL = gL.cpu().numpy()
    assert np.all(np.isfinite(gL))
    G = rays.ray_root_T(geo, o, r, ref, gt, gn)
    assert rel(gL, scaled_cotangent(geo, G, plan.P_pad)) < tol_g
    return kind, ref


@pytest.mark.parametrize("io", ["f64", "f32"])
def test_ray_root_face_crossings_stage(F, io):
    """Every ray crosses the level by the jump at the face x = 0: the GPU reports face hits in
    the earlier cell, and its backward inserts only the surface-gradient term, as the checker
    (whose rule is pinned by central differences)."""
    wl = _wl(n=8, K=3, io=io, R=64)
    plan = _plan(F, wl)
    geo = oracle_geometry(wl)
    rng = np.random.default_rng(41)
    dt = np.float64 if io == "f64" else np.float32
    Lt, Lphys = _face_field(plan, geo, dt, rng)
    R = 64
    o = np.stack([np.full(R, -2.0), rng.uniform(-0.8, 0.8, R), rng.uniform(-0.8, 0.8, R)], axis=1)
    r = np.stack([np.ones(R), rng.uniform(-0.15, 0.15, R), rng.uniform(-0.15, 0.15, R)], axis=1)
    r /= np.linalg.norm(r, axis=1, keepdims=True)
    o, r = o.astype(dt), r.astype(dt)
    kind, ref = _root_stage_compare(F, plan, geo, Lt, Lphys, o, r, io, 1e-12 if io == "f64" else 1e-6,
                                    1e-10 if io == "f64" else 1e-5)
    assert ref["hit"].all() and (kind == F.ROOT_FACE).all()
    assert plan.grazing_roots(reset=True) == 0


@pytest.mark.parametrize("io", ["f64", "f32"])
def test_ray_root_grazing_stage(F, io):
    """Rays along +x through an inflection crossing: untilted and 1e-6-tilted rays are grazing
    (masked: dipole term only, counted on the device), 1e-2-tilted rays are smooth roots whose
    backward inserts the implicit-function term."""
    wl = _wl(n=8, K=3, io=io, R=6)
    plan = _plan(F, wl)
    geo = oracle_geometry(wl)
    dt = np.float64 if io == "f64" else np.float32
    Lt, Lphys = _grazing_field(plan, geo, dt)
    tilt = np.array([0.0, 1e-6, -1e-6, 1e-2, -1e-2, 2e-2])
    # every ray passes through the cell centre (0.125, 0.125, 0.125), where the level is crossed
    o = np.stack([np.full(6, -2.0), 0.125 - 2.125 * tilt, np.full(6, 0.125)], axis=1)
    r = np.stack([np.ones(6), tilt, np.zeros(6)], axis=1)
    r /= np.linalg.norm(r, axis=1, keepdims=True)
    o, r = o.astype(dt), r.astype(dt)
    plan.grazing_roots(reset=True)
    # the root of the untilted ray is a triple one: both sides locate it to about the cube root
    # of the rounding, so positions and the dipole term agree to that level
    kind, ref = _root_stage_compare(F, plan, geo, Lt, Lphys, o, r, io, 1e-4, 1e-4)
    assert kind.tolist() == [F.ROOT_GRAZING] * 3 + [F.ROOT_SMOOTH] * 3
    assert plan.grazing_roots(reset=True) == 3


def test_ray_edge_cases(F):
    wl = _wl(n=8, K=3, io="f64", R=4)
    plan = _plan(F, wl)
    Lt = np.zeros(plan.local_shape())
    Lt[0, :, 0] = 1.0
    # rays that miss the domain, a ray along a grid line, a ray starting inside, and R = 0
    o = np.array([[3.0, 3.0, 3.0], [-2.0, 0.0, 0.0], [0.1, 0.2, 0.3], [0.0, 5.0, 0.0]])
    r = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 1.0, 0.0]])
    y = plan.ray_integral(_dev(Lt), _dev(o), _dev(r), 0.0, 4.0).cpu().numpy()[:, 0]
    assert y[0] == 0.0 and y[3] == 0.0
    assert abs(y[1] - 2.0) < 1e-12            # f = 1 across the whole box, length 2
    assert abs(y[2] - 0.7) < 1e-12            # from z = 0.3 to the face z = 1
    y0 = plan.ray_integral(_dev(Lt), _dev(o[:0]), _dev(r[:0]), 0.0, 4.0)
    assert y0.shape == (0, 1)
    t, nrm, hit, saved = plan.ray_root(_dev(Lt), _dev(o), _dev(r), 0.0, 4.0, 0.5)
    assert hit.cpu().numpy().tolist() == [0, 0, 0, 0]   # constant field: f >= tau at entry or no samples

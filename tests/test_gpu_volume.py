"""GPU parity of the volumetric rendering layer (section 6.1.2 forward, section 6.2.2
backward) against the FP64 checker, through the C-ABI.

Stage tests feed both sides the same four-channel expansion (density, R, G, B), rounded to the
IO type first; the end-to-end test runs the GPU's expansion, rendering and backward through
the autograd wrapper against the checker's whole chain.  Rays whose stop decision sits within
rounding of the threshold (an exit depth within a small margin of 4.5, as the checker reports
it) are left out of the comparisons: the two sides may then stop in different cells, both
correctly."""
import numpy as np
import pytest

from oracle import fmm, volume
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


def _wl(n=8, K=4, io="f64", N=2000, sigma=0.08, R=40):
    return W.Workload("v", 3, n, -1.0, 1.0, K, "gaussian", sigma, N, 0, R, io, "volume", "shell")


def _plan(F, wl):
    return F.Plan(3, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K,
                  m2l="f64" if wl.io == "f64" else "f32", io=wl.io, channels=4)


def _field(rng, geo, P_pad, dt, dens):
    """Random four-channel locals with a positive density (physical units, then the library's
    layout rounded to the IO type and back)."""
    L0 = 0.3 * rng.standard_normal((4,) + (geo.n,) * 3 + (geo.P,))
    L0[0, ..., 0] = dens + 0.2 * rng.random((geo.n,) * 3)
    Lt = scaled_locals(geo, L0, P_pad).astype(dt)
    return Lt, physical_locals(geo, Lt)


@pytest.mark.parametrize("io,K,dens", [("f64", 4, 0.8), ("f64", 4, 2.5), ("f32", 4, 1.8), ("f64", 5, 1.8),
                                       ("f32", 2, 1.0), ("f64", 3, 3.0)])
def test_volume_stage(F, io, K, dens):
    wl = _wl(K=K, io=io)
    geo = oracle_geometry(wl)
    plan = _plan(F, wl)
    rng = np.random.default_rng(60 + K)
    dt = np.float64 if io == "f64" else np.float32
    Lt, L0 = _field(rng, geo, plan.P_pad, dt, dens)
    o, r = rays_toward_origin(rng, wl.R, jitter=0.4)
    o, r = o.astype(dt), r.astype(dt)
    bg = np.array([0.25, -0.5, 1.0])
    ref = volume.render(geo, L0, o, r, 0.0, 4.0, bg)
    ok = ref["margin"] > (1e-6 if io == "f64" else 1e-4)
    assert ok.sum() >= 0.9 * len(ok)
    y, tr = plan.ray_volume(_dev(Lt), _dev(o), _dev(r), 0.0, 4.0, bg, with_trans=True)
    y, tr = y.cpu().numpy(), tr.cpu().numpy()
    tol = 1e-9 if io == "f64" else 2e-6
    assert rel(y[ok], ref["y"][ok]) < tol
    assert np.max(np.abs(tr[ok] - ref["T_end"][ok])) < tol
    # the media: thin (every ray sees the background), mixed, or dense (every ray stops)
    frac = ref["stopped"].mean()
    assert {0.8: frac == 0, 1.0: frac == 0, 1.8: 0 < frac < 1, 2.5: frac == 1, 3.0: frac == 1}[dens]
    # backward on the clear rays only
    gy = np.where(ok[:, None], rng.standard_normal((wl.R, 3)), 0.0).astype(dt)
    gL = plan.new_local()
    plan.ray_volume_backward(_dev(Lt), _dev(o), _dev(r), 0.0, 4.0, _dev(gy), gL, bg)
    gL = gL.cpu().numpy()
    G = volume.render_T(geo, L0, o, r, 0.0, 4.0, ref, gy, bg)
    want = scaled_cotangent(geo, G, plan.P_pad)
    assert np.all(np.isfinite(gL))
    assert rel(gL, want) < (1e-9 if io == "f64" else 5e-6)
    for ch in range(4):
        assert rel(gL[ch], want[ch]) < (1e-9 if io == "f64" else 5e-6), ch


def test_volume_backward_is_the_derivative_of_the_gpu_forward(F):
    """<gL, dL> against central differences of the GPU's own forward (FP64) along a random
    direction: the backward is the derivative of what the forward computes."""
    wl = _wl(K=4, io="f64")
    geo = oracle_geometry(wl)
    plan = _plan(F, wl)
    rng = np.random.default_rng(70)
    Lt, L0 = _field(rng, geo, plan.P_pad, np.float64, 1.0)
    o, r = rays_toward_origin(rng, wl.R, jitter=0.4)
    bg = np.array([0.3, 0.6, 0.9])
    ok = volume.render(geo, L0, o, r, 0.0, 4.0, bg)["margin"] > 1e-4
    gy = np.where(ok[:, None], rng.standard_normal((wl.R, 3)), 0.0)
    dL = rng.standard_normal(Lt.shape)
    dL[:, :, plan.P:] = 0.0
    gL = plan.new_local()
    plan.ray_volume_backward(_dev(Lt), _dev(o), _dev(r), 0.0, 4.0, _dev(gy), gL, bg)
    eps = 1e-6
    loss = lambda L: float(np.sum(gy * plan.ray_volume(_dev(L), _dev(o), _dev(r), 0.0, 4.0, bg).cpu().numpy()))
    fd = (loss(Lt + eps * dL) - loss(Lt - eps * dL)) / (2 * eps)
    an = float(np.sum(gL.cpu().numpy() * dL))
    assert abs(fd - an) < 1e-6 * max(1.0, abs(an))


def test_volume_edge_cases(F):
    """No rays; a ray that misses the domain and one through a zero field both see the
    background through the transmittance mexp(0) (1 to within the fit's error); a plan with
    the wrong channel count is refused."""
    wl = _wl(K=3, io="f64")
    plan = _plan(F, wl)
    Lt = plan.new_local()
    e = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    assert plan.ray_volume(Lt, e, e, 0.0, 4.0).shape == (0, 3)
    gL = plan.new_local()
    plan.ray_volume_backward(Lt, e, e, 0.0, 4.0, e, gL)
    assert float(gL.abs().sum()) == 0.0
    o = np.array([[5.0, 5.0, 5.0], [0.0, 0.0, -3.0]])
    r = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    bg = (0.1, 0.2, 0.3)
    y, tr = plan.ray_volume(Lt, _dev(o), _dev(r), 0.0, 8.0, bg, with_trans=True)
    m = volume.mexp_coefficients()
    assert np.allclose(tr.cpu().numpy(), [m[0], m[0]], rtol=1e-12)
    assert np.allclose(y.cpu().numpy(), np.outer([m[0], m[0]], bg), rtol=1e-12)
    one = F.Plan(3, 8, -1.0, 1.0, "gaussian", 0.08, 3, m2l="f64", io="f64", channels=1)
    with pytest.raises(F.FC2T2Error):
        one.ray_volume(one.new_local(), _dev(o), _dev(r), 0.0, 4.0)


def test_volume_end_to_end_and_gradients(F):
    """Expansion of four-channel sources (non-negative density weights) + rendering + backward
    through the autograd wrapper against the checker's chain."""
    wl = _wl(n=16, K=4, io="f32", N=3000, sigma=0.06, R=64)
    x = W.make(wl, seed=25)
    w = x["w"]
    assert w.shape == (wl.N, 4) and np.all(w[:, 0] >= 0)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    bg = np.array([0.2, 0.4, 0.6])
    L0 = fmm.expand(geo, ker, x["p"].astype(np.float64), w.astype(np.float64))
    ref = volume.render(geo, L0, x["o"], x["r"], 0.0, 4.0, bg)
    ok = ref["margin"] > 1e-3
    assert ok.sum() >= 0.9 * len(ok)
    assert ref["stopped"].any() and (~ref["stopped"]).any()
    gy = np.where(ok[:, None], np.random.default_rng(8).standard_normal((wl.R, 3)), 0.0).astype(np.float32)
    p = _dev(x["p"]).requires_grad_(True)
    wd = _dev(w).requires_grad_(True)
    y = F.RayVolume.apply(plan, p, wd, _dev(x["o"]), _dev(x["r"]), 0.0, 4.0, bg)
    (y * _dev(gy)).sum().backward()
    assert rel(y.detach().cpu().numpy()[ok], ref["y"][ok]) < 1e-5
    G = volume.render_T(geo, L0, x["o"], x["r"], 0.0, 4.0, ref, gy, bg)
    gw, gp = fmm.p2m_T(geo, fmm.expand_T(geo, ker, G), x["p"], w)
    assert rel(wd.grad.cpu().numpy(), gw) < 1e-4
    assert rel(p.grad.cpu().numpy(), gp) < 1e-4


@pytest.mark.parametrize("n,dens", [(8, 2.5), (8, 4.0), (16, 6.0)])
def test_volume_lane_cuts_on_cell_faces(F, n, dens):
    """Rays along the axes across the whole box: each ray's parameter range is cut into equal
    sub-ranges for the lanes that walk it, and with n a multiple of the lane count the cuts fall
    on cell faces (up to rounding).  The stop decision must still be taken at every cell exit,
    forward and backward."""
    wl = _wl(n=n, K=4, io="f64", R=48)
    geo = oracle_geometry(wl)
    plan = _plan(F, wl)
    rng = np.random.default_rng(90 + n)
    Lt, L0 = _field(rng, geo, plan.P_pad, np.float64, dens)
    o, r = [], []
    for axis in range(3):
        for sign in (1.0, -1.0):
            for _ in range(wl.R // 6):
                d = np.zeros(3)
                d[axis] = sign
                p = rng.uniform(-0.95, 0.95, 3)
                p[axis] = -3.0 * sign
                o.append(p)
                r.append(d)
    o, r = np.array(o), np.array(r)
    bg = np.array([0.3, 0.6, 0.9])
    ref = volume.render(geo, L0, o, r, 0.0, 10.0, bg)
    ok = ref["margin"] > 1e-6
    assert ok.sum() >= 0.9 * len(ok) and ref["stopped"][ok].any()
    y = plan.ray_volume(_dev(Lt), _dev(o), _dev(r), 0.0, 10.0, bg).cpu().numpy()
    assert np.max(np.abs(y[ok] - ref["y"][ok])) < 1e-10
    gy = np.where(ok[:, None], rng.standard_normal((len(o), 3)), 0.0)
    gL = plan.new_local()
    plan.ray_volume_backward(_dev(Lt), _dev(o), _dev(r), 0.0, 10.0, _dev(gy), gL, bg)
    G = volume.render_T(geo, L0, o, r, 0.0, 10.0, ref, gy, bg)
    assert rel(gL.cpu().numpy(), scaled_cotangent(geo, G, plan.P_pad)) < 1e-9

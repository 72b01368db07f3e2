"""Full-size parity of every throughput workload, in the launch configuration bench.py times
(FP16x3 M2L, FP32 IO), against the FP64 checker on sampled outputs:

* explicit layers (256^2 and 64^3 with 10^7 queries): y and q_bar at sampled queries (the
  checker's locals computed cell by cell from the full moment pyramid), w_bar and p_bar at
  sampled sources (the checker's moment cotangents computed cell by cell from the full pyramid
  of local cotangents, itself the transpose of L2P over every query);
* ray layers (128^3): y or (t*, grad f) on sampled rays, and w_bar at sampled sources for the
  cotangents of a subsample of rays (ray insertion, or the implicit-function insertion, then
  the whole expansion backward at full size);
* volumetric rendering (64^3, 2^23 four-channel sources, 10^5 rays): the colour of sampled
  rays, and w_bar at sampled sources for the colour cotangents of those rays.

Tolerances are the error contract: 1e-5 on values and w_bar, 1e-4 on the differentiated p_bar
and q_bar."""
import numpy as np
import pytest

from oracle import fmm, rays, volume
from paper_2111_00110_amd import workloads as W

from helpers import oracle_geometry, oracle_kernel, rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")

BENCH_M2L = "f16x3"


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_00110_amd import fc2t2
    return fc2t2


def _plan(F, wl):
    return F.Plan(wl.dim, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K, m2l=BENCH_M2L, io=wl.io,
                  channels=4 if wl.layer == "volume" else 1)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sampled_source_grads(geo, ker, G_L0, p, w, idx):
    """(w_bar, p_bar) of the sources idx from the full local cotangent G_L0."""
    GLs = fmm.local_cotangent_pyramid(geo, G_L0)
    cells = geo.cell_index(p[idx])
    rows = fmm.moment_cotangents_at_cells(geo, ker, GLs, cells)
    return fmm.p2m_T_rows(geo, rows, p[idx], w[idx])


@pytest.mark.parametrize("name", ["explicit2d", "explicit3d_imq"])
def test_explicit_full_size_forward_and_backward(F, name):
    wl = W.workload(name)
    x = W.make(wl)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    p, w, q, gy = (_dev(x[k]) for k in ("p", "w", "q", "gy"))
    Lt = plan.expand(p, w)
    y, _, _ = plan.eval(Lt, q)
    gL = plan.new_local()
    gq = torch.empty_like(q)
    plan.eval_backward(Lt, q, gy, gL, gq, accumulate=False)
    gp, gw = torch.empty_like(p), torch.empty_like(w)
    plan.expand_backward(gL, p, w, gp, gw, accumulate=False)
    y, gq, gp, gw = (t.cpu().numpy() for t in (y, gq, gp, gw))
    # queries: y and q_bar
    iq = W.subsample(5, 192, wl.M)
    qs = x["q"][iq]
    cells = geo.cell_index(qs)
    Lc = fmm.locals_at_cells(geo, ker, fmm.moments_all_levels(geo, x["p"], x["w"]), cells)
    dvec = qs.astype(np.float64) - geo.centre(0, cells)
    want_y = np.einsum("csp,sp->sc", Lc, fmm.monomials(dvec, geo.idx))
    want_gq = np.einsum("sc,csp,spj->sj", x["gy"][iq].astype(np.float64), Lc, fmm.monomial_grads(dvec, geo.idx))
    assert rel(y[iq], want_y) < 1e-5
    assert rel(gq[iq], want_gq) < 1e-4
    # sources: w_bar and p_bar
    isrc = W.subsample(6, 192, wl.N)
    G_L0 = fmm.l2p_T(geo, x["q"], x["gy"])
    want_gw, want_gp = _sampled_source_grads(geo, ker, G_L0, x["p"], x["w"], isrc)
    assert rel(gw[isrc], want_gw) < 1e-5
    assert rel(gp[isrc], want_gp) < 1e-4


def _sparse_locals(geo, ker, Ms, cells):
    """Physical locals at the given cells inside an otherwise empty full-size array."""
    cells = np.unique(np.asarray(cells, dtype=np.int64).reshape(-1, geo.dim), axis=0)
    C = Ms[0].shape[0]
    L = np.zeros((C,) + (geo.n,) * geo.dim + (geo.P,))
    vals = fmm.locals_at_cells(geo, ker, Ms, cells)
    for c in range(C):
        L[(c,) + tuple(cells[:, j] for j in range(geo.dim))] = vals[c]
    return L


def _ray_cells(geo, o, r, t0, t1):
    out = []
    for i in range(len(o)):
        out += [c for c, _, _ in rays.segments(geo, o[i], r[i], t0, t1)]
    return np.array(out)


def test_ray_integral3d_full_size(F):
    wl = W.workload("ray_integral3d")
    x = W.make(wl)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    p, w, o, r = (_dev(x[k]) for k in ("p", "w", "o", "r"))
    Lt = plan.expand(p, w)
    y = plan.ray_integral(Lt, o, r, wl.t0, wl.t1).cpu().numpy()
    idx = W.subsample(8, 6, wl.R)
    os_, rs, gys = x["o"][idx], x["r"][idx], x["gy"][idx]
    Ms = fmm.moments_all_levels(geo, x["p"], x["w"])
    L = _sparse_locals(geo, ker, Ms, _ray_cells(geo, os_, rs, wl.t0, wl.t1))
    assert rel(y[idx], rays.ray_integral(geo, L, os_, rs, wl.t0, wl.t1)) < 1e-5
    # backward of the sampled rays' integrals through the whole expansion at full size
    gL = plan.new_local()
    plan.ray_integral_backward(_dev(os_), _dev(rs), wl.t0, wl.t1, _dev(gys), gL)
    gw = torch.empty_like(w)
    plan.expand_backward(gL, p, w, None, gw, accumulate=False)
    gw = gw.cpu().numpy()
    G_L0 = rays.ray_integral_T(geo, os_, rs, wl.t0, wl.t1, gys, 1)
    isrc = W.subsample(10, 160, wl.N)
    want_gw, _ = _sampled_source_grads(geo, ker, G_L0, x["p"], x["w"], isrc)
    assert rel(gw[isrc], want_gw) < 1e-5


def test_ray_root3d_full_size(F):
    wl = W.workload("ray_root3d")
    x = W.make(wl)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    p, w, o, r = (_dev(x[k]) for k in ("p", "w", "o", "r"))
    Lt = plan.expand(p, w)
    t, nrm, hit, _ = plan.ray_root(Lt, o, r, wl.t0, wl.t1, 0.5)
    t, nrm, hit = t.cpu().numpy(), nrm.cpu().numpy(), hit.cpu().numpy()
    assert hit.mean() > 0.9
    idx = W.subsample(9, 6, wl.R)
    os_, rs = x["o"][idx], x["r"][idx]
    Ms = fmm.moments_all_levels(geo, x["p"], x["w"])
    L = _sparse_locals(geo, ker, Ms, _ray_cells(geo, os_, rs, wl.t0, wl.t1))
    ref = rays.ray_root(geo, L, os_, rs, wl.t0, wl.t1)
    assert np.array_equal(hit[idx], ref["hit"])
    h = ref["hit"] == 1
    assert np.max(np.abs(t[idx][h] - ref["t"][h])) < 1e-5
    assert rel(nrm[idx][h], ref["normal"][h]) < 1e-4
    # implicit-function backward of the sampled rays through the whole expansion at full size
    gts, gns = x["gt"][idx], x["gn"][idx]
    _, _, hit_s, saved_s = plan.ray_root(Lt, _dev(os_), _dev(rs), wl.t0, wl.t1, 0.5)
    gL = plan.new_local()
    plan.ray_root_backward(saved_s, hit_s, _dev(gts), _dev(gns), gL)
    gw = torch.empty_like(w)
    plan.expand_backward(gL, p, w, None, gw, accumulate=False)
    gw = gw.cpu().numpy()
    G_L0 = rays.ray_root_T(geo, os_, rs, ref, gts, gns)
    isrc = W.subsample(11, 160, wl.N)
    want_gw, _ = _sampled_source_grads(geo, ker, G_L0, x["p"], x["w"], isrc)
    assert rel(gw[isrc], want_gw) < 1e-4


def test_volume3d_full_size(F):
    wl = W.workload("volume3d")
    x = W.make(wl)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    p, w, o, r = (_dev(x[k]) for k in ("p", "w", "o", "r"))
    bg = tuple(float(v) for v in x["bg"])
    Lt = plan.expand(p, w)
    y, tr = plan.ray_volume(Lt, o, r, wl.t0, wl.t1, bg, with_trans=True)
    y, tr = y.cpu().numpy(), tr.cpu().numpy()
    # the medium: some rays end inside it, others reach the background
    assert 0.05 < float(np.mean(tr == 0)) < 0.95
    idx = W.subsample(12, 8, wl.R)
    os_, rs = x["o"][idx], x["r"][idx]
    Ms = fmm.moments_all_levels(geo, x["p"], x["w"])
    L = _sparse_locals(geo, ker, Ms, _ray_cells(geo, os_, rs, wl.t0, wl.t1))
    ref = volume.render(geo, L, os_, rs, wl.t0, wl.t1, np.array(bg))
    ok = ref["margin"] > 1e-3          # stop decisions clear of rounding
    assert ok.sum() >= 6
    assert rel(y[idx][ok], ref["y"][ok]) < 1e-5
    # backward of the sampled rays' colours through the whole expansion at full size
    gys = np.where(ok[:, None], x["gy"][idx], 0.0).astype(np.float32)
    gL = plan.new_local()
    plan.ray_volume_backward(Lt, _dev(os_), _dev(rs), wl.t0, wl.t1, _dev(gys), gL, bg)
    gw = torch.empty_like(w)
    plan.expand_backward(gL, p, w, None, gw, accumulate=False)
    gw = gw.cpu().numpy()
    G_L0 = volume.render_T(geo, L, os_, rs, wl.t0, wl.t1, ref, gys, np.array(bg))
    isrc = W.subsample(13, 160, wl.N)
    want_gw, _ = _sampled_source_grads(geo, ker, G_L0, x["p"], x["w"], isrc)
    assert rel(gw[isrc], want_gw) < 1e-5

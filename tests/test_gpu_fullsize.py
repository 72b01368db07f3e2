"""Full-size parity of the 3-D workloads, in the launch configuration bench.py times (BF16x3
M2L, FP32 IO): sampled outputs against the FP64 checker, whose locals are computed cell by
cell from the full moment pyramid only at the cells the samples need."""
import numpy as np
import pytest

from oracle import fmm, rays
from paper_2111_00110_amd import workloads as W

from helpers import oracle_geometry, oracle_kernel, rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_00110_amd import fc2t2
    return fc2t2


def _plan(F, wl):
    return F.Plan(wl.dim, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K, m2l="bf16x3", io=wl.io)


def _sparse_locals(geo, ker, Ms, cells):
    """Physical locals at the given cells inside an otherwise empty full-size array."""
    cells = np.unique(np.asarray(cells, dtype=np.int64).reshape(-1, geo.dim), axis=0)
    L = np.zeros((1,) + (geo.n,) * geo.dim + (geo.P,))
    vals = fmm.locals_at_cells(geo, ker, Ms, cells)
    L[(0,) + tuple(cells[:, j] for j in range(geo.dim))] = vals[0]
    return L


def test_explicit3d_imq_full_size(F):
    wl = W.workload("explicit3d_imq")
    x = W.make(wl)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    p, w, q = (torch.from_numpy(x[k]).cuda() for k in ("p", "w", "q"))
    Lt = plan.expand(p, w)
    y, g, _ = plan.eval(Lt, q, grad=True)
    idx = W.subsample(7, 192, wl.M)
    y, g = y.cpu().numpy()[idx], g.cpu().numpy()[idx]
    qs = x["q"][idx]
    cells = geo.cell_index(qs)
    Ms = fmm.moments_all_levels(geo, x["p"], x["w"])
    Lc = fmm.locals_at_cells(geo, ker, Ms, cells)
    dvec = qs.astype(np.float64) - geo.centre(0, cells)
    want_y = np.einsum("csp,sp->sc", Lc, fmm.monomials(dvec, geo.idx))
    want_g = np.einsum("csp,spj->scj", Lc, fmm.monomial_grads(dvec, geo.idx))
    assert rel(y, want_y) < 3e-5
    assert rel(g, want_g) < 5e-5


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
    p, w, o, r = (torch.from_numpy(x[k]).cuda() for k in ("p", "w", "o", "r"))
    Lt = plan.expand(p, w)
    y = plan.ray_integral(Lt, o, r, wl.t0, wl.t1).cpu().numpy()
    idx = W.subsample(8, 4, wl.R)
    os_, rs = x["o"][idx], x["r"][idx]
    Ms = fmm.moments_all_levels(geo, x["p"], x["w"])
    L = _sparse_locals(geo, ker, Ms, _ray_cells(geo, os_, rs, wl.t0, wl.t1))
    want = rays.ray_integral(geo, L, os_, rs, wl.t0, wl.t1)
    assert rel(y[idx], want) < 3e-5


def test_ray_root3d_full_size(F):
    wl = W.workload("ray_root3d")
    x = W.make(wl)
    geo, ker = oracle_geometry(wl), oracle_kernel(wl)
    plan = _plan(F, wl)
    p, w, o, r = (torch.from_numpy(x[k]).cuda() for k in ("p", "w", "o", "r"))
    Lt = plan.expand(p, w)
    t, nrm, hit, _ = plan.ray_root(Lt, o, r, wl.t0, wl.t1, 0.5)
    t, nrm, hit = t.cpu().numpy(), nrm.cpu().numpy(), hit.cpu().numpy()
    assert hit.mean() > 0.9
    idx = W.subsample(9, 4, wl.R)
    os_, rs = x["o"][idx], x["r"][idx]
    Ms = fmm.moments_all_levels(geo, x["p"], x["w"])
    L = _sparse_locals(geo, ker, Ms, _ray_cells(geo, os_, rs, wl.t0, wl.t1))
    ref = rays.ray_root(geo, L, os_, rs, wl.t0, wl.t1)
    assert np.array_equal(hit[idx], ref["hit"])
    h = ref["hit"] == 1
    assert np.max(np.abs(t[idx][h] - ref["t"][h])) < 1e-4
    assert rel(nrm[idx][h], ref["normal"][h]) < 1e-3

"""FP64 torch.autograd.gradcheck of the autograd wrappers: the hand-written backward passes
(section 4.1 for the explicit layer, section 6.2.1 for the line integral, section 5.2 for the
ray root) against central differences of the GPU forward itself, in FP64 end to end.

The ray-root check uses given per-ray levels (the level is held fixed in the backward, as the
paper's bias is) on rays whose root is a smooth crossing inside a cell."""
import numpy as np
import pytest

from paper_2111_00110_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_00110_amd import fc2t2
    return fc2t2


def _dev(a, grad=False):
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    return t.requires_grad_(grad)


def _shell(rng, N):
    u = rng.standard_normal((N, 3))
    return 0.5 * u / np.linalg.norm(u, axis=1, keepdims=True) + 0.01 * rng.standard_normal((N, 3))


@pytest.mark.parametrize("dim,kernel,param,K", [(2, "gaussian", 0.1, 4), (3, "imq", 0.3, 3)])
def test_explicit_gradcheck(F, dim, kernel, param, K):
    rng = np.random.default_rng(60 + dim)
    lo, hi = (0.0, 1.0) if dim == 2 else (-1.0, 1.0)
    plan = F.Plan(dim, 8, lo, hi, kernel, param, K, m2l="f64", io="f64")
    p = _dev(rng.uniform(lo + 0.05, hi - 0.05, (24, dim)), True)
    w = _dev(rng.standard_normal((24, 1)), True)
    q = _dev(rng.uniform(lo + 0.05, hi - 0.05, (16, dim)), True)
    assert torch.autograd.gradcheck(lambda a, b, c: F.Explicit.apply(plan, a, b, c), (p, w, q),
                                    eps=1e-6, atol=1e-7, rtol=1e-5)


def test_ray_integral_gradcheck(F):
    rng = np.random.default_rng(62)
    plan = F.Plan(3, 8, -1.0, 1.0, "gaussian", 0.2, 3, m2l="f64", io="f64")
    p = _dev(_shell(rng, 20), True)
    w = _dev(rng.uniform(0.5, 1.5, (20, 1)), True)
    x = W.make(W.Workload("g", 3, 8, -1.0, 1.0, 3, "gaussian", 0.2, 4, 0, 6, "f64", "ray_integral", "shell"),
               seed=63)
    o, r = _dev(x["o"]), _dev(x["r"])
    assert torch.autograd.gradcheck(lambda a, b: F.RayIntegral.apply(plan, a, b, o, r, 0.0, 4.0), (p, w),
                                    eps=1e-6, atol=1e-7, rtol=1e-5)


def test_ray_root_gradcheck_at_given_levels(F):
    rng = np.random.default_rng(64)
    plan = F.Plan(3, 16, -1.0, 1.0, "gaussian", 0.15, 4, m2l="f64", io="f64")
    pn = _shell(rng, 60)
    wn = rng.uniform(0.5, 1.5, (60, 1))
    x = W.make(W.Workload("g", 3, 16, -1.0, 1.0, 4, "gaussian", 0.15, 4, 0, 12, "f64", "ray_root", "shell"),
               seed=65)
    o, r = _dev(x["o"]), _dev(x["r"])
    Lt = plan.expand(_dev(pn), _dev(wn))
    t, _, hit, saved = plan.ray_root(Lt, o, r, 0.0, 4.0, 0.5)
    kind = F.Plan.root_kind(saved)
    # smooth crossings away from cell faces (a root within eps of a face could change cells)
    q = (o + t[:, None] * r).detach().cpu().numpy()
    u = (q + 1.0) / plan.h
    far = np.all(np.abs(u - np.round(u)) > 1e-3, axis=1)
    keep = np.nonzero((hit.cpu().numpy() == 1) & (kind.cpu().numpy() == F.ROOT_SMOOTH) & far)[0][:6]
    assert len(keep) >= 4
    keep_t = torch.from_numpy(keep).cuda()
    o, r, tau = o[keep_t].contiguous(), r[keep_t].contiguous(), saved[keep_t, 8].contiguous()

    def f(a, b):
        tt, nrm, _ = F.RayRoot.apply(plan, a, b, o, r, 0.0, 4.0, 0.5, tau)
        return tt, nrm
    assert torch.autograd.gradcheck(f, (_dev(pn, True), _dev(wn, True)), eps=1e-6, atol=1e-6, rtol=1e-4)

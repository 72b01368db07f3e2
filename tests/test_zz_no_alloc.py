"""The no-allocation ray-root backward (fixed device scratch, for callers that cannot allocate)
against the workspace entry point it varies, through the C-ABI: two calls in a row, the second
with fewer rays, bitwise equal (same kernels, same summation order); sizes beyond the fixed
scratch are rejected on the host."""
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


@pytest.mark.parametrize("io", ["f32", "f64"])
def test_noalloc_ray_root_backward_matches_workspace_call(F, io):
    wl = W.Workload("na", 3, 32, -1.0, 1.0, 4, "gaussian", 0.05, 20000, 0, 6000, io, "ray_root", "shell")
    x = W.make(wl, seed=71)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    plan = F.Plan(3, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K, m2l="f64" if io == "f64" else "f32", io=io)
    Lt = plan.expand(dev(x["p"]), dev(x["w"]))
    t, nrm, hit, saved = plan.ray_root(Lt, dev(x["o"]), dev(x["r"]), 0.0, 4.0, 0.5)
    assert int(hit.sum()) > 0.5 * wl.R
    gt, gn = dev(x["gt"]), dev(x["gn"])
    for R in (wl.R, 1500):
        ref = plan.new_local()
        plan.ray_root_backward(saved[:R].contiguous(), hit[:R].contiguous(), gt[:R].contiguous(),
                               gn[:R].contiguous(), ref)
        got = plan.new_local().fill_(0.0)
        plan.ray_root_backward_noalloc(saved[:R].contiguous(), hit[:R].contiguous(), gt[:R].contiguous(),
                                       gn[:R].contiguous(), got)
        torch.cuda.synchronize()
        assert float(ref.abs().max()) > 0.0
        assert torch.equal(got, ref), R


def test_noalloc_rejects_sizes_beyond_its_scratch(F):
    plan = F.Plan(3, 128, -1.0, 1.0, "gaussian", 0.02, 4, m2l="f32", io="f32")
    R = 1 << 21
    assert plan.workspace("ray_root_backward", R).numel() > F.lib().fc2t2_workspace_size(plan.handle, 4, 131072)
    saved = torch.zeros((R, F.ROOT_SAVED), dtype=torch.float32, device="cuda")
    hit = torch.zeros(R, dtype=torch.int32, device="cuda")
    gt = torch.zeros(R, dtype=torch.float32, device="cuda")
    gL = plan.new_local()
    with pytest.raises(F.FC2T2Error, match="no-allocation"):
        plan.ray_root_backward_noalloc(saved, hit, gt, None, gL)
    # the largest documented size fits
    assert F.lib().fc2t2_workspace_size(plan.handle, 4, 131072) <= 16 << 20

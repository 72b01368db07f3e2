"""The sort's failure path, forced from the host: with the test aid enabled one tile of every
one-sweep pass withholds its counts and the look-back's bounded wait gives up after a few polls
(every kernel still ends).  The failure must be counted on the plan, reported in debug mode, and
the stages after the sort must not read the unsorted records; normal sorting afterwards gives
the same results as a fresh plan."""
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


def test_failed_sort_is_counted_and_contained(F, monkeypatch):
    wl = W.workload("explicit2d", N=1 << 15, M=1 << 14, n=64)
    x = W.make(wl, seed=16)
    d = {k: torch.from_numpy(v).cuda() for k, v in x.items()}
    mk = lambda: F.Plan(2, wl.n, wl.lo, wl.hi, wl.kernel, wl.param, wl.K, m2l="f16x3", io="f32")
    plan = mk()
    L_ok = plan.expand(d["p"], d["w"])
    y_ok, _ = plan.eval_sorted(L_ok, d["q"])
    torch.cuda.synchronize()
    assert plan.sort_failures() == 0
    F.lib().fc2t2_debug_sort_fault(1)
    try:
        L_bad = plan.expand(d["p"], d["w"])
        _, ws = plan.eval_sorted(L_bad, d["q"])
        torch.cuda.synchronize()
        assert plan.sort_failures() >= 2          # the sources' sort and the queries'
        # every cell came out empty: no moments, so the locals are zero
        assert float(L_bad.abs().max()) == 0.0
        monkeypatch.setenv("FC2T2_DEBUG", "1")
        with pytest.raises(F.FC2T2Error, match="sort"):
            plan.expand(d["p"], d["w"])
        monkeypatch.delenv("FC2T2_DEBUG")
    finally:
        F.lib().fc2t2_debug_sort_fault(0)
    plan.sort_failures(reset=True)
    L2 = plan.expand(d["p"], d["w"])
    y2, _ = plan.eval_sorted(L2, d["q"])
    torch.cuda.synchronize()
    assert plan.sort_failures() == 0
    assert torch.equal(L2, L_ok) and torch.equal(y2, y_ok)
    assert torch.equal(mk().expand(d["p"], d["w"]), L_ok)

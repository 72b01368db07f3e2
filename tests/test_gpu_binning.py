"""Binning and the stable sort by cell (section 3.3), through fc2t2_bin_points, bit-exact
against numpy: the cell of each point (the integer part of its scaled coordinates in the IO
precision, clamped to the grid), a stable argsort of the cell indices, the cell starts, and
the payload carried through the sort.  Grids from 2^4 to 2^21 cells cover one, two and three
passes of 8-bit digits; sizes from one point to several hundred tiles with a ragged last
tile."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_00110_amd import fc2t2
    return fc2t2


def _expected_keys(x, lo, hi, n, dt):
    """The cell index of each point with the library's arithmetic: u = (x - lo) * scale in the
    IO precision, floor, clamp to [0, n - 1]; row-major with the first coordinate slowest."""
    x = x.astype(dt)
    scale = dt(n / (hi - lo))
    u = (x - dt(lo)) * scale
    c = np.floor(u).astype(np.int64)
    c = np.where(u >= 0, c, 0)
    c = np.clip(c, 0, n - 1)
    key = np.zeros(len(x), dtype=np.int64)
    for j in range(x.shape[1]):
        key = key * n + c[:, j]
    return key


def _points(rng, N, dim, lo, hi, n, dt, outside=0.01):
    x = rng.uniform(lo, hi, size=(N, dim))
    # a few points outside the domain (clamped into the boundary cells and counted), and a few
    # on cell faces
    k = int(outside * N)
    if k:
        x[:k] = rng.uniform(lo - 0.5, hi + 0.5, size=(k, dim))
    f = min(N - k, 16)
    if f > 0:
        h = (hi - lo) / n
        x[k:k + f] = lo + h * rng.integers(0, n + 1, size=(f, dim))
    return x.astype(dt)


@pytest.mark.parametrize("dim,n", [(2, 16), (2, 64), (2, 256), (2, 512), (3, 8), (3, 32), (3, 64), (3, 128)])
@pytest.mark.parametrize("N", [1, 1000, 2049, 300_001])
def test_bin_points_matches_numpy(F, dim, n, N):
    lo, hi = -1.0, 1.0
    plan = F.Plan(dim, n, lo, hi, "gaussian", 0.05, 2, m2l="f32", io="f32")
    rng = np.random.default_rng(1000 * dim + n + N)
    x = _points(rng, N, dim, lo, hi, n, np.float32)
    extra = rng.standard_normal(N).astype(np.float32)
    keys = _expected_keys(x, lo, hi, n, np.float32)
    perm = np.argsort(keys, kind="stable")
    starts = np.searchsorted(keys[perm], np.arange(n ** dim + 1), side="left")
    xd, ed = torch.from_numpy(x).cuda(), torch.from_numpy(extra).cuda()
    plan.out_of_domain(reset=True)
    ks, pm, st = plan.bin_points(xd)
    assert np.array_equal(ks.cpu().numpy().astype(np.int64), keys[perm])
    assert np.array_equal(pm.cpu().numpy(), perm)
    assert np.array_equal(st.cpu().numpy().astype(np.int64), starts)
    u = (x - np.float32(lo)) * np.float32(n / (hi - lo))
    n_out = int(np.sum(np.any(~((u >= 0) & (u <= n)), axis=1)))
    assert plan.out_of_domain() == n_out
    # the payload variants: coordinates, and coordinates with one value per point
    ks2, pm2, st2, pay = plan.bin_points(xd, with_payload=True)
    assert np.array_equal(pm2.cpu().numpy(), perm) and np.array_equal(pay.cpu().numpy(), x[perm])
    ks3, pm3, st3, pay3 = plan.bin_points(xd, extra=ed)
    assert np.array_equal(pm3.cpu().numpy(), perm)
    assert np.array_equal(pay3.cpu().numpy(), np.concatenate([x, extra[:, None]], axis=1)[perm])
    assert plan.sort_failures() == 0


@pytest.mark.parametrize("dim,n", [(3, 64), (2, 16)])
def test_bin_points_f64_and_degenerate(F, dim, n):
    """FP64 coordinates; every point in one cell (one digit value, the stable order is the
    input order); no points (all starts zero)."""
    lo, hi = 0.0, 1.0
    plan = F.Plan(dim, n, lo, hi, "gaussian", 0.05, 2, m2l="f64", io="f64")
    rng = np.random.default_rng(7 + n)
    x = _points(rng, 5000, dim, lo, hi, n, np.float64)
    keys = _expected_keys(x, lo, hi, n, np.float64)
    perm = np.argsort(keys, kind="stable")
    ks, pm, st = plan.bin_points(torch.from_numpy(x).cuda())
    assert np.array_equal(pm.cpu().numpy(), perm)
    assert np.array_equal(ks.cpu().numpy().astype(np.int64), keys[perm])
    same = np.full((3000, dim), 0.5 * (lo + hi) + 0.1 / n)
    ks, pm, st = plan.bin_points(torch.from_numpy(same).cuda())
    assert np.array_equal(pm.cpu().numpy(), np.arange(3000))
    c = int(_expected_keys(same[:1], lo, hi, n, np.float64)[0])
    st = st.cpu().numpy()
    assert st[c] == 0 and st[c + 1] == 3000 and st[-1] == 3000
    ks, pm, st = plan.bin_points(torch.empty((0, dim), dtype=torch.float64, device="cuda"))
    assert ks.numel() == 0 and int(st.abs().sum()) == 0
    with pytest.raises(F.FC2T2Error):
        plan.bin_points(torch.from_numpy(x).cuda(), with_payload=True)   # the payload is FP32 only

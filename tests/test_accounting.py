"""Host checks of the work model used for roofline figures (paper_2111_00110_amd/accounting.py):
the admissible-pair count against brute-force enumeration of the parity-window / hole rule, and
the executed-flop count of the tile-skipping M2L against its dense and empty limits."""
import itertools

import numpy as np

from paper_2111_00110_amd import accounting as A


def _brute_pairs(dim, n, finest):
    """(target, source) cell pairs at one level by the rule itself: per dimension o = j - i in
    [-2, 3] for even i and [-3, 2] for odd i, j inside the grid, hole max|o| <= 1 excluded above
    the finest level."""
    count = 0
    for i in itertools.product(range(n), repeat=dim):
        for o in itertools.product(range(-3, 4), repeat=dim):
            ok = True
            for d in range(dim):
                lo, hi = (-2, 3) if i[d] % 2 == 0 else (-3, 2)
                if not (lo <= o[d] <= hi and 0 <= i[d] + o[d] < n):
                    ok = False
                    break
            if ok and not finest and max(abs(v) for v in o) <= 1:
                ok = False
            count += ok
    return count


def test_pair_count_matches_brute_force():
    for dim, n in [(2, 4), (2, 8), (2, 16), (3, 4), (3, 8)]:
        for finest in (True, False):
            assert A.m2l_pairs(dim, n, finest) == _brute_pairs(dim, n, finest), (dim, n, finest)


def test_executed_flops_dense_and_empty_limits():
    for dim, n, K in [(2, 64, 4), (3, 16, 3)]:
        levels = A.levels_of(n)
        dense = [np.ones((n >> l,) * dim, dtype=bool) for l in range(levels)]
        empty = [np.zeros((n >> l,) * dim, dtype=bool) for l in range(levels)]
        full = A.m2l_flops(dim, n, K)
        assert A.m2l_flops_executed(dim, K, dense, False) == full
        assert A.m2l_flops_executed(dim, K, dense, True) == full
        assert A.m2l_flops_executed(dim, K, empty, False) == 0
        assert A.m2l_flops_executed(dim, K, empty, True) == 0


def test_occupancy_pyramid_and_partial_skipping():
    rng = np.random.default_rng(3)
    n, dim, K = 32, 3, 3
    x = 0.2 + 0.05 * rng.random((500, dim)) * 2.0 - 1.0      # a small cluster in one corner of [-1, 1]^3
    occ = A.occupancy_pyramid(x, -1.0, 1.0, n, dim)
    assert [o.shape[0] for o in occ] == [32, 16, 8, 4]
    for fine, coarse in zip(occ[:-1], occ[1:]):
        m = coarse.shape[0]
        assert np.array_equal(coarse, fine.reshape(m, 2, m, 2, m, 2).any(axis=(1, 3, 5)))
    full = A.m2l_flops(dim, n, K)
    fwd = A.m2l_flops_executed(dim, K, occ, False)
    tr = A.m2l_flops_executed(dim, K, occ, True)
    assert 0 < tr <= fwd < full


def test_stage_bytes_formula():
    # 2-D, K = 6 (P = 28, P_pad = 28), 256^2 cells, FP32: P2M reads (2 + 1) * 4 B per point and
    # writes one 112-byte row (plus a 4-byte start) per cell
    assert A.stage_bytes("p2m", 2, 256, 6, N=1 << 20) == (1 << 20) * 12 + 65536 * (4 + 112)
    assert A.stage_bytes("l2p", 2, 256, 6, M=1 << 20) == (1 << 20) * 12 + 65536 * 112


def test_separable_pass_entries_closed_forms():
    """2-D: the first pass maps S0 onto the full square, sum over n_x of (K + 1 - n_x) inputs
    times K + 1 outputs; the second maps the square back onto S0, P inputs-times-outputs pairs
    of K + 1.  Both are (K + 1)^2 (K + 2) / 2.  3-D passes are symmetric in the first and last."""
    for K in range(1, 7):
        e = A.sep_pass_entries(2, K)
        assert e == [(K + 1) ** 2 * (K + 2) // 2] * 2
        assert e[1] == A.n_terms(2, K) * (K + 1)
    for K in range(1, 6):
        e = A.sep_pass_entries(3, K)
        assert e[0] == e[2] == A.n_terms(3, K) * (K + 1)
        # middle pass: (k_x, n_z) groups, (K + 1 - n_z) inputs x (K + 1 - k_x) outputs
        assert e[1] == ((K + 1) * (K + 2) // 2) ** 2


def test_separable_flops_far_below_dense():
    assert A.m2l_flops_separable(2, 256, 6) * 9 < A.m2l_flops(2, 256, 6)
    assert A.m2l_flops_separable(3, 64, 5) * 80 < A.m2l_flops(3, 64, 5)

"""Pins of the FP64 CPU checker against facts fixed by the paper and by mathematics.

Every check here compares the checker with something other than itself: printed sizes,
closed forms, library routines (sympy, scipy), exactness for polynomial kernels, brute
force on tiny inputs, adjoint identities and finite differences.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import direct, fmm, kernels, rays

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v, _cite = line.split()
            out[k] = float(v)
    return out


def random_poly_kernel(rng, d, deg):
    """Random polynomial psi of total degree <= deg with odd and even terms."""
    return kernels.Polynomial({a: rng.standard_normal() for a in fmm.multi_indices(d, deg)}, d)


# ----------------------------------------------------------------------------- printed sizes

def test_multi_index_counts_match_paper():
    g = _golden("paper_sizes.txt")
    assert len(fmm.multi_indices(3, 4)) == g["P_3d_rho4"]
    assert len(fmm.multi_indices(2, 1)) == g["P_2d_rho1"]
    assert len(fmm.multi_indices(2, 2)) == g["P_2d_rho2"]
    for d in (2, 3):
        for K in range(0, 7):
            idx = fmm.multi_indices(d, K)
            assert len(idx) == math.comb(K + d, d)
            assert len(set(idx)) == len(idx)
            degs = [sum(a) for a in idx]
            assert degs == sorted(degs)


def test_expansion_memory_matches_paper():
    g = _golden("paper_sizes.txt")
    P = len(fmm.multi_indices(3, 4))
    for lv, n in ((4, 32), (5, 64), (6, 128)):
        geo = fmm.Geometry(3, n, -1.0, 1.0, 4)
        assert geo.levels == lv
        mb = n ** 3 * P * 4 / 1e6
        assert math.floor(mb * 10) / 10 == g["mb_level%d" % lv]
    assert fmm.Geometry(3, int(g["n_levels4"]), -1, 1, 4).levels == 4


# ----------------------------------------------------------------------------- derivatives

def test_gaussian_derivatives_match_sympy():
    import sympy as sp
    sigma = 0.37
    ker = kernels.Gaussian(sigma)
    xs = sp.symbols("x0:3", real=True)
    expr = sp.exp(-(xs[0] ** 2 + xs[1] ** 2 + xs[2] ** 2) / (2 * sp.Float(sigma, 30) ** 2))
    rng = np.random.default_rng(3)
    pts = rng.uniform(-1, 1, (5, 3))
    gammas = [g for g in fmm.multi_indices(3, 8) if sum(g) in (0, 1, 3, 8)]
    got = ker.derivs(pts, gammas)
    for gi, g in enumerate(gammas):
        e = expr
        for j, m in enumerate(g):
            if m:
                e = sp.diff(e, xs[j], m)
        f = sp.lambdify(xs, e, "mpmath")
        want = np.array([float(f(*map(float, p))) for p in pts])
        np.testing.assert_allclose(got[:, gi], want, rtol=1e-10, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("kind", ["gaussian", "imq"])
def test_derivatives_reproduce_kernel_by_taylor_series(kind):
    """sum_g D_g(x0) h^g / g! -> psi(x0 + h) with error O(|h|^(order+1))."""
    d = 3
    ker = kernels.Gaussian(0.5) if kind == "gaussian" else kernels.IMQ(0.3, d)
    rng = np.random.default_rng(4)
    x0 = rng.uniform(-0.6, 0.6, 3)
    order = 8
    gammas = fmm.multi_indices(d, order)
    D = ker.derivs(x0[None], gammas)[0]
    errs = []
    for scale in (0.02, 0.01):
        h = scale * rng.standard_normal(3)
        approx = sum(D[i] * np.prod(h ** np.array(g)) / fmm.ifact(g) for i, g in enumerate(gammas))
        errs.append(abs(approx - ker.value((x0 + h)[None])[0]))
    assert errs[0] < 1e-12 and errs[1] < 1e-13


@pytest.mark.parametrize("kind", ["gaussian", "imq"])
def test_kernel_gradient_matches_finite_differences(kind):
    ker = kernels.Gaussian(0.3) if kind == "gaussian" else kernels.IMQ(0.2, 3)
    rng = np.random.default_rng(5)
    x = rng.uniform(-0.5, 0.5, (7, 3))
    g = ker.grad(x)
    eps = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = eps
        fd = (ker.value(x + e) - ker.value(x - e)) / (2 * eps)
        np.testing.assert_allclose(g[:, j], fd, rtol=1e-7, atol=1e-9)
    # first-order entries of derivs agree with grad
    D = ker.derivs(x, [(1, 0, 0), (0, 1, 0), (0, 0, 1)])
    np.testing.assert_allclose(D, g, rtol=1e-12, atol=1e-14)


# ----------------------------------------------------------------------------- exactness

@pytest.mark.parametrize("d,n,K,deg", [(2, 4, 2, 2), (2, 8, 4, 4), (2, 16, 3, 3), (2, 8, 6, 5),
                                       (3, 4, 2, 2), (3, 8, 3, 3)])
@pytest.mark.parametrize("triangular", [False, True])
def test_polynomial_kernel_is_exact(d, n, K, deg, triangular):
    """For psi a polynomial of total degree <= K every stage is exact, so the expansion
    equals the direct sum to rounding, forward and backward (catches signs, factorials,
    multi-index order, shift directions and the level partition)."""
    rng = np.random.default_rng(100 + 10 * d + n + K)
    ker = random_poly_kernel(rng, d, deg)
    geo = fmm.Geometry(d, n, -0.7, 1.3, K)
    N, M = 150, 120
    p = rng.uniform(-0.7, 1.3, (N, d))
    q = rng.uniform(-0.7, 1.3, (M, d))
    w = rng.standard_normal((N, 2))
    gy = rng.standard_normal((M, 2))
    y, gw, gp, gq = fmm.explicit_forward_backward(geo, ker, p, w, q, gy, triangular)
    yd = direct.explicit_y(ker, p, w, q)
    gwd, gpd, gqd = direct.explicit_grads(ker, p, w, q, gy)
    assert rel(y, yd) < 1e-12
    assert rel(gw, gwd) < 1e-12
    assert rel(gp, gpd) < 1e-11
    assert rel(gq, gqd) < 1e-11


def test_constant_kernel_counts_every_pair_once():
    """psi == 1: every query sees sum_n w_n exactly once (no pair missed or doubled)."""
    for d, n in ((2, 16), (2, 32), (3, 8)):
        ker = kernels.Polynomial({(0,) * d: 1.0}, d)
        geo = fmm.Geometry(d, n, 0.0, 1.0, 1)
        rng = np.random.default_rng(n)
        p = rng.uniform(0, 1, (200, d))
        w = rng.standard_normal((200, 1))
        q = rng.uniform(0, 1, (50, d))
        y = fmm.l2p(geo, fmm.expand(geo, ker, p, w), q)
        np.testing.assert_allclose(y[:, 0], np.full(50, w.sum()), rtol=1e-13)


def test_interaction_lists_partition_all_cell_pairs():
    """Brute force over finest cell pairs: the level rule assigns each pair exactly once."""
    for d, n in ((2, 16), (3, 8)):
        geo = fmm.Geometry(d, n, 0, 1, 1)
        count = {}
        for lv in range(geo.levels):
            n_l = geo.cells(lv)
            for o in fmm.offsets(d):
                if not fmm.in_window(o, lv == 0):
                    continue
                mask = fmm.window_mask(n_l, o)
                for i in zip(*np.nonzero(mask)):
                    j = tuple(a + b for a, b in zip(i, o))
                    # expand level-lv cell pair to finest pairs
                    s = 1 << lv
                    for ii in itertools.product(*[range(a * s, a * s + s) for a in i]):
                        for jj in itertools.product(*[range(a * s, a * s + s) for a in j]):
                            count[(ii, jj)] = count.get((ii, jj), 0) + 1
        assert len(count) == (n ** d) ** 2
        assert set(count.values()) == {1}


# ----------------------------------------------------------------------------- operators

def test_m2m_equals_direct_coarse_p2m():
    rng = np.random.default_rng(6)
    for d in (2, 3):
        geo = fmm.Geometry(d, 16, -1, 1, 4)
        p = rng.uniform(-1, 1, (300, d))
        w = rng.standard_normal((300, 1))
        M1 = fmm.m2m(geo, 0, fmm.p2m(geo, p, w))
        coarse = fmm.Geometry(d, 8, -1, 1, 4)
        np.testing.assert_allclose(M1, fmm.p2m(coarse, p, w), rtol=1e-12, atol=1e-14)


def test_l2l_preserves_the_parent_polynomial():
    rng = np.random.default_rng(7)
    d = 3
    geo = fmm.Geometry(d, 8, -1, 1, 4)
    parent = rng.standard_normal((1, 4, 4, 4, geo.P))
    child = fmm.l2l(geo, 0, parent)
    x = rng.uniform(-1, 1, (100, d))
    coarse = fmm.Geometry(d, 4, -1, 1, 4)
    np.testing.assert_allclose(fmm.l2p(geo, child, x), fmm.l2p(coarse, parent, x), rtol=1e-11)


def test_sampled_locals_equal_full_expansion():
    rng = np.random.default_rng(8)
    geo = fmm.Geometry(3, 8, -1, 1, 3)
    ker = kernels.Gaussian(0.2)
    p = rng.uniform(-1, 1, (200, 3))
    w = rng.standard_normal((200, 2))
    L0 = fmm.expand(geo, ker, p, w)
    cells = rng.integers(0, 8, (6, 3))
    got = fmm.locals_at_cells(geo, ker, fmm.moments_all_levels(geo, p, w), cells)
    want = L0[:, cells[:, 0], cells[:, 1], cells[:, 2], :]
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14)


# ----------------------------------------------------------------------------- invariants

def test_linear_in_w_and_translation_invariant():
    rng = np.random.default_rng(9)
    geo = fmm.Geometry(2, 16, 0.0, 1.0, 4)
    ker = kernels.Gaussian(0.05)
    p = rng.uniform(0, 1, (300, 2))
    q = rng.uniform(0, 1, (100, 2))
    w1 = rng.standard_normal((300, 1))
    w2 = rng.standard_normal((300, 1))
    f = lambda w: fmm.l2p(geo, fmm.expand(geo, ker, p, w), q)
    np.testing.assert_allclose(f(2 * w1 - 3 * w2), 2 * f(w1) - 3 * f(w2), rtol=1e-11, atol=1e-13)
    shift = 0.25                                       # dyadic: cell indices unchanged
    g2 = fmm.Geometry(2, 16, shift, 1.0 + shift, 4)
    y2 = fmm.l2p(g2, fmm.expand(g2, ker, p + shift, w1), q + shift)
    np.testing.assert_allclose(y2, f(w1), rtol=1e-11, atol=1e-13)


def test_gaussian_error_shrinks_with_order():
    rng = np.random.default_rng(10)
    geo_k = lambda K: fmm.Geometry(2, 16, 0, 1, K)
    ker = kernels.Gaussian(0.08)
    p = rng.uniform(0, 1, (400, 2))
    q = rng.uniform(0, 1, (200, 2))
    w = rng.standard_normal((400, 1))
    yd = direct.explicit_y(ker, p, w, q)
    errs = [rel(fmm.l2p(geo_k(K), fmm.expand(geo_k(K), ker, p, w), q), yd) for K in (2, 4, 6)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3 and errs[2] < 1e-3


def test_adjoint_identity_gaussian():
    """sum gy . y = sum w . w_bar for the expansion (y is linear in w)."""
    rng = np.random.default_rng(11)
    for d, n in ((2, 16), (3, 8)):
        geo = fmm.Geometry(d, n, -1, 1, 3)
        ker = kernels.Gaussian(0.15)
        p = rng.uniform(-1, 1, (200, d))
        q = rng.uniform(-1, 1, (150, d))
        w = rng.standard_normal((200, 2))
        gy = rng.standard_normal((150, 2))
        y, gw, gp, gq = fmm.explicit_forward_backward(geo, ker, p, w, q, gy)
        assert abs(np.sum(gy * y) - np.sum(w * gw)) < 1e-12 * np.sum(np.abs(gy * y))


def test_gradients_match_finite_differences_with_cells_fixed():
    rng = np.random.default_rng(12)
    geo = fmm.Geometry(2, 8, 0, 1, 4)
    ker = kernels.Gaussian(0.12)
    h = geo.h(0)
    # keep points away from cell faces so +-eps never changes a cell
    def interior(m):
        c = rng.integers(0, 8, (m, 2))
        return (c + rng.uniform(0.2, 0.8, (m, 2))) * h
    p, q = interior(40), interior(30)
    w = rng.standard_normal((40, 1))
    gy = rng.standard_normal((30, 1))
    y, gw, gp, gq = fmm.explicit_forward_backward(geo, ker, p, w, q, gy)
    loss = lambda pp, qq: float(np.sum(gy * fmm.l2p(geo, fmm.expand(geo, ker, pp, w), qq)))
    eps = 1e-6
    for s, j in ((3, 0), (17, 1)):
        e = np.zeros_like(p)
        e[s, j] = eps
        fd = (loss(p + e, q) - loss(p - e, q)) / (2 * eps)
        assert abs(fd - gp[s, j]) < 1e-6 * max(1.0, abs(fd))
    for m, j in ((5, 1), (22, 0)):
        e = np.zeros_like(q)
        e[m, j] = eps
        fd = (loss(p, q + e) - loss(p, q - e)) / (2 * eps)
        assert abs(fd - gq[m, j]) < 1e-6 * max(1.0, abs(fd))


def test_direct_gradients_match_finite_differences():
    rng = np.random.default_rng(13)
    ker = kernels.Gaussian(0.2)
    p = rng.uniform(0, 1, (20, 2))
    q = rng.uniform(0, 1, (15, 2))
    w = rng.standard_normal((20, 1))
    gy = rng.standard_normal((15, 1))
    gw, gp, gq = direct.explicit_grads(ker, p, w, q, gy)
    loss = lambda pp, ww, qq: float(np.sum(gy * direct.explicit_y(ker, pp, ww, qq)))
    eps = 1e-6
    e = np.zeros_like(p); e[4, 1] = eps
    assert abs((loss(p + e, w, q) - loss(p - e, w, q)) / (2 * eps) - gp[4, 1]) < 1e-7
    e = np.zeros_like(q); e[7, 0] = eps
    assert abs((loss(p, w, q + e) - loss(p, w, q - e)) / (2 * eps) - gq[7, 0]) < 1e-7
    e = np.zeros_like(w); e[2, 0] = eps
    assert abs((loss(p, w + e, q) - loss(p, w - e, q)) / (2 * eps) - gw[2, 0]) < 1e-7


def test_cell_index_rounding_rule():
    geo32 = fmm.Geometry(3, 64, -1.0, 1.0, 1, np.float32)
    face = np.float32(-1.0 + 2.0 / 64)                      # between cells 0 and 1
    below = np.nextafter(face, np.float32(-2.0))
    x = np.array([[-1.0, 1.0, 0.0], [below, face, 0.0]], dtype=np.float32)
    c = geo32.cell_index(x)
    assert c[0].tolist() == [0, 63, 32]          # x = lo -> 0, x = hi -> last cell, 0 -> n/2
    assert c[1].tolist() == [0, 1, 32]           # just below a face stays below, a face goes up


# ----------------------------------------------------------------------------- rays

def _rays(rng, R):
    v = rng.standard_normal((R, 3))
    o = 2.0 * v / np.linalg.norm(v, axis=1, keepdims=True)
    r = -o + rng.uniform(-0.3, 0.3, (R, 3))
    return o, r / np.linalg.norm(r, axis=1, keepdims=True)


def test_segments_tile_the_clipped_ray():
    rng = np.random.default_rng(14)
    geo = fmm.Geometry(3, 16, -1, 1, 2)
    o, r = _rays(rng, 20)
    for i in range(20):
        segs = rays.segments(geo, o[i], r[i], 0.0, 4.0)
        ta, tb = direct.clip_ray(o[i], r[i], 0.0, 4.0, -1, 1)
        assert abs(segs[0][1] - ta) < 1e-15 and abs(segs[-1][2] - tb) < 1e-15
        assert len(segs) <= 3 * geo.n
        for (c0, _, b0), (c1, a1, _) in zip(segs[:-1], segs[1:]):
            assert b0 == a1
            assert sum(abs(x - y) for x, y in zip(c0, c1)) == 1   # face neighbours


def test_ray_integral_exact_for_polynomial_kernel():
    rng = np.random.default_rng(15)
    ker = random_poly_kernel(rng, 3, 3)
    geo = fmm.Geometry(3, 8, -1, 1, 3)
    p = rng.uniform(-0.8, 0.8, (60, 3))
    w = rng.standard_normal((60, 2))
    o, r = _rays(rng, 6)
    L0 = fmm.expand(geo, ker, p, w)
    y = rays.ray_integral(geo, L0, o, r, 0.0, 4.0)
    xg, wg = np.polynomial.legendre.leggauss(8)        # exact for degree <= 15
    for i in range(6):
        ta, tb = direct.clip_ray(o[i], r[i], 0.0, 4.0, -1, 1)
        t = 0.5 * (tb - ta) * xg + 0.5 * (tb + ta)
        f = direct.explicit_y(ker, p, w, o[i][None] + t[:, None] * r[i][None])
        want = 0.5 * (tb - ta) * (wg @ f)
        np.testing.assert_allclose(y[i], want, rtol=1e-11, atol=1e-11)


def test_gaussian_ray_integral_closed_form_matches_quadrature():
    from scipy import integrate
    rng = np.random.default_rng(16)
    ker = kernels.Gaussian(0.1)
    p = rng.uniform(-0.5, 0.5, (30, 3))
    w = rng.standard_normal((30, 1))
    o, r = _rays(rng, 3)
    for i in range(3):
        ta, tb = direct.clip_ray(o[i], r[i], 0.0, 4.0, -1, 1)
        cf = direct.ray_integral_gaussian(0.1, p, w, o[i], r[i], ta, tb)[0]
        f = lambda t: direct.explicit_y(ker, p, w, (o[i] + t * r[i])[None], threads=1)[0, 0]
        qv = integrate.quad(f, ta, tb, limit=200, epsabs=1e-13, epsrel=1e-12)[0]
        assert abs(cf - qv) < 1e-10


def test_ray_integral_adjoint_identity():
    rng = np.random.default_rng(17)
    geo = fmm.Geometry(3, 8, -1, 1, 3)
    o, r = _rays(rng, 5)
    L0 = rng.standard_normal((2, 8, 8, 8, geo.P))
    gy = rng.standard_normal((5, 2))
    lhs = np.sum(gy * rays.ray_integral(geo, L0, o, r, 0.0, 4.0))
    rhs = np.sum(L0 * rays.ray_integral_T(geo, o, r, 0.0, 4.0, gy, 2))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_line2poly_agrees_with_pointwise_l2p():
    rng = np.random.default_rng(18)
    geo = fmm.Geometry(3, 8, -1, 1, 4)
    L0 = rng.standard_normal((1, 8, 8, 8, geo.P))
    o, r = _rays(rng, 3)
    for i in range(3):
        for cell, ta, tb in rays.segments(geo, o[i], r[i], 0.0, 4.0)[::5]:
            d = o[i] + ta * r[i] - geo.centre(0, np.asarray(cell))
            a = rays.line2poly(geo.idx, L0[(0,) + cell], d, r[i])
            u = np.linspace(0, tb - ta, 4)
            x = o[i][None] + (ta + u)[:, None] * r[i][None]
            mono = fmm.monomials(x - geo.centre(0, np.asarray(cell)), geo.idx)
            np.testing.assert_allclose(np.polynomial.polynomial.polyval(u, a),
                                       mono @ L0[(0,) + cell], rtol=1e-12, atol=1e-12)


def test_real_roots_match_numpy_roots():
    rng = np.random.default_rng(19)
    for _ in range(50):
        roots_true = np.sort(rng.uniform(-1, 2, 5))
        c = np.polynomial.polynomial.polyfromroots(roots_true) * rng.uniform(0.5, 2)
        got = rays.real_roots(c, 0.0, 1.0)
        want = [x for x in roots_true if 0.0 <= x <= 1.0]
        np.testing.assert_allclose(got, want, atol=1e-12)


def test_ray_root_exact_for_polynomial_field():
    """A polynomial psi makes f along the ray one global polynomial; its max and first
    upward level crossing follow from numpy.roots on that polynomial."""
    rng = np.random.default_rng(20)
    d, K = 3, 4
    ker = kernels.Polynomial({(0, 0, 0): 1.0, (2, 0, 0): -1.0, (0, 2, 0): -1.0, (0, 0, 2): -1.0,
                              (1, 0, 0): 0.3, (1, 1, 0): 0.2}, d)
    geo = fmm.Geometry(d, 8, -1, 1, K)
    p = rng.uniform(-0.3, 0.3, (25, 3))
    w = rng.uniform(0.5, 1.0, (25, 1))
    o, r = _rays(rng, 4)
    L0 = fmm.expand(geo, ker, p, w)
    res = rays.ray_root(geo, L0, o, r, 0.0, 4.0)
    for i in range(4):
        ta, tb = direct.clip_ray(o[i], r[i], 0.0, 4.0, -1, 1)
        ts = np.linspace(ta, tb, 9)
        vals = direct.explicit_y(ker, p, w, o[i][None] + ts[:, None] * r[i][None])[:, 0]
        g = np.polynomial.polynomial.polyfit(ts, vals, 8)
        crit = [x.real for x in np.roots(np.polynomial.polynomial.polyder(g)[::-1])
                if abs(x.imag) < 1e-9 and ta <= x.real <= tb]
        fmax = max(np.polynomial.polynomial.polyval(x, g) for x in crit + [ta, tb])
        tau = 0.5 * fmax
        assert abs(res["tau"][i] - tau) < 1e-9 * abs(tau)
        g2 = g.copy(); g2[0] -= tau
        cand = sorted(x.real for x in np.roots(g2[::-1]) if abs(x.imag) < 1e-9 and ta <= x.real <= tb
                      and np.polynomial.polynomial.polyval(x.real, np.polynomial.polynomial.polyder(g)) > 0)
        if np.polynomial.polynomial.polyval(ta, g2) >= 0 or not cand:
            assert res["hit"][i] == 0
        else:
            assert res["hit"][i] == 1
            assert abs(res["t"][i] - cand[0]) < 1e-9


def test_ray_root_gaussian_close_to_direct_root():
    rng = np.random.default_rng(21)
    sigma = 0.1
    ker = kernels.Gaussian(sigma)
    geo = fmm.Geometry(3, 32, -1, 1, 5)
    u = rng.standard_normal((300, 3))
    p = 0.5 * u / np.linalg.norm(u, axis=1, keepdims=True)
    w = rng.uniform(0.5, 1.5, (300, 1))
    o, r = _rays(rng, 3)
    L0 = fmm.expand(geo, ker, p, w)
    res = rays.ray_root(geo, L0, o, r, 0.0, 4.0)
    for i in range(3):
        ta, tb = direct.clip_ray(o[i], r[i], 0.0, 4.0, -1, 1)
        t_d, tau_d = direct.ray_root(ker, p, w, o[i], r[i], ta, tb, sigma / 8)
        assert res["hit"][i] == 1
        assert abs(res["tau"][i] - tau_d) < 1e-2 * tau_d
        assert abs(res["t"][i] - t_d) < 2e-3


def test_ray_root_backward_matches_finite_differences():
    """IFT cotangents (tau held fixed) against central differences of the checker's root."""
    rng = np.random.default_rng(22)
    sigma = 0.15
    ker = kernels.Gaussian(sigma)
    geo = fmm.Geometry(3, 16, -1, 1, 4)
    u = rng.standard_normal((80, 3))
    p = 0.5 * u / np.linalg.norm(u, axis=1, keepdims=True)
    w = rng.uniform(0.5, 1.5, (80, 1))
    o, r = _rays(rng, 3)
    L0 = fmm.expand(geo, ker, p, w)
    res = rays.ray_root(geo, L0, o, r, 0.0, 4.0)
    assert res["hit"].all()
    gt = rng.standard_normal(3)
    gn = rng.standard_normal((3, 3))
    GL = rays.ray_root_T(geo, o, r, res, gt, gn)
    gw, gp = fmm.p2m_T(geo, fmm.expand_T(geo, ker, GL), p, w)

    def loss(ww):
        rr = rays.ray_root(geo, fmm.expand(geo, ker, p, ww), o, r, 0.0, 4.0, tau_override=res["tau"])
        return float(gt @ rr["t"] + np.sum(gn * rr["normal"]))
    eps = 1e-6
    for s in (0, 11, 57):
        e = np.zeros_like(w); e[s, 0] = eps
        fd = (loss(w + e) - loss(w - e)) / (2 * eps)
        assert abs(fd - gw[s, 0]) < 1e-5 * max(1.0, abs(fd))


def test_ray_root_face_crossing_belongs_to_earlier_cell():
    """Piecewise-constant field: 0 in the cells x < 0, 1 for x >= 0.  Along +x the level
    0.5 * max = 0.5 is crossed only across the face x = 0, which the root rule assigns to
    the earlier cell (t at the face)."""
    geo = fmm.Geometry(3, 8, -1, 1, 2)
    L0 = np.zeros((1, 8, 8, 8, geo.P))
    L0[0, 4:, :, :, 0] = 1.0
    o = np.array([[-2.0, 0.1, -0.05]])
    r = np.array([[1.0, 0.0, 0.0]])
    res = rays.ray_root(geo, L0, o, r, 0.0, 4.0)
    assert res["hit"][0] == 1 and abs(res["tau"][0] - 0.5) < 1e-15
    assert abs(res["t"][0] - 2.0) < 1e-15
    assert tuple(res["cell"][0]) == (3, 4, 3)
    assert res["kind"][0] == rays.ROOT_FACE


def _face_crossing_field(rng, geo):
    """Locals with a jump across the face x = 0: smooth and below 0.5 in the cells x < 0 next
    to it (x index 3), about 1 beyond it, zero elsewhere; random first and second order terms
    so that the surface gradient and the Hessian are generic."""
    L0 = np.zeros((1,) + (geo.n,) * 3 + (geo.P,))
    L0[0, 3] = 0.04 * rng.standard_normal(L0[0, 3].shape)
    L0[0, 3, ..., 0] += 0.2
    L0[0, 4:] = 0.04 * rng.standard_normal(L0[0, 4:].shape)
    L0[0, 4:, ..., 0] += 1.0
    return L0


def test_ray_root_face_crossing_backward_matches_finite_differences():
    """At a face crossing the root stays on the face when the locals move a little (the jump
    persists), so dt*/dL = 0 and the surface gradient moves only through the locals of the
    earlier cell at the fixed point.  Central differences of the checker's root (tau held
    fixed) against ray_root_T, on a ray that is not axis-aligned."""
    rng = np.random.default_rng(31)
    geo = fmm.Geometry(3, 8, -1, 1, 2)
    L0 = _face_crossing_field(rng, geo)
    o = np.array([[-2.0, 0.1, -0.05]])
    r = np.array([[1.0, 0.05, -0.03]])
    r /= np.linalg.norm(r)
    res = rays.ray_root(geo, L0, o, r, 0.0, 4.0)
    assert res["hit"][0] == 1 and res["kind"][0] == rays.ROOT_FACE
    assert tuple(res["cell"][0]) == (3, 4, 3)
    assert abs(o[0, 0] + res["t"][0] * r[0, 0]) < 1e-14          # on the face x = 0
    gt = np.array([0.7])
    gn = np.array([[0.3, -1.1, 0.4]])
    G = rays.ray_root_T(geo, o, r, res, gt, gn)

    def loss(L):
        rr = rays.ray_root(geo, L, o, r, 0.0, 4.0, tau_override=res["tau"])
        return float(gt @ rr["t"] + np.sum(gn * rr["normal"]))
    eps = 1e-6
    for cell in [(3, 4, 3), (4, 4, 3)]:
        for k in range(geo.P):
            e = np.zeros_like(L0)
            e[(0,) + cell + (k,)] = eps
            fd = (loss(L0 + e) - loss(L0 - e)) / (2 * eps)
            assert abs(fd - G[(0,) + cell + (k,)]) < 1e-7 * max(1.0, abs(fd)), (cell, k)
    # only the earlier cell's locals move the outputs
    assert np.abs(G[0, 4, 4, 3]).max() == 0.0 and np.abs(G[0, 3, 4, 3]).max() > 0.1


def test_ray_root_grazing_root_is_masked():
    """f = A + B x^3 + C y in one cell ((x, y, z) = q - c, the checker's locals are physical
    derivatives at the centre): along +x at fixed y the level A is crossed upward at the cell
    centre with zero slope along the ray, so r . grad f = 0 while grad f = (0, C, 0) is not.  The root is reported as grazing, and its cotangent holds only
    the dipole term n_bar . grad (q* - c)^k / k!, finite.  The same field tilted so that the
    slope along the ray is clearly non-zero gives a smooth root whose cotangent matches central
    differences."""
    geo = fmm.Geometry(3, 8, -1, 1, 3)
    idx = geo.idx
    A, B, C = 0.6, 0.5, 0.3

    def field(slope):
        L0 = np.zeros((1, 8, 8, 8, geo.P))
        L0[0, :4, :, :, 0] = A - 0.5                 # below the level before the cell
        row = np.zeros(geo.P)
        row[idx.index((0, 0, 0))] = A
        row[idx.index((3, 0, 0))] = 6.0 * B          # B x^3 = L x^k / k! with k = (3, 0, 0)
        row[idx.index((0, 1, 0))] = C
        row[idx.index((1, 0, 0))] = slope
        L0[0, 4, 4, 4] = row
        return L0

    o = np.array([[-2.0, 0.125, 0.125]])       # through the centre of cell (4, 4, 4) in y and z
    r = np.array([[1.0, 0.0, 0.0]])
    tau = np.array([A])
    L0 = field(0.0)
    res = rays.ray_root(geo, L0, o, r, 0.0, 4.0, tau_override=tau)
    assert res["hit"][0] == 1 and res["kind"][0] == rays.ROOT_GRAZING
    assert abs(res["t"][0] - (2.0 + 0.125)) < 1e-6    # cube root of rounding at the centre
    np.testing.assert_allclose(res["normal"][0], [0.0, C, 0.0], atol=1e-9)
    gt, gn = np.array([1.3]), np.array([[0.2, -0.5, 0.9]])
    G = rays.ray_root_T(geo, o, r, res, gt, gn)
    assert np.all(np.isfinite(G))
    q = o[0] + res["t"][0] * r[0]
    dq = q - geo.centre(0, np.array([4, 4, 4]))
    np.testing.assert_allclose(G[0, 4, 4, 4], fmm.monomial_grads(dq[None], idx)[0] @ gn[0], atol=1e-12)

    L1 = field(0.2)
    res1 = rays.ray_root(geo, L1, o, r, 0.0, 4.0, tau_override=tau)
    assert res1["hit"][0] == 1 and res1["kind"][0] == rays.ROOT_SMOOTH
    G1 = rays.ray_root_T(geo, o, r, res1, gt, gn)

    def loss(L):
        rr = rays.ray_root(geo, L, o, r, 0.0, 4.0, tau_override=tau)
        return float(gt @ rr["t"] + np.sum(gn * rr["normal"]))
    for k in range(geo.P):
        e = np.zeros_like(L1)
        e[0, 4, 4, 4, k] = 1e-7
        fd = (loss(L1 + e) - loss(L1 - e)) / 2e-7
        assert abs(fd - G1[0, 4, 4, 4, k]) < 1e-5 * max(1.0, abs(fd)), k


def test_smooth_roots_are_not_masked():
    """Roots of a generic field cross the level at a clear angle: none is flagged."""
    rng = np.random.default_rng(22)
    ker = kernels.Gaussian(0.15)
    geo = fmm.Geometry(3, 16, -1, 1, 4)
    u = rng.standard_normal((80, 3))
    p = 0.5 * u / np.linalg.norm(u, axis=1, keepdims=True)
    w = rng.uniform(0.5, 1.5, (80, 1))
    o, r = _rays(rng, 6)
    res = rays.ray_root(geo, fmm.expand(geo, ker, p, w), o, r, 0.0, 4.0)
    assert res["hit"].all() and (res["kind"] == rays.ROOT_SMOOTH).all()


def test_clip_ray_against_dense_membership():
    """The clipped interval against membership of dense samples of the ray in the box, and
    axis-aligned cases with known intervals (entering, starting inside, missing, parallel)."""
    rng = np.random.default_rng(32)
    for _ in range(40):
        o = rng.uniform(-3, 3, 3)
        r = rng.standard_normal(3)
        r /= np.linalg.norm(r)
        ta, tb = direct.clip_ray(o, r, 0.0, 4.0, -1.0, 1.0)
        t = np.linspace(0.0, 4.0, 40001)
        inside = np.all(np.abs(o[None] + t[:, None] * r[None]) <= 1.0, axis=1)
        if not inside.any():
            assert not tb > ta
            continue
        assert abs(t[inside].min() - ta) <= 1e-4 and abs(t[inside].max() - tb) <= 1e-4
    cases = [((-2.0, 0.0, 0.0), (1.0, 0.0, 0.0), (1.0, 3.0)),
             ((0.5, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.5)),
             ((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), (0.0, 1.0)),
             ((-2.0, 1.5, 0.0), (1.0, 0.0, 0.0), None),
             ((-6.0, 0.0, 0.0), (1.0, 0.0, 0.0), None)]
    for o, r, want in cases:
        ta, tb = direct.clip_ray(np.array(o), np.array(r), 0.0, 4.0, -1.0, 1.0)
        if want is None:
            assert not tb > ta
        else:
            assert (ta, tb) == want


# ---------------------------------------------------------------------------------------
# Least-squares fitted M2L tensors (section 3.1)

def _poly_kernel(d, deg, seed):
    rng = np.random.default_rng(seed)
    return kernels.Polynomial({a: rng.standard_normal() for a in fmm.multi_indices(d, deg)}, d)


@pytest.mark.parametrize("d,K", [(2, 3), (2, 6), (3, 2), (3, 4)])
def test_lsq_tensor_exact_for_polynomial_kernels(d, K):
    """A kernel of degree <= K has derivatives that are polynomials of degree <= K in the source
    offset: the fit reproduces them, so the fitted tensor equals the Taylor tensor (computed from
    derivatives at one point, with no sampling)."""
    ker = _poly_kernel(d, K, 3 + K)
    taylor = fmm.Geometry(d, 16, -1.0, 1.0, K)
    fit = fmm.Geometry(d, 16, -1.0, 1.0, K, fit="lsq")
    deg = np.array([sum(a) for a in taylor.idx])
    for level, o in [(0, (0,) * d), (0, (2,) + (-1,) * (d - 1)), (1, (-3,) + (3,) * (d - 1)), (2, (1,) * d)]:
        # compared in cell-scaled units (entry [k, n] times h^(|k| + |n|)), where entries are O(1)
        s = taylor.h(level) ** (deg[:, None] + deg[None, :])
        A = fmm.m2l_tensor(ker, taylor, level, o) * s
        B = fmm.m2l_tensor(ker, fit, level, o) * s
        assert np.abs(A - B).max() <= 1e-9 * np.abs(A).max(), (level, o)


def test_lsq_fit_is_closer_than_taylor_over_the_cell():
    """The fitted polynomial of each derivative is at least as close as the Taylor polynomial in
    L2 over the source cell (measured on an independent 40^2 midpoint grid), and clearly closer
    in total when the Gaussian is narrow against the cell."""
    d, K, sig = 2, 4, 0.01
    ker = kernels.Gaussian(sig)
    geo_t = fmm.Geometry(d, 64, 0.0, 1.0, K)
    geo_f = fmm.Geometry(d, 64, 0.0, 1.0, K, fit="lsq")
    level, o = 0, (2, 1)
    h = geo_t.h(level)
    m = (np.arange(40) + 0.5) / 40 - 0.5
    X = np.array(list(itertools.product(m, m))) * h
    V = fmm.monomials(X, geo_t.idx)
    exact = ker.derivs(-np.asarray(o, float) * h - X, geo_t.idx)           # [S, P(k)]
    err_t = np.linalg.norm(V @ fmm.m2l_tensor(ker, geo_t, level, o).T - exact, axis=0)
    err_f = np.linalg.norm(V @ fmm.m2l_tensor(ker, geo_f, level, o).T - exact, axis=0)
    assert np.all(err_f <= err_t * 1.02 + 1e-12 * np.abs(exact).max())
    assert err_f.sum() < 0.5 * err_t.sum()


def test_lsq_explicit_layer_closer_to_direct_sum():
    """Figure 3's point on the whole layer: with sigma / h = 0.64 the fitted tensors bring the
    expansion closer to the exact sum than the Taylor tensors at the same order."""
    rng = np.random.default_rng(21)
    d, n, K, sig = 2, 64, 4, 0.01
    p = rng.uniform(0, 1, (3000, d))
    q = rng.uniform(0, 1, (500, d))
    w = rng.standard_normal((3000, 1))
    ker = kernels.Gaussian(sig)
    yd = direct.explicit_y(ker, p, w, q)
    err = {}
    for fit in ("taylor", "lsq"):
        geo = fmm.Geometry(d, n, 0.0, 1.0, K, fit=fit)
        y = fmm.l2p(geo, fmm.expand(geo, ker, p, w), q)
        err[fit] = np.linalg.norm(y - yd) / np.linalg.norm(yd)
    assert err["lsq"] < 0.8 * err["taylor"]


@pytest.mark.parametrize("d,n,K", [(2, 16, 4), (3, 8, 3)])
def test_sampled_moment_cotangents_equal_full_transpose(d, n, K):
    """The cell-by-cell transpose (for spot checks at full size) against the full exact
    transpose chain at every cell of a small grid, and the per-row P2M transpose against p2m_T."""
    rng = np.random.default_rng(40 + d)
    ker = kernels.Gaussian(0.1)
    geo = fmm.Geometry(d, n, -1.0, 1.0, K)
    G_L0 = rng.standard_normal((2,) + (n,) * d + (geo.P,))
    full = fmm.expand_T(geo, ker, G_L0)
    cells = np.array(list(itertools.product(range(n), repeat=d)))
    got = fmm.moment_cotangents_at_cells(geo, ker, fmm.local_cotangent_pyramid(geo, G_L0), cells)
    want = full[(slice(None),) + tuple(cells[:, j] for j in range(d))]
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    p = rng.uniform(-1, 1, (50, d))
    w = rng.standard_normal((50, 2))
    pc = geo.cell_index(p)
    rows = full[(slice(None),) + tuple(pc[:, j] for j in range(d))]
    gw, gp = fmm.p2m_T_rows(geo, rows, p, w)
    gw2, gp2 = fmm.p2m_T(geo, full, p, w)
    assert np.abs(gw - gw2).max() <= 1e-12 * np.abs(gw2).max()
    assert np.abs(gp - gp2).max() <= 1e-12 * np.abs(gp2).max()


# ---------------------------------------------------------------------------------------
# Volumetric rendering layer (sections 6.1.2 and 6.2.2)

from oracle import volume  # noqa: E402


def test_mexp_is_the_l2_projection_of_exp():
    """The transmittance polynomial is the L2-best degree-4 fit of exp(-x) on [0, 5]: its residual
    is orthogonal to 1, x, ..., x^4 (scipy quad), and it stays within the fit's error of exp."""
    from scipy import integrate
    m = volume.mexp_coefficients()
    assert len(m) == 5
    for j in range(5):
        v, _ = integrate.quad(lambda x: (math.exp(-x) - np.polynomial.polynomial.polyval(x, m)) * x ** j,
                              0.0, 5.0, epsabs=1e-13, epsrel=1e-12, limit=200)
        assert abs(v) < 1e-11, j
    x = np.linspace(0, 5, 2001)
    err = np.abs(np.polynomial.polynomial.polyval(x, m) - np.exp(-x))
    assert err.max() < 0.06 and err.mean() < 0.02


def _volume_field(rng, geo, dens=0.8):
    L0 = 0.3 * rng.standard_normal((4,) + (geo.n,) * 3 + (geo.P,))
    L0[0, ..., 0] = dens + 0.2 * rng.random((geo.n,) * 3)      # positive density
    return L0


def test_volume_forward_matches_pointwise_quadrature():
    """The cell-by-cell polynomial algebra (line to polynomial, integral, composition with the
    fit, products) against pointwise evaluation of the locals at Gauss-Legendre nodes, with the
    depth at each node integrated separately: the same model by another route."""
    rng = np.random.default_rng(50)
    geo = fmm.Geometry(3, 8, -1, 1, 3)
    L0 = _volume_field(rng, geo, dens=2.0)
    o, r = _rays(rng, 6)
    bg = np.array([0.1, 0.2, 0.3])
    got = volume.render(geo, L0, o, r, 0.0, 4.0, bg)
    m = volume.mexp_coefficients()
    xg, wg = np.polynomial.legendre.leggauss(30)
    assert got["stopped"].any() and not got["stopped"].all()
    for i in range(6):
        D, y, stopped = 0.0, np.zeros(3), False
        for cell, ta, tb in rays.segments(geo, o[i], r[i], 0.0, 4.0):
            s = tb - ta
            c = geo.centre(0, np.asarray(cell))
            f = lambda u: fmm.monomials(o[i][None] + (ta + np.atleast_1d(u))[:, None] * r[i][None] - c, geo.idx) \
                @ L0[(slice(None),) + cell].T                          # [nodes, 4]
            u = 0.5 * s * (xg + 1)
            vals = f(u)
            S = np.array([D + 0.5 * ui * np.sum(wg * f(0.5 * ui * (xg + 1))[:, 0]) for ui in u])
            T = np.polynomial.polynomial.polyval(S, m)
            y += 0.5 * s * np.einsum("n,nk->k", wg * vals[:, 0] * T, vals[:, 1:])
            D += 0.5 * s * np.sum(wg * vals[:, 0])
            if D > volume.STOP_DEPTH:
                stopped = True
                break
        y += bg * (0.0 if stopped else np.polynomial.polynomial.polyval(D, m))
        assert stopped == got["stopped"][i]
        np.testing.assert_allclose(got["y"][i], y, rtol=1e-11, atol=1e-12)


def test_volume_constant_field_closed_form():
    """Constant density s0 and colour c0 along a ray through the box: S grows linearly, so
    y = c0 int_0^{D_end} mexp(x) dx + c_bg mexp(D_end); with a dense medium the traversal stops
    after the cell where the depth passes 4.5 and the background is not seen."""
    geo = fmm.Geometry(3, 8, -1, 1, 2)
    m = volume.mexp_coefficients()
    M = np.polynomial.polynomial.polyint(m)
    c0 = np.array([0.2, 0.5, 0.7])
    bg = np.array([1.0, 0.5, 0.25])
    o = np.array([[-2.0, 0.1, 0.3]])
    r = np.array([[1.0, 0.0, 0.0]])
    for s0, stop_cell in ((0.3, None), (5.0, 3)):
        L0 = np.zeros((4,) + (8,) * 3 + (geo.P,))
        L0[0, ..., 0] = s0
        L0[1:, ..., 0] = c0[:, None, None, None]
        got = volume.render(geo, L0, o, r, 0.0, 4.0, bg)
        if stop_cell is None:
            D = s0 * 2.0
            want = c0 * np.polynomial.polynomial.polyval(D, M) + bg * np.polynomial.polynomial.polyval(D, m)
            assert not got["stopped"][0]
        else:
            D = s0 * 0.25 * (stop_cell + 1)          # depth at the exit of the stopping cell
            want = c0 * np.polynomial.polynomial.polyval(D, M)
            assert got["stopped"][0]
        assert abs(got["D_end"][0] - D) < 1e-13
        np.testing.assert_allclose(got["y"][0], want, rtol=1e-13)


@pytest.mark.parametrize("dens,bgv", [(0.8, (0.3, -0.2, 0.5)), (2.5, (0.0, 0.0, 0.0))])
def test_volume_backward_matches_finite_differences(dens, bgv):
    """The backward (colour insertion, and the density insertion with the running integral of
    c sigma mexp'(S)) against central differences of the forward on entries of all four
    channels; with a medium thin enough to see the background and one dense enough to stop."""
    rng = np.random.default_rng(51)
    geo = fmm.Geometry(3, 4, -1, 1, 2)
    L0 = _volume_field(rng, geo, dens=dens)
    o, r = _rays(rng, 3)
    bg = np.array(bgv)
    gy = rng.standard_normal((3, 3))
    fwd = volume.render(geo, L0, o, r, 0.0, 4.0, bg)
    G = volume.render_T(geo, L0, o, r, 0.0, 4.0, fwd, gy, bg)
    loss = lambda L: float(np.sum(gy * volume.render(geo, L, o, r, 0.0, 4.0, bg)["y"]))
    flat = np.flatnonzero(np.abs(G) > 0)
    picks = rng.choice(flat, size=24, replace=False)
    eps = 1e-6
    for f in picks:
        e = np.zeros(L0.size)
        e[f] = eps
        e = e.reshape(L0.shape)
        fd = (loss(L0 + e) - loss(L0 - e)) / (2 * eps)
        assert abs(fd - G.flat[f]) < 1e-6 * max(1.0, abs(fd)), (np.unravel_index(f, L0.shape), fd, G.flat[f])

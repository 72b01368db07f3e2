"""Volumetric rendering layer on the local expansions, FP64 numpy -- TEST INFRASTRUCTURE ONLY.

Section 6.1.2 (forward) and section 6.2.2 (backward) of the paper.  Four channels of locals:
channel 0 is the density sigma, channels 1..3 the colour c = (R, G, B).  Along a ray the colour
is y = int T(x) sigma(x) c(x) dx + c_bg T_end with the transmittance T(x) = exp(-S(x)),
S(x) = int_0^x sigma.  As in the paper, exp(-S) is replaced by a degree-4 polynomial `mexp`
fitted to exp(-x) on [0, 5] (the paper names neither the fit nor its norm; reading: the L2-best
polynomial on [0, 5]), so inside one cell every factor is a polynomial of the ray parameter and
each cell's integral is exact:
    S(u) = D + int_0^u sigma,    T(u) = mexp(S(u)),    y += int_0^s c(u) sigma(u) T(u) du,
with D the optical depth at the cell's entry; the traversal stops after the first cell whose
exit depth exceeds 4.5 (the fit is only used below 5), and then T_end = 0, else
T_end = mexp(D_end).

Backward (reading): the exact derivative of this forward.  The colour locals receive
    int mono(u) sigma(u) T(u) du * y_bar_k          (the paper's case 1),
and the density locals
    int mono(u) H(u) du,  H = sum_k y_bar_k [c_k T + G_k(end) - G_k(x)] + (y_bar . c_bg) mexp'(D_end),
with G_k(x) = int_0^x c_k sigma mexp'(S): a change of sigma at x changes S at every later point.
The paper writes the same sums with -T in place of mexp'(S) (exact for exp, since
d/dS exp(-S) = -exp(-S)), the "ordered causal" form in which the later part is the forward's
total minus the running sum; the degree-4 fit satisfies that identity only approximately, so the
exact derivative of the computed forward uses mexp'.  The stop decision is not differentiated
(it changes only at measure-zero depths).  mono(u) = (d + r u)^n / n!, d = entry point - centre.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import polynomial as npoly

from . import fmm, rays

MEXP_DEGREE = 4
MEXP_RANGE = 5.0
STOP_DEPTH = 4.5


def mexp_coefficients() -> np.ndarray:
    """Coefficients (low to high, in x) of the degree-4 polynomial closest to exp(-x) in L2 on
    [0, 5]: the normal equations in t = x / 5, Gram matrix 1 / (i + j + 1), right-hand side
    int_0^1 t^i exp(-5 t) dt = i! / 5^(i+1) (1 - exp(-5) sum_{k<=i} 5^k / k!)."""
    n = MEXP_DEGREE + 1
    a = MEXP_RANGE
    G = np.array([[1.0 / (i + j + 1) for j in range(n)] for i in range(n)])
    b = np.array([math.factorial(i) / a ** (i + 1) * (1.0 - math.exp(-a) * sum(a ** k / math.factorial(k)
                                                                           for k in range(i + 1)))
                  for i in range(n)])
    ct = np.linalg.solve(G, b)                   # in t
    return ct / a ** np.arange(n)                # in x


def _compose(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """p(q(u)) by Horner over polynomials."""
    out = np.array([p[-1]])
    for c in p[-2::-1]:
        out = npoly.polyadd(npoly.polymul(out, q), [c])
    return out


def _int0(c: np.ndarray, s: float) -> float:
    """int_0^s of the polynomial c."""
    return float(npoly.polyval(s, npoly.polyint(c)))


def _cell_polys(geo, L0, cell, d, r):
    return [rays.line2poly(geo.idx, L0[(ch,) + cell], d, r) for ch in range(4)]


def render(geo: fmm.Geometry, L0: np.ndarray, o, r, t0: float, t1: float, bg=(0.0, 0.0, 0.0)) -> dict:
    """Per ray: colour y [R, 3], exit transmittance T_end [R], exit depth D_end [R], whether the
    traversal stopped [R], G [R, 3] = int c_k sigma mexp'(S) over the traversal (kept for
    the backward), and margin [R] = the smallest |exit depth - STOP_DEPTH| over the cells
    visited (how far the stop decision is from flipping).  L0 has four channels (density, R,
    G, B), physical units."""
    m = mexp_coefficients()
    mp = npoly.polyder(m)
    bg = np.asarray(bg, dtype=np.float64)
    R = len(o)
    out = {"y": np.zeros((R, 3)), "T_end": np.zeros(R), "D_end": np.zeros(R),
           "stopped": np.zeros(R, dtype=bool), "G": np.zeros((R, 3)), "margin": np.full(R, np.inf)}
    for ri in range(R):
        D = 0.0
        y = np.zeros(3)
        G = np.zeros(3)
        stopped = False
        for cell, ta, tb in rays.segments(geo, o[ri], r[ri], t0, t1):
            d = rays._seg_local(geo, cell, o[ri], r[ri], ta)
            s = tb - ta
            sig, *cols = _cell_polys(geo, L0, cell, d, r[ri])
            S = npoly.polyint(sig)
            S[0] += D
            T = _compose(m, S)
            Tp = _compose(mp, S)
            for k in range(3):
                cs = npoly.polymul(cols[k], sig)
                y[k] += _int0(npoly.polymul(cs, T), s)
                G[k] += _int0(npoly.polymul(cs, Tp), s)
            D = float(npoly.polyval(s, S))
            out["margin"][ri] = min(out["margin"][ri], abs(D - STOP_DEPTH))
            if D > STOP_DEPTH:
                stopped = True
                break
        T_end = 0.0 if stopped else float(npoly.polyval(D, m))
        out["y"][ri] = y + bg * T_end
        out["T_end"][ri] = T_end
        out["D_end"][ri] = D
        out["stopped"][ri] = stopped
        out["G"][ri] = G
    return out


def render_T(geo: fmm.Geometry, L0: np.ndarray, o, r, t0: float, t1: float, fwd: dict, gy,
             bg=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Cotangent of the four channels of locals from colour cotangents gy [R, 3] (the exact
    derivative of `render`, module docstring)."""
    m = mexp_coefficients()
    mp = npoly.polyder(m)
    bg = np.asarray(bg, dtype=np.float64)
    gy = np.asarray(gy, dtype=np.float64).reshape(len(o), 3)
    G_out = np.zeros((4,) + (geo.n,) * geo.dim + (geo.P,))
    for ri in range(len(o)):
        D = 0.0
        Gb = np.zeros(3)
        bg_term = 0.0 if fwd["stopped"][ri] else float(gy[ri] @ bg) * float(npoly.polyval(fwd["D_end"][ri], mp))
        for cell, ta, tb in rays.segments(geo, o[ri], r[ri], t0, t1):
            d = rays._seg_local(geo, cell, o[ri], r[ri], ta)
            s = tb - ta
            sig, *cols = _cell_polys(geo, L0, cell, d, r[ri])
            S = npoly.polyint(sig)
            S[0] += D
            T = _compose(m, S)
            Tp = _compose(mp, S)
            sigT = npoly.polymul(sig, T)
            H = np.array([bg_term])
            for k in range(3):
                cs = npoly.polymul(cols[k], sig)
                run = npoly.polyint(npoly.polymul(cs, Tp))          # int_0^u within the cell
                run[0] += Gb[k]
                Hk = npoly.polyadd(npoly.polymul(cols[k], T), npoly.polysub([fwd["G"][ri, k]], run))
                H = npoly.polyadd(H, gy[ri, k] * Hk)
                Gb[k] += _int0(npoly.polymul(cs, Tp), s)
            for j, mono in enumerate(rays.monomial_polys(geo.idx, d, r[ri])):
                G_out[(0,) + cell + (j,)] += _int0(npoly.polymul(mono, H), s)
                w = _int0(npoly.polymul(mono, sigT), s)
                for k in range(3):
                    G_out[(k + 1,) + cell + (j,)] += w * gy[ri, k]
            D = float(npoly.polyval(s, S))
            if D > STOP_DEPTH:
                break
    return G_out

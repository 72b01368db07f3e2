"""Ray layers on the local expansions, FP64 numpy -- TEST INFRASTRUCTURE ONLY.

* Line to polynomial (section 5.1.1): inside a cell with centre c the local Taylor
  polynomial restricted to the ray d + r u (d = entry point - c) is a 1-D polynomial in u
  of degree <= K.
* Line integral (section 6.1.1): sum over the cells the ray crosses of the integral of that
  polynomial over the segment length s.
* Ray insertion, 'line2taylor' (section 6.2.1): the cotangent of the locals of a cell is
  gy * I_k with I_k = int_0^s (d + r u)^k / k! du.  The paper prints this insertion
  without the 1/k!; we keep 1/k! so that it is the segment integral of the same
  monomials P2M inserts (a reading of the paper, taken where its formula and its P2M
  disagree).
* Ray root (section 5.1.2): tau = frac * max of f along the clipped ray, then the first
  parameter where f - tau changes sign from - to +, cell by cell in ray order.  A root on
  a cell face belongs to the earlier cell; tangent roots are ignored; a ray with
  f - tau >= 0 at entry or without a crossing is dead.  The expansion is piecewise
  (one polynomial per cell), so f can jump across a face: when the previous segment ends
  below tau and the next starts at or above it, the crossing is the face itself and
  belongs to the earlier cell.
* Ray-root backward (section 5.2, implicit function theorem): with t_bar and n_bar the
  cotangents of the root t* and of the surface gradient grad f(q*), the cotangent of the
  finest locals is a (q* - c)^k / k! + sum_j n_bar_j d/dq_j (q* - c)^k / k! with
  a = -(t_bar + n_bar . H r) / (r . grad f).  tau is treated as a constant (like the
  paper's bias).  The theorem needs r . grad f != 0 (section 5.2 assumes the derivative
  along the ray invertible); two kinds of hit do not meet it and keep only the dipole term
  (a = 0):
    - a face crossing: t* sits on the face for every small change of the locals (the jump
      persists), so dt*/dL = 0 and only grad f(q*) at the fixed point moves;
    - a grazing root: |r . grad f| <= GRAZE_COS |r| |grad f| (the ray is tangent to the
      level set to within that cosine); the root's sensitivity is unbounded there and is
      masked rather than inserted.
  ray_root reports the kind of each hit (ROOT_SMOOTH, ROOT_FACE, ROOT_GRAZING).

Segments come from exact FP64 intersection with every grid plane (no incremental
traversal): the crossing parameters are sorted and each segment is assigned the cell
containing its midpoint.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np
from numpy.polynomial import polynomial as npoly
from scipy import optimize

from . import fmm
from .direct import clip_ray

ROOT_SMOOTH, ROOT_FACE, ROOT_GRAZING = 0, 1, 2
GRAZE_COS = 1e-4      # cosine between the ray and grad f(q*) below which a root is grazing


def segments(geo: fmm.Geometry, o, r, t0: float, t1: float):
    """[(cell tuple, ta, tb)] in ray order for o + t r, t in [t0, t1], clipped to the grid."""
    o = np.asarray(o, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    ta, tb = clip_ray(o, r, t0, t1, geo.lo, geo.hi)
    if not tb > ta:
        return []
    h = geo.h(0)
    ts = [ta, tb]
    for j in range(geo.dim):
        if r[j] == 0.0:
            continue
        for k in range(geo.n + 1):
            t = (geo.lo + k * h - o[j]) / r[j]
            if ta < t < tb:
                ts.append(t)
    ts.sort()
    out = []
    for a, b in zip(ts[:-1], ts[1:]):
        if not b > a:
            continue
        mid = o + 0.5 * (a + b) * r
        cell = tuple(int(v) for v in np.clip(np.floor((mid - geo.lo) / h), 0, geo.n - 1))
        out.append((cell, a, b))
    return out


def _factor_poly(dj: float, rj: float, kj: int) -> np.ndarray:
    """(dj + rj u)^kj / kj! as coefficients in u (low to high)."""
    c = np.array([1.0])
    for _ in range(kj):
        c = npoly.polymul(c, [dj, rj])
    return c / math.factorial(kj)


def monomial_polys(idx, d, r) -> List[np.ndarray]:
    """For every multi-index k: (d + r u)^k / k! as a polynomial in u."""
    out = []
    for k in idx:
        c = np.array([1.0])
        for j in range(len(k)):
            c = npoly.polymul(c, _factor_poly(d[j], r[j], k[j]))
        out.append(c)
    return out


def line2poly(idx, Lrow, d, r) -> np.ndarray:
    """f(d + r u) = sum_k L[k] (d + r u)^k / k! as coefficients a_0..a_K in u."""
    K = max(sum(k) for k in idx)
    a = np.zeros(K + 1)
    for c, poly in zip(Lrow, monomial_polys(idx, d, r)):
        a[:len(poly)] += c * poly
    return a


def line2taylor(idx, d, r, s: float) -> np.ndarray:
    """I_k = int_0^s (d + r u)^k / k! du for every multi-index k."""
    out = np.empty(len(idx))
    for i, poly in enumerate(monomial_polys(idx, d, r)):
        out[i] = npoly.polyval(s, npoly.polyint(poly))
    return out


def _seg_local(geo, cell, o, r, ta):
    c = geo.centre(0, np.asarray(cell))
    return np.asarray(o, dtype=np.float64) + ta * np.asarray(r, dtype=np.float64) - c


def ray_integral(geo: fmm.Geometry, L0: np.ndarray, o, r, t0, t1) -> np.ndarray:
    """y[R, C] = sum over segments of int_0^s f_cell(d + r u) du."""
    C = L0.shape[0]
    y = np.zeros((len(o), C))
    for ri in range(len(o)):
        for cell, ta, tb in segments(geo, o[ri], r[ri], t0, t1):
            d = _seg_local(geo, cell, o[ri], r[ri], ta)
            I = line2taylor(geo.idx, d, r[ri], tb - ta)
            y[ri] += L0[(slice(None),) + cell + (slice(None),)] @ I
    return y


def ray_integral_T(geo: fmm.Geometry, o, r, t0, t1, gy, C: int) -> np.ndarray:
    """Cotangent of L0 from ray cotangents gy [R, C]: G_L0[cell] += gy_r I(d, r, s)."""
    gy = np.asarray(gy, dtype=np.float64).reshape(len(o), -1)
    G = np.zeros((C,) + (geo.n,) * geo.dim + (geo.P,))
    for ri in range(len(o)):
        for cell, ta, tb in segments(geo, o[ri], r[ri], t0, t1):
            d = _seg_local(geo, cell, o[ri], r[ri], ta)
            I = line2taylor(geo.idx, d, r[ri], tb - ta)
            G[(slice(None),) + cell + (slice(None),)] += gy[ri][:, None] * I[None, :]
    return G


# ----------------------------------------------------------------------------- roots

def _trim(c: np.ndarray) -> np.ndarray:
    c = np.asarray(c, dtype=np.float64)
    nz = np.nonzero(c)[0]
    return c[:nz[-1] + 1] if len(nz) else np.zeros(1)


def real_roots(c, lo: float, hi: float) -> List[float]:
    """Sign-changing real roots of the polynomial c (low to high) on [lo, hi]: the roots of
    the derivative split the interval into monotone pieces, each holding at most one root,
    found by brentq when the piece's end values differ in sign."""
    c = _trim(c)
    deg = len(c) - 1
    if deg <= 0:
        return []
    if deg == 1:
        x = -c[0] / c[1]
        return [x] if lo <= x <= hi else []
    crit = real_roots(npoly.polyder(c), lo, hi)
    pts = [lo] + sorted(x for x in crit if lo < x < hi) + [hi]
    out = []
    for a, b in zip(pts[:-1], pts[1:]):
        fa, fb = npoly.polyval(a, c), npoly.polyval(b, c)
        if fa == 0.0:
            out.append(a)
        elif fa * fb < 0.0:
            out.append(optimize.brentq(lambda x: npoly.polyval(x, c), a, b,
                                       xtol=1e-16, rtol=1e-15, maxiter=500))
    if npoly.polyval(hi, c) == 0.0:
        out.append(hi)
    return sorted(set(out))


def _monotone_pieces(c, s):
    crit = real_roots(npoly.polyder(_trim(c)), 0.0, s) if len(_trim(c)) > 2 else []
    pts = [0.0] + sorted(x for x in crit if 0.0 < x < s) + [s]
    return list(zip(pts[:-1], pts[1:]))


def segment_max(c, s: float) -> float:
    """max of the polynomial c over [0, s] (end points and interior critical points)."""
    cand = [0.0, s] + [x for x in (real_roots(npoly.polyder(_trim(c)), 0.0, s) if len(_trim(c)) > 1 else [])]
    return max(npoly.polyval(x, c) for x in cand)


def first_upward_root(c, s: float):
    """First u in (0, s] where the polynomial goes from < 0 to >= 0, or None."""
    c = _trim(c)
    for a, b in _monotone_pieces(c, s):
        fa, fb = npoly.polyval(a, c), npoly.polyval(b, c)
        if fa < 0.0 <= fb:
            if fb == 0.0:
                return b
            return optimize.brentq(lambda x: npoly.polyval(x, c), a, b,
                                   xtol=1e-16, rtol=1e-15, maxiter=500)
    return None


def ray_root(geo: fmm.Geometry, L0: np.ndarray, o, r, t0, t1, frac: float = 0.5,
             tau_override=None) -> dict:
    """Per ray: t* (nan if dead), hit, tau, the root's cell, grad f(q*), H(q*) and the kind
    of the hit (ROOT_SMOOTH, ROOT_FACE or ROOT_GRAZING; 0 for dead rays).  L0 has one
    channel."""
    R = len(o)
    res = {
        "t": np.full(R, np.nan), "hit": np.zeros(R, dtype=np.int32), "tau": np.zeros(R),
        "cell": np.zeros((R, geo.dim), dtype=np.int64), "normal": np.zeros((R, geo.dim)),
        "hess": np.zeros((R, geo.dim, geo.dim)), "kind": np.zeros(R, dtype=np.int32),
    }
    for ri in range(R):
        segs = segments(geo, o[ri], r[ri], t0, t1)
        if not segs:
            continue
        polys = []
        for cell, ta, tb in segs:
            d = _seg_local(geo, cell, o[ri], r[ri], ta)
            polys.append(line2poly(geo.idx, L0[(0,) + cell], d, r[ri]))
        fmax = max(segment_max(c, tb - ta) for c, (_, ta, tb) in zip(polys, segs))
        tau = frac * fmax if tau_override is None else float(tau_override[ri])
        res["tau"][ri] = tau
        if npoly.polyval(0.0, polys[0]) - tau >= 0.0:
            continue
        prev = None                       # (end value, cell, tb) of the previous segment
        for c, (cell, ta, tb) in zip(polys, segs):
            g = c.copy()
            g[0] -= tau
            if prev is not None and prev[0] < 0.0 <= npoly.polyval(0.0, g):
                # the crossing happens across the face: it lies on the face, earlier cell
                t, rcell, kind = prev[2], prev[1], ROOT_FACE
            else:
                u = first_upward_root(g, tb - ta)
                if u is None:
                    prev = (npoly.polyval(tb - ta, g), cell, tb)
                    continue
                t, rcell, kind = ta + u, cell, ROOT_SMOOTH
            q = np.asarray(o[ri], dtype=np.float64) + t * np.asarray(r[ri], dtype=np.float64)
            dq = q - geo.centre(0, np.asarray(rcell))
            row = L0[(0,) + rcell]
            res["t"][ri] = t
            res["hit"][ri] = 1
            res["cell"][ri] = rcell
            grad = row @ fmm.monomial_grads(dq[None], geo.idx)[0]
            rr = np.asarray(r[ri], dtype=np.float64)
            if kind == ROOT_SMOOTH and abs(rr @ grad) <= GRAZE_COS * np.linalg.norm(rr) * np.linalg.norm(grad):
                kind = ROOT_GRAZING
            res["normal"][ri] = grad
            res["hess"][ri] = np.einsum("p,pab->ab", row,
                                        fmm.monomial_hessians(dq[None], geo.idx)[0])
            res["kind"][ri] = kind
            break
    return res


def ray_root_T(geo: fmm.Geometry, o, r, root: dict, gt, gn) -> np.ndarray:
    """Cotangent of L0 (one channel) from root cotangents (implicit function theorem).
    Face crossings and grazing roots insert only the dipole term (module docstring)."""
    G = np.zeros((1,) + (geo.n,) * geo.dim + (geo.P,))
    R = len(o)
    gt = np.zeros(R) if gt is None else np.asarray(gt, dtype=np.float64)
    gn = np.zeros((R, geo.dim)) if gn is None else np.asarray(gn, dtype=np.float64)
    for ri in range(R):
        if not root["hit"][ri]:
            continue
        rr = np.asarray(r[ri], dtype=np.float64)
        q = np.asarray(o[ri], dtype=np.float64) + root["t"][ri] * rr
        cell = tuple(int(v) for v in root["cell"][ri])
        dq = q - geo.centre(0, np.asarray(cell))
        mgrad = fmm.monomial_grads(dq[None], geo.idx)[0]
        G[(0,) + cell] += mgrad @ gn[ri]
        if root["kind"][ri] == ROOT_SMOOTH:
            denom = rr @ root["normal"][ri]
            a = -(gt[ri] + gn[ri] @ root["hess"][ri] @ rr) / denom
            G[(0,) + cell] += a * fmm.monomials(dq[None], geo.idx)[0]
    return G

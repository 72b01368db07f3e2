"""Exact O(NM) sums in FP64 -- TEST INFRASTRUCTURE ONLY.

The quantity the method approximates (section 3, eq. (1)): y_m = sum_n psi(q_m - p_n) w_n,
and the explicit layer's vector-Jacobian products (section 4.1):
  q_bar_m = gy_m . sum_n w_n grad psi(q_m - p_n)
  w_bar_n = sum_m gy_m psi(q_m - p_n)
  p_bar_n = -sum_m gy_m . w_n grad psi(q_m - p_n)
(the paper writes the p and q cotangents through a symmetric phi; this is the same thing
for an even psi).

Also the line integral of section 6.1 (closed form for the Gaussian) and the first level
crossing along a ray of section 5 (dense sampling plus Brent's method).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
from scipy import optimize, special

from .kernels import Gaussian, Kernel


def _threads() -> int:
    return max(1, os.cpu_count() or 1)


def _chunks(total: int, size: int):
    return [(s, min(total, s + size)) for s in range(0, total, size)]


def explicit_y(kernel: Kernel, p, w, q, chunk: int = 256, threads: int | None = None):
    """y[m, c] = sum_n psi(q_m - p_n) w[n, c], chunked over queries on a thread pool."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64).reshape(len(p), -1)
    out = np.zeros((len(q), w.shape[1]))

    def work(rng):
        a, b = rng
        k = kernel.value(q[a:b, None, :] - p[None, :, :])         # [m, N]
        out[a:b] = k @ w

    with ThreadPoolExecutor(threads or _threads()) as ex:
        list(ex.map(work, _chunks(len(q), chunk)))
    return out


def explicit_grads(kernel: Kernel, p, w, q, gy, chunk: int = 256, threads: int | None = None):
    """(w_bar [N, C], p_bar [N, d], q_bar [M, d]) of L = sum gy * y."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64).reshape(len(p), -1)
    gy = np.asarray(gy, dtype=np.float64).reshape(len(q), -1)
    gq = np.zeros(q.shape)
    gw_parts, gp_parts = [], []

    def work(rng):
        a, b = rng
        x = q[a:b, None, :] - p[None, :, :]                       # [m, N, d]
        k = kernel.value(x)                                       # [m, N]
        g = kernel.grad(x)                                        # [m, N, d]
        gq[a:b] = np.einsum("mc,nc,mnj->mj", gy[a:b], w, g)
        gw = k.T @ gy[a:b]                                        # [N, C]
        gp = -np.einsum("mc,nc,mnj->nj", gy[a:b], w, g)
        return gw, gp

    with ThreadPoolExecutor(threads or _threads()) as ex:
        parts = list(ex.map(work, _chunks(len(q), chunk)))
    gw = sum(pp[0] for pp in parts)
    gp = sum(pp[1] for pp in parts)
    return gw, gp, gq


def clip_ray(o, r, t0, t1, lo, hi):
    """Parameter interval of o + t r inside [lo, hi]^3 intersected with [t0, t1] (slab
    method, FP64).  Returns (ta, tb) with ta >= tb meaning empty."""
    ta, tb = float(t0), float(t1)
    for j in range(len(o)):
        if r[j] == 0.0:
            if not (lo <= o[j] <= hi):
                return 0.0, 0.0
            continue
        a = (lo - o[j]) / r[j]
        b = (hi - o[j]) / r[j]
        ta = max(ta, min(a, b))
        tb = min(tb, max(a, b))
    return ta, tb


def ray_integral_gaussian(sigma: float, p, w, o, r, ta: float, tb: float):
    """int_ta^tb sum_n w_n exp(-|o + t r - p_n|^2 / (2 sigma^2)) dt for a unit r, closed
    form: with a = (p - o).r and d_perp^2 = |p - o|^2 - a^2,
    sigma sqrt(pi/2) exp(-d_perp^2 / 2 sigma^2) [erf((tb - a)/(sqrt2 sigma)) - erf((ta - a)/(sqrt2 sigma))]."""
    p = np.asarray(p, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64).reshape(len(p), -1)
    o = np.asarray(o, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    v = p - o
    a = v @ r
    dperp2 = np.maximum(np.sum(v * v, axis=1) - a * a, 0.0)
    s2 = math.sqrt(2.0) * sigma
    per = sigma * math.sqrt(math.pi / 2.0) * np.exp(-dperp2 / (2 * sigma * sigma)) * \
        (special.erf((tb - a) / s2) - special.erf((ta - a) / s2))
    return per @ w


def field_along_ray(kernel: Kernel, p, w, o, r, t: np.ndarray):
    """f(o + t r) for an array of t (single channel)."""
    x = np.asarray(o)[None, :] + np.asarray(t)[:, None] * np.asarray(r)[None, :]
    return explicit_y(kernel, p, w, x, threads=1)[:, 0]


def ray_root(kernel: Kernel, p, w, o, r, ta: float, tb: float, dt: float, frac: float = 0.5):
    """First upward crossing of f - tau on [ta, tb], tau = frac * max f along the segment.
    f is sampled every dt, the maximum refined with a bounded scalar minimisation around the
    best sample, and the crossing bracketed on the samples then solved by brentq.
    Returns (t_star or nan, tau)."""
    n = max(2, int(math.ceil((tb - ta) / dt)) + 1)
    ts = np.linspace(ta, tb, n)
    fs = field_along_ray(kernel, p, w, o, r, ts)
    i = int(np.argmax(fs))
    a, b = ts[max(i - 1, 0)], ts[min(i + 1, n - 1)]
    f1 = lambda t: -field_along_ray(kernel, p, w, o, r, np.array([t]))[0]
    res = optimize.minimize_scalar(f1, bounds=(a, b), method="bounded",
                                   options={"xatol": 1e-13})
    fmax = max(fs[i], -res.fun)
    tau = frac * fmax
    g = fs - tau
    for j in range(n - 1):
        if g[j] < 0.0 <= g[j + 1]:
            fr = lambda t: field_along_ray(kernel, p, w, o, r, np.array([t]))[0] - tau
            return optimize.brentq(fr, ts[j], ts[j + 1], xtol=1e-15, rtol=1e-15), tau
    return float("nan"), tau

"""Shared test helpers: oracle set-up for a workload and comparisons."""
import math

import numpy as np

from oracle import fmm, kernels
from paper_2111_00110_amd import workloads as W


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def oracle_geometry(wl: W.Workload) -> fmm.Geometry:
    return fmm.Geometry(wl.dim, wl.n, wl.lo, wl.hi, wl.K,
                        np.float32 if wl.io == "f32" else np.float64)


def oracle_kernel(wl: W.Workload, coef=None):
    if wl.kernel == "poly":
        return kernels.Polynomial(coef, wl.dim)
    return kernels.make_kernel(wl.kernel, wl.param, wl.dim)


def scaled_locals(geo: fmm.Geometry, L0: np.ndarray, P_pad: int) -> np.ndarray:
    """Physical oracle locals (C, n, ..., n, P) -> the library's layout [C][n^d][P_pad] in
    cell-scaled units h^|k| d^k f."""
    C = L0.shape[0]
    scale = np.array([geo.h(0) ** sum(k) for k in geo.idx])
    flat = L0.reshape(C, -1, geo.P) * scale
    out = np.zeros((C, flat.shape[1], P_pad))
    out[:, :, :geo.P] = flat
    return out


def poly_coef_list(kernel: kernels.Polynomial, dim: int, deg: int):
    """Coefficient list in the graded multi-index order of degree <= deg."""
    return [kernel.coef.get(a, 0.0) for a in fmm.multi_indices(dim, deg)]


def physical_locals(geo: fmm.Geometry, Lt: np.ndarray) -> np.ndarray:
    """The library's scaled layout [C][n^d][P_pad] -> physical (C, n, ..., n, P)."""
    C = Lt.shape[0]
    scale = np.array([geo.h(0) ** sum(k) for k in geo.idx])
    out = np.asarray(Lt, dtype=np.float64)[:, :, :geo.P] / scale
    return out.reshape((C,) + (geo.n,) * geo.dim + (geo.P,))


def scaled_cotangent(geo: fmm.Geometry, G: np.ndarray, P_pad: int) -> np.ndarray:
    """Cotangent of physical locals -> cotangent of the scaled locals h^|k| L[k]."""
    C = G.shape[0]
    scale = np.array([geo.h(0) ** sum(k) for k in geo.idx])
    flat = G.reshape(C, -1, geo.P) / scale
    out = np.zeros((C, flat.shape[1], P_pad))
    out[:, :, :geo.P] = flat
    return out


def rays_toward_origin(rng, R, jitter=0.1):
    """Origins on the radius-2 sphere aimed at the origin with a uniform aim jitter."""
    v = rng.standard_normal((R, 3))
    o = 2.0 * v / np.linalg.norm(v, axis=1, keepdims=True)
    r = -o + rng.uniform(-jitter, jitter, (R, 3))
    return o, r / np.linalg.norm(r, axis=1, keepdims=True)

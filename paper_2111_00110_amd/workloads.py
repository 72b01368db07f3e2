"""Seeded synthetic workloads for the FC^2T^2 explicit, ray-integral and ray-root layers.

This module only draws random inputs.  It holds none of the method's arithmetic, so the
GPU path and the FP64 CPU checker can both consume the same arrays.

Six workloads mirror the paper's shapes (section 3.3 benchmarks; section 4.3 SDF fitting
with N = 8 m sources and M = 10 m targets; sections 5-6 rays through a level-6 grid; the
volumetric layer's experiment with a level-6 expansion, 8 m sources and 100,000 rays per
iteration):

  explicit2d_small   2-D, N = M = 4096, Gaussian sigma = 0.05, 16^2 grid, K = 4, FP64
  explicit2d         2-D, N = M = 2^20, Gaussian sigma = 0.01, 256^2 grid, K = 6, FP32
  explicit3d_imq     3-D shell sources N = 2^21, M = 10^7 uniform queries,
                     inverse multiquadric eps = 0.02, 64^3 grid, K = 4
  ray_integral3d     3-D shell sources N = 2^22, 65,536 rays, Gaussian sigma = 0.02,
                     128^3 grid, K = 4
  ray_root3d         3-D shell sources N = 2^23, 65,536 rays, Gaussian sigma = 0.015,
                     128^3 grid, K = 5
  volume3d           3-D shell sources N = 2^23 with four channels (density, R, G, B),
                     100,000 rays aimed at uniform points of [-0.6, 0.6]^3 (camera rays over
                     the object and around it), Gaussian sigma = 0.02, 64^3 grid, K = 4;
                     density weights 0.009 |N(0, 1)| (non-negative, as the paper keeps them):
                     a ray through both walls of the shell, or along one, ends in the medium,
                     one that misses it reaches the background

Draw order with numpy's PCG64 (default_rng(seed)), all in FP64, then one cast to the
workload's IO precision: sources, weights, queries (or ray origins, then aim points),
source jitter, cotangents.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    n: int                  # finest cells per dimension (a power of two >= 4)
    lo: float               # domain is [lo, hi]^dim
    hi: float
    K: int                  # Taylor order (the paper's rho)
    kernel: str             # "gaussian" | "imq"
    param: float            # sigma for the Gaussian, eps for the IMQ
    N: int                  # sources
    M: int                  # queries (explicit layer)
    R: int                  # rays (ray layers)
    io: str                 # "f32" | "f64"
    layer: str              # "explicit" | "ray_integral" | "ray_root" | "volume"
    sources: str            # "uniform" | "shell"
    t0: float = 0.0         # ray parameter range
    t1: float = 4.0
    dens: float = 1.0       # volume: density weights are dens * |N(0, 1)|
    aim: float = 0.1        # rays aim at uniform points of [-aim, aim]^3


WORKLOADS = {
    "explicit2d_small": Workload("explicit2d_small", 2, 16, 0.0, 1.0, 4, "gaussian", 0.05,
                                 4096, 4096, 0, "f64", "explicit", "uniform"),
    "explicit2d": Workload("explicit2d", 2, 256, 0.0, 1.0, 6, "gaussian", 0.01,
                           1 << 20, 1 << 20, 0, "f32", "explicit", "uniform"),
    "explicit3d_imq": Workload("explicit3d_imq", 3, 64, -1.0, 1.0, 4, "imq", 0.02,
                               1 << 21, 10_000_000, 0, "f32", "explicit", "shell"),
    "ray_integral3d": Workload("ray_integral3d", 3, 128, -1.0, 1.0, 4, "gaussian", 0.02,
                               1 << 22, 0, 65536, "f32", "ray_integral", "shell"),
    "ray_root3d": Workload("ray_root3d", 3, 128, -1.0, 1.0, 5, "gaussian", 0.015,
                           1 << 23, 0, 65536, "f32", "ray_root", "shell"),
    "volume3d": Workload("volume3d", 3, 64, -1.0, 1.0, 4, "gaussian", 0.02,
                         1 << 23, 0, 100_000, "f32", "volume", "shell", dens=0.009, aim=0.6),
}


def workload(name: str, **overrides) -> Workload:
    """A named workload, optionally with some fields replaced (e.g. smaller N for tests)."""
    return dataclasses.replace(WORKLOADS[name], **overrides)


def _shell(rng: np.random.Generator, count: int) -> np.ndarray:
    # Direction uniform on the sphere, radius 0.5; the isotropic N(0, 0.01^2) jitter is
    # drawn later in the documented order and added by the caller.
    u = rng.standard_normal((count, 3))
    return 0.5 * u / np.linalg.norm(u, axis=1, keepdims=True)


def make(wl: Workload, seed: int = 0, channels: int = 1) -> dict:
    """Draw the inputs of one workload.

    Returns a dict of numpy arrays in the workload's IO precision:
      p [N, d], w [N, C]; explicit: q [M, d], gy [M, C];
      ray_integral: o [R, 3], r [R, 3], gy [R, C];
      ray_root: o, r, gt [R], gn [R, 3];
      volume: w [N, 4] (density, R, G, B; the density column dens * |N(0, 1)|), o, r,
              gy [R, 3], bg [3] (the background colour, fixed).
    """
    rng = np.random.default_rng(seed)
    d = wl.dim
    out: dict = {}
    if wl.sources == "uniform":
        p = rng.uniform(wl.lo, wl.hi, size=(wl.N, d))
    else:
        p = _shell(rng, wl.N)
    if wl.layer == "volume":
        channels = 4
    w = rng.standard_normal((wl.N, channels))
    if wl.layer == "volume":
        w[:, 0] = wl.dens * np.abs(w[:, 0])
    if wl.layer == "explicit":
        out["q"] = rng.uniform(wl.lo, wl.hi, size=(wl.M, d))
    else:
        v = rng.standard_normal((wl.R, 3))
        o = 2.0 * v / np.linalg.norm(v, axis=1, keepdims=True)
        aim = rng.uniform(-wl.aim, wl.aim, size=(wl.R, 3))
        r = -o + aim
        r = r / np.linalg.norm(r, axis=1, keepdims=True)
        out["o"] = o
        out["r"] = r
    if wl.sources == "shell":
        p = p + 0.01 * rng.standard_normal((wl.N, 3))
    out["p"] = p
    out["w"] = w
    if wl.layer == "explicit":
        out["gy"] = rng.standard_normal((wl.M, channels))
    elif wl.layer == "ray_integral":
        out["gy"] = rng.standard_normal((wl.R, channels))
    elif wl.layer == "volume":
        out["gy"] = rng.standard_normal((wl.R, 3))
        out["bg"] = np.array([0.2, 0.4, 0.6])
    else:
        out["gt"] = rng.standard_normal(wl.R)
        out["gn"] = rng.standard_normal((wl.R, 3))
    dt = np.float32 if wl.io == "f32" else np.float64
    return {k: np.ascontiguousarray(v.astype(dt)) for k, v in out.items()}


def subsample(rng_seed: int, count: int, size: int) -> np.ndarray:
    """Sorted distinct indices of a seeded subsample (for spot checks at full size)."""
    rng = np.random.default_rng(rng_seed)
    count = min(count, size)
    return np.sort(rng.choice(size, size=count, replace=False))


__all__ = ["Workload", "WORKLOADS", "workload", "make", "subsample"]

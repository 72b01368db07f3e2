"""Kernels psi(x) and their partial derivatives, FP64 (checker only).

The method needs a translation-invariant kernel phi(q, p) = psi(q - p) whose radius of
convergence grows with distance (section 3, derivation before eq. (2)).  The M2L tensor
holds the partial derivatives d^(k+n) psi at cell-centre offsets (section 3, the
K^{M2L} definition), so we need every partial derivative up to total order 2K.

* Gaussian psi(x) = exp(-|x|^2 / (2 sigma^2)) = prod_j exp(-x_j^2 / (2 sigma^2)); each
  1-D factor has the closed form d^m/dx^m exp(-x^2/(2 s^2)) = (-1/s)^m He_m(x/s) exp(..)
  with He_m the probabilists' Hermite polynomial (recurrence He_{m+1} = x He_m - m He_{m-1}).
* Inverse multiquadric psi(x) = (|x|^2 + eps^2)^(-1/2): sympy.diff of the symbolic
  expression, lambdified to numpy.
* Polynomial psi(x) = sum_a c_a x^a: d^g x^a = a!/(a-g)! x^(a-g) for a >= g.
"""
from __future__ import annotations

import functools
import math
from typing import Dict, Sequence, Tuple

import numpy as np

MultiIndex = Tuple[int, ...]


class Kernel:
    """psi, grad psi and all partial derivatives of psi up to a given order."""

    name = "kernel"
    even = True

    def value(self, x: np.ndarray) -> np.ndarray:        # x [..., d] -> [...]
        raise NotImplementedError

    def grad(self, x: np.ndarray) -> np.ndarray:         # -> [..., d]
        raise NotImplementedError

    def derivs(self, x: np.ndarray, gammas: Sequence[MultiIndex]) -> np.ndarray:
        """d^gamma psi(x) for each gamma: x [..., d] -> [..., len(gammas)]."""
        raise NotImplementedError


def hermite_prob(m: int, x: np.ndarray) -> np.ndarray:
    """Probabilists' Hermite polynomial He_m(x) by its three-term recurrence."""
    h0 = np.ones_like(x)
    if m == 0:
        return h0
    h1 = x.copy()
    for j in range(1, m):
        h0, h1 = h1, x * h1 - j * h0
    return h1


class Gaussian(Kernel):
    name = "gaussian"

    def __init__(self, sigma: float):
        self.sigma = float(sigma)

    def value(self, x):
        return np.exp(-np.sum(x * x, axis=-1) / (2.0 * self.sigma ** 2))

    def grad(self, x):
        return -x / self.sigma ** 2 * self.value(x)[..., None]

    def _d1(self, m: int, x: np.ndarray) -> np.ndarray:
        s = self.sigma
        return (-1.0 / s) ** m * hermite_prob(m, x / s) * np.exp(-x * x / (2 * s * s))

    def derivs(self, x, gammas):
        x = np.asarray(x, dtype=np.float64)
        out = np.empty(x.shape[:-1] + (len(gammas),))
        cache: Dict[Tuple[int, int], np.ndarray] = {}
        for gi, g in enumerate(gammas):
            acc = np.ones(x.shape[:-1])
            for j, m in enumerate(g):
                key = (j, m)
                if key not in cache:
                    cache[key] = self._d1(m, x[..., j])
                acc = acc * cache[key]
            out[..., gi] = acc
        return out


class IMQ(Kernel):
    name = "imq"

    def __init__(self, eps: float, dim: int):
        self.eps = float(eps)
        self.dim = dim

    def value(self, x):
        return 1.0 / np.sqrt(np.sum(x * x, axis=-1) + self.eps ** 2)

    def grad(self, x):
        r2 = np.sum(x * x, axis=-1) + self.eps ** 2
        return -x * (r2 ** -1.5)[..., None]

    @functools.lru_cache(maxsize=None)
    def _lambdified(self, g: MultiIndex):
        import sympy as sp
        xs = sp.symbols("x0:%d" % self.dim, real=True)
        expr = (sum(v * v for v in xs) + sp.Float(self.eps, 30) ** 2) ** sp.Rational(-1, 2)
        for j, m in enumerate(g):
            if m:
                expr = sp.diff(expr, xs[j], m)
        return sp.lambdify(xs, expr, "numpy")

    def derivs(self, x, gammas):
        x = np.asarray(x, dtype=np.float64)
        out = np.empty(x.shape[:-1] + (len(gammas),))
        cols = [x[..., j] for j in range(self.dim)]
        for gi, g in enumerate(gammas):
            out[..., gi] = self._lambdified(tuple(g))(*cols)
        return out


class Polynomial(Kernel):
    """psi(x) = sum_a coef[a] x^a (test kernel; not even unless its odd terms vanish)."""

    name = "poly"

    def __init__(self, coef: Dict[MultiIndex, float], dim: int):
        self.coef = {tuple(a): float(c) for a, c in coef.items()}
        self.dim = dim
        self.even = all(sum(a) % 2 == 0 for a, c in self.coef.items() if c != 0.0)

    def _deriv_one(self, x, g):
        acc = np.zeros(x.shape[:-1])
        for a, c in self.coef.items():
            if any(ai < gi for ai, gi in zip(a, g)):
                continue
            term = np.full(x.shape[:-1], c)
            for j, (ai, gi) in enumerate(zip(a, g)):
                term = term * (math.factorial(ai) / math.factorial(ai - gi)) * x[..., j] ** (ai - gi)
            acc = acc + term
        return acc

    def value(self, x):
        return self._deriv_one(np.asarray(x, dtype=np.float64), (0,) * self.dim)

    def grad(self, x):
        x = np.asarray(x, dtype=np.float64)
        cols = []
        for j in range(self.dim):
            g = [0] * self.dim
            g[j] = 1
            cols.append(self._deriv_one(x, tuple(g)))
        return np.stack(cols, axis=-1)

    def derivs(self, x, gammas):
        x = np.asarray(x, dtype=np.float64)
        return np.stack([self._deriv_one(x, tuple(g)) for g in gammas], axis=-1)


def make_kernel(kind: str, param, dim: int) -> Kernel:
    if kind == "gaussian":
        return Gaussian(param)
    if kind == "imq":
        return IMQ(param, dim)
    if kind == "poly":
        return Polynomial(param, dim)
    raise ValueError(kind)

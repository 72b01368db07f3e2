"""The FC^2T^2 expansion, step by step, in FP64 numpy -- TEST INFRASTRUCTURE ONLY.

Follows section 3 of the paper (derivation of eq. (2), the single-level algorithm, the
multilevel M2M / L2L shifts, the M2L convolution with its parity window and near-field
hole) and section 4.1 (the explicit layer's vector-Jacobian products), in physical units.

Readings taken where the paper is silent or inconsistent (each one stated here):

* Sign (section 3 derivation): phi(q, p) = psi(q - p).  With moments
  M[n] = sum w (p - c_p)^n / n! and locals L[k] = d^k f(c_q), the M2L tensor is
  T[k, n] = (-1)^|n| d^(k+n) psi(c_q - c_p).
* Truncation: the square set |k| <= K, |n| <= K (the paper's P x P kernel and its
  35^2 * 6^3 * 2 flop count), so derivatives up to order 2K are used.  ``triangular=True``
  selects |k| + |n| <= K instead.
* Levels: the finest grid has n = 2^(levels+1) cells per dimension and the coarsest 4.
  Target cell i receives source cell j at level l iff their parents are equal or
  adjacent and (l is the finest level or i and j are not adjacent); adjacency is
  Chebyshev distance <= 1.  Per dimension this is the window j - i in [-2, 3] for an even
  index of i and [-3, 2] for an odd one, with the hole [-1, 1]^d removed above the
  finest level.  At the coarsest level (4 cells) the window covers the whole grid.
* The L2P loop bound is |k| <= K and M2L accumulates (the printed pseudo-code has '<'
  and '=').
* Cell index: i = clamp(floor((x - lo) * (n / (hi - lo))), 0, n - 1) evaluated in the IO
  precision with one rounding per operation, so points on or near a face land in the same
  cell on every implementation.
* Least-squares tensors (section 3.1, ``Geometry.fit = "lsq"``): the paper fits polynomials
  to the kernel and its derivatives for a given radius and order without saying over what
  region or with which samples.  Reading: for each k, T[k, :] are the coefficients of the
  polynomial sum_{|n| <= K} c_n x^n / n! closest in L2 over the source cell
  (x in [-h/2, h/2]^d) to d^k psi(delta - x); the integral is taken by tensor
  Gauss-Legendre quadrature with K + 2 nodes per dimension.  Parity unpinned against the
  paper (it gives no numbers); pinned by exactness on polynomial kernels.

Arrays: a grid quantity at level l has shape (C, n_l, ..., n_l, P) with dimension 0 the
slowest; P = C(K + d, d) multi-indices in graded order (total degree, then the first
component descending).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

from .kernels import Kernel

MultiIndex = Tuple[int, ...]


# ----------------------------------------------------------------------------- indices

def _compositions(total: int, d: int) -> List[MultiIndex]:
    if d == 1:
        return [(total,)]
    out = []
    for a in range(total, -1, -1):
        for rest in _compositions(total - a, d - 1):
            out.append((a,) + rest)
    return out


def multi_indices(d: int, K: int) -> List[MultiIndex]:
    """All n in N^d with |n| <= K in graded order (section 3: 'arbitrary but consistent')."""
    out: List[MultiIndex] = []
    for t in range(K + 1):
        out.extend(_compositions(t, d))
    return out


def ifact(a: MultiIndex) -> float:
    return float(np.prod([math.factorial(v) for v in a]))


# ----------------------------------------------------------------------------- geometry

@dataclass
class Geometry:
    dim: int
    n: int            # finest cells per dimension
    lo: float
    hi: float
    K: int
    io: type = np.float64   # precision in which cell indices are computed
    fit: str = "taylor"     # M2L tensor: "taylor" (derivatives) or "lsq" (section 3.1 fit)

    def __post_init__(self):
        if self.n < 4 or (self.n & (self.n - 1)):
            raise ValueError("n must be a power of two >= 4")
        self.levels = int(round(math.log2(self.n))) - 1
        self.idx = multi_indices(self.dim, self.K)
        self.P = len(self.idx)

    def cells(self, level: int) -> int:
        return self.n >> level

    def h(self, level: int) -> float:
        return (self.hi - self.lo) * (1 << level) / self.n

    def centre(self, level: int, i: np.ndarray) -> np.ndarray:
        """Centre of cell with integer index i [..., d] at a level (FP64)."""
        return self.lo + (np.asarray(i, dtype=np.float64) + 0.5) * self.h(level)

    def cell_index(self, x: np.ndarray) -> np.ndarray:
        """Finest-level cell of each point x [..., d] (one rounding per operation)."""
        t = self.io
        x = np.asarray(x).astype(t)
        scale = t(self.n / (self.hi - self.lo))
        u = (x - t(self.lo)).astype(t) * scale
        i = np.floor(u.astype(t)).astype(np.int64)
        return np.clip(i, 0, self.n - 1)


# ----------------------------------------------------------------------------- monomials

def monomials(x: np.ndarray, idx: Sequence[MultiIndex]) -> np.ndarray:
    """x^n / n! for every multi-index n: x [..., d] -> [..., P]."""
    x = np.asarray(x, dtype=np.float64)
    return np.stack([np.prod([x[..., j] ** a[j] for j in range(len(a))], axis=0) / ifact(a)
                     for a in idx], axis=-1)


def monomial_grads(x: np.ndarray, idx: Sequence[MultiIndex]) -> np.ndarray:
    """d/dx_j of x^n / n!: x [..., d] -> [..., P, d]."""
    x = np.asarray(x, dtype=np.float64)
    d = x.shape[-1]
    cols = []
    for a in idx:
        per_dim = []
        for j in range(d):
            if a[j] == 0:
                per_dim.append(np.zeros(x.shape[:-1]))
                continue
            b = list(a)
            b[j] -= 1
            per_dim.append(np.prod([x[..., m] ** b[m] for m in range(d)], axis=0) / ifact(tuple(b)))
        cols.append(np.stack(per_dim, axis=-1))
    return np.stack(cols, axis=-2)


def monomial_hessians(x: np.ndarray, idx: Sequence[MultiIndex]) -> np.ndarray:
    """d^2/dx_a dx_b of x^n / n!: x [..., d] -> [..., P, d, d]."""
    x = np.asarray(x, dtype=np.float64)
    d = x.shape[-1]
    out = np.zeros(x.shape[:-1] + (len(idx), d, d))
    for pi, a in enumerate(idx):
        for ja in range(d):
            for jb in range(d):
                b = list(a)
                b[ja] -= 1
                b[jb] -= 1
                if min(b) < 0:
                    continue
                out[..., pi, ja, jb] = np.prod([x[..., m] ** b[m] for m in range(d)], axis=0) / ifact(tuple(b))
    return out


# ----------------------------------------------------------------------------- operators

def shift_matrix(e: np.ndarray, idx: Sequence[MultiIndex]) -> np.ndarray:
    """S[n, m] = e^(n - m) / (n - m)! for m <= n componentwise (section 3, M2M binomial
    shift).  M2M uses M_parent = sum_children S(c_child - c_parent) M_child, and L2L uses
    L_child = S(c_child - c_parent)^T L_parent (the Taylor shift of section 3)."""
    P = len(idx)
    S = np.zeros((P, P))
    for a, n in enumerate(idx):
        for b, m in enumerate(idx):
            if all(mm <= nn for mm, nn in zip(m, n)):
                diff = tuple(nn - mm for nn, mm in zip(n, m))
                S[a, b] = np.prod([e[j] ** diff[j] for j in range(len(n))]) / ifact(diff)
    return S


def child_offsets(d: int):
    """Child position bits b in {0,1}^d (child index = 2 * parent + b)."""
    return list(itertools.product((0, 1), repeat=d))


def _child_slice(b):
    return tuple(slice(bj, None, 2) for bj in b)


def in_window(o: Sequence[int], finest: bool) -> bool:
    """Whether offset o = j - i can occur at all (inside [-3, 3]^d and outside the hole)."""
    if finest:
        return True
    return max(abs(v) for v in o) > 1


def window_mask(n_l: int, o: Sequence[int]) -> np.ndarray:
    """Mask over target cells i of one level for source offset o (parity window and grid
    bounds, per dimension as an outer product)."""
    masks = []
    for oj in o:
        i = np.arange(n_l)
        even = (i % 2 == 0)
        ok = np.where(even, (oj >= -2) & (oj <= 3), (oj >= -3) & (oj <= 2))
        ok &= (i + oj >= 0) & (i + oj < n_l)
        masks.append(ok)
    m = masks[0]
    for mk in masks[1:]:
        m = np.multiply.outer(m, mk)
    return m


def m2l_tensor(kernel: Kernel, geo: Geometry, level: int, o: Sequence[int],
               triangular: bool = False) -> np.ndarray:
    """T[k, n] = (-1)^|n| d^(k+n) psi(c_target - c_source), with c_target - c_source =
    -o * h_level for o = j - i.  Memoised on the kernel object."""
    cache = kernel.__dict__.setdefault("_m2l_cache", {})
    key = (geo.dim, geo.n, geo.lo, geo.hi, geo.K, geo.fit, level, tuple(o), triangular)
    if key not in cache:
        if geo.fit == "lsq":
            if triangular:
                raise ValueError("the least-squares tensor uses the square set")
            cache[key] = _m2l_tensor_lsq(kernel, geo, level, o)
        else:
            cache[key] = _m2l_tensor(kernel, geo, level, o, triangular)
    return cache[key]


def _m2l_tensor(kernel, geo, level, o, triangular):
    idx = geo.idx
    delta = -np.asarray(o, dtype=np.float64) * geo.h(level)
    gammas = sorted({tuple(a + b for a, b in zip(k, n)) for k in idx for n in idx})
    D = dict(zip(gammas, kernel.derivs(delta[None, :], gammas)[0]))
    P = len(idx)
    T = np.zeros((P, P))
    for a, k in enumerate(idx):
        for b, n in enumerate(idx):
            if triangular and sum(k) + sum(n) > geo.K:
                continue
            g = tuple(x + y for x, y in zip(k, n))
            T[a, b] = (-1.0) ** sum(n) * D[g]
    return T


def lsq_nodes(geo: Geometry, level: int):
    """Tensor Gauss-Legendre nodes [J, d] and weights [J] on the source cell [-h/2, h/2]^d,
    K + 2 nodes per dimension."""
    h = geo.h(level)
    t, wq = np.polynomial.legendre.leggauss(geo.K + 2)
    X = np.array(list(itertools.product(0.5 * h * t, repeat=geo.dim)))
    W = np.prod(np.array(list(itertools.product(0.5 * h * wq, repeat=geo.dim))), axis=1)
    return X, W


def _m2l_tensor_lsq(kernel, geo, level, o):
    """Section 3.1: T[k, n] = c_n of the weighted least-squares polynomial
    sum_n c_n x^n / n! fitted to d^k psi(delta - x) over the source cell, delta = -o h."""
    X, W = lsq_nodes(geo, level)
    h = geo.h(level)
    delta = -np.asarray(o, dtype=np.float64) * h
    G = kernel.derivs(delta[None, :] - X, geo.idx)          # [J, P(k)]
    # solved in t = 2 x / h in [-1, 1] with the basis t^n (well conditioned), then
    # sum_n c_t[n] t^n = sum_n c_t[n] (2/h)^|n| n! x^n / n!
    Tn = X * (2.0 / h)
    Vt = np.stack([np.prod(Tn ** np.asarray(a, dtype=np.float64), axis=1) for a in geo.idx], axis=1)
    sw = np.sqrt(W)[:, None]
    Ct = np.linalg.lstsq(sw * Vt, sw * G, rcond=None)[0]     # [P(n), P(k)]
    scale = np.array([(2.0 / h) ** sum(a) * ifact(a) for a in geo.idx])
    return (Ct * scale[:, None]).T


def _pad3(A: np.ndarray, d: int) -> np.ndarray:
    pad = [(0, 0)] + [(3, 3)] * d + [(0, 0)]
    return np.pad(A, pad)


def _shift_view(Ap: np.ndarray, o: Sequence[int], n_l: int) -> np.ndarray:
    """View of the padded array at i + o for all i (padding of 3 cells per side)."""
    sl = (slice(None),) + tuple(slice(3 + oj, 3 + oj + n_l) for oj in o) + (slice(None),)
    return Ap[sl]


def offsets(d: int):
    return list(itertools.product(range(-3, 4), repeat=d))


# ----------------------------------------------------------------------------- forward

def p2m(geo: Geometry, p: np.ndarray, w: np.ndarray) -> np.ndarray:
    """M_0[c, n] = sum_{s in cell c} w_s (p_s - centre_c)^n / n!  (section 3, P2M)."""
    d, n = geo.dim, geo.n
    w = np.asarray(w, dtype=np.float64).reshape(len(p), -1)
    C = w.shape[1]
    M = np.zeros((C,) + (n,) * d + (geo.P,))
    for a in range(0, len(p), 1 << 20):          # chunks bound the monomial array's memory
        pc = p[a:a + (1 << 20)]
        cell = geo.cell_index(pc)
        dvec = np.asarray(pc, dtype=np.float64) - geo.centre(0, cell)
        mono = monomials(dvec, geo.idx)                               # [chunk, P]
        for ch in range(C):
            np.add.at(M[ch], tuple(cell[:, j] for j in range(d)), mono * w[a:a + (1 << 20), ch:ch + 1])
    return M


def m2m(geo: Geometry, level: int, M_child: np.ndarray) -> np.ndarray:
    """Moments one level up: M_{l+1}[I] = sum_b S(c(2I+b) - c(I)) M_l[2I+b]."""
    h = geo.h(level)
    out = 0.0
    for b in child_offsets(geo.dim):
        e = (np.asarray(b) - 0.5) * h
        S = shift_matrix(e, geo.idx)
        out = out + M_child[(slice(None),) + _child_slice(b) + (slice(None),)] @ S.T
    return out


def l2l(geo: Geometry, level: int, L_parent: np.ndarray) -> np.ndarray:
    """Parent locals re-expanded at the children of `level`:
    L_l[2I+b, k] = sum_{m >= k} e^(m-k)/(m-k)! L_{l+1}[I, m]."""
    h = geo.h(level)
    C = L_parent.shape[0]
    n_l = geo.cells(level)
    out = np.zeros((C,) + (n_l,) * geo.dim + (geo.P,))
    for b in child_offsets(geo.dim):
        e = (np.asarray(b) - 0.5) * h
        S = shift_matrix(e, geo.idx)
        out[(slice(None),) + _child_slice(b) + (slice(None),)] = L_parent @ S
    return out


def m2l(geo: Geometry, kernel: Kernel, level: int, M: np.ndarray,
        triangular: bool = False) -> np.ndarray:
    """L_l[i] = sum over admissible o of T(o) M_l[i + o]  (section 3, M2L convolution with
    the hole and the parity-dependent windows)."""
    n_l = geo.cells(level)
    finest = level == 0
    Mp = _pad3(M, geo.dim)
    L = np.zeros_like(M)
    for o in offsets(geo.dim):
        if not in_window(o, finest):
            continue
        mask = window_mask(n_l, o)
        if not mask.any():
            continue
        T = m2l_tensor(kernel, geo, level, o, triangular)
        L += mask[None, ..., None] * (_shift_view(Mp, o, n_l) @ T.T)
    return L


def expand(geo: Geometry, kernel: Kernel, p, w, triangular: bool = False,
           return_levels: bool = False):
    """P2M -> M2M (up) -> M2L (every level) -> L2L (down): finest-level locals L_0."""
    Ms = [p2m(geo, p, w)]
    for lv in range(geo.levels - 1):
        Ms.append(m2m(geo, lv, Ms[-1]))
    Ls = [m2l(geo, kernel, lv, Ms[lv], triangular) for lv in range(geo.levels)]
    acc = Ls[-1]
    for lv in range(geo.levels - 2, -1, -1):
        acc = Ls[lv] + l2l(geo, lv, acc)
    if return_levels:
        return acc, Ms, Ls
    return acc


def _gather_cells(geo: Geometry, L0: np.ndarray, x: np.ndarray):
    cell = geo.cell_index(x)
    dvec = np.asarray(x, dtype=np.float64) - geo.centre(0, cell)
    rows = L0[(slice(None),) + tuple(cell[:, j] for j in range(geo.dim))]   # [C, M, P]
    return rows, dvec


def l2p(geo: Geometry, L0: np.ndarray, q: np.ndarray):
    """f(q) = sum_k L_0[cell(q), k] (q - c)^k / k!: returns [M, C]."""
    rows, dvec = _gather_cells(geo, L0, q)
    return np.einsum("cmp,mp->mc", rows, monomials(dvec, geo.idx))


def l2p_grad(geo: Geometry, L0: np.ndarray, q: np.ndarray):
    """grad_q f: [M, C, d]."""
    rows, dvec = _gather_cells(geo, L0, q)
    return np.einsum("cmp,mpj->mcj", rows, monomial_grads(dvec, geo.idx))


def l2p_hess(geo: Geometry, L0: np.ndarray, q: np.ndarray):
    """Hessian of f: [M, C, d, d]."""
    rows, dvec = _gather_cells(geo, L0, q)
    return np.einsum("cmp,mpab->mcab", rows, monomial_hessians(dvec, geo.idx))


# ----------------------------------------------------------------------------- backward

def l2p_T(geo: Geometry, q: np.ndarray, gy: np.ndarray) -> np.ndarray:
    """Transpose of L2P: G_L0[c, k] = sum_{q in c} gy_q (q - c)^k / k!  (queries taken in
    chunks of 2^20, each chunk's per-cell sums added with bincount: the same sums, with memory
    bounded at 10^7 queries)."""
    gy = np.asarray(gy, dtype=np.float64).reshape(len(q), -1)
    C = gy.shape[1]
    G = np.zeros((C, geo.cells(0) ** geo.dim, geo.P))
    for a in range(0, len(q), 1 << 20):
        qc = q[a:a + (1 << 20)]
        cell = geo.cell_index(qc)
        lin = np.ravel_multi_index(tuple(cell[:, j] for j in range(geo.dim)), (geo.n,) * geo.dim)
        mono = monomials(np.asarray(qc, dtype=np.float64) - geo.centre(0, cell), geo.idx)
        for ch in range(C):
            wk = mono * gy[a:a + (1 << 20), ch:ch + 1]
            for k in range(geo.P):
                G[ch, :, k] += np.bincount(lin, weights=wk[:, k], minlength=G.shape[1])
    return G.reshape((C,) + (geo.n,) * geo.dim + (geo.P,))


def l2l_T(geo: Geometry, level: int, G_child: np.ndarray) -> np.ndarray:
    """Transpose of l2l(level): cotangent of the parent locals."""
    h = geo.h(level)
    out = 0.0
    for b in child_offsets(geo.dim):
        e = (np.asarray(b) - 0.5) * h
        S = shift_matrix(e, geo.idx)
        out = out + G_child[(slice(None),) + _child_slice(b) + (slice(None),)] @ S.T
    return out


def m2l_T(geo: Geometry, kernel: Kernel, level: int, GL: np.ndarray,
          triangular: bool = False) -> np.ndarray:
    """Transpose of m2l: G_M[i + o] += T(o)^T G_L[i] over the same admissible pairs."""
    n_l = geo.cells(level)
    finest = level == 0
    GMp = np.zeros(_pad3(GL, geo.dim).shape)
    for o in offsets(geo.dim):
        if not in_window(o, finest):
            continue
        mask = window_mask(n_l, o)
        if not mask.any():
            continue
        T = m2l_tensor(kernel, geo, level, o, triangular)
        sl = (slice(None),) + tuple(slice(3 + oj, 3 + oj + n_l) for oj in o) + (slice(None),)
        GMp[sl] += mask[None, ..., None] * (GL @ T)
    crop = (slice(None),) + (slice(3, 3 + n_l),) * geo.dim + (slice(None),)
    return GMp[crop]


def m2m_T(geo: Geometry, level: int, G_parent: np.ndarray) -> np.ndarray:
    """Transpose of m2m(level): cotangent of the child moments."""
    h = geo.h(level)
    C = G_parent.shape[0]
    n_l = geo.cells(level)
    out = np.zeros((C,) + (n_l,) * geo.dim + (geo.P,))
    for b in child_offsets(geo.dim):
        e = (np.asarray(b) - 0.5) * h
        S = shift_matrix(e, geo.idx)
        out[(slice(None),) + _child_slice(b) + (slice(None),)] = G_parent @ S
    return out


def expand_T(geo: Geometry, kernel: Kernel, G_L0: np.ndarray, triangular: bool = False):
    """Transpose of `expand` (without P2M): cotangent of the finest moments M_0."""
    GLs = [G_L0]
    for lv in range(geo.levels - 1):
        GLs.append(l2l_T(geo, lv, GLs[-1]))
    GMs = [m2l_T(geo, kernel, lv, GLs[lv], triangular) for lv in range(geo.levels)]
    acc = GMs[-1]
    for lv in range(geo.levels - 2, -1, -1):
        acc = GMs[lv] + m2m_T(geo, lv, acc)
    return acc


def p2m_T(geo: Geometry, G_M0: np.ndarray, p: np.ndarray, w: np.ndarray):
    """Transpose of P2M: w_bar[s, c] = sum_n G_M0[c, cell(s), n] (p_s - centre)^n / n!, and
    p_bar[s] = sum_c w[s, c] sum_n G_M0[c, cell(s), n] grad_p (p_s - centre)^n / n!."""
    w = np.asarray(w, dtype=np.float64).reshape(len(p), -1)
    rows, dvec = _gather_cells(geo, G_M0, p)                       # [C, N, P]
    gw = np.einsum("cnp,np->nc", rows, monomials(dvec, geo.idx))
    gp = np.einsum("cnp,npj,nc->nj", rows, monomial_grads(dvec, geo.idx), w)
    return gw, gp


def explicit_forward_backward(geo: Geometry, kernel: Kernel, p, w, q, gy,
                              triangular: bool = False):
    """The explicit layer y = f(q; p, w) and the vector-Jacobian products of section 4.1
    as exact transposes of the discrete expansion: (y, w_bar, p_bar, q_bar)."""
    L0 = expand(geo, kernel, p, w, triangular)
    y = l2p(geo, L0, q)
    gy = np.asarray(gy, dtype=np.float64).reshape(len(q), -1)
    gq = np.einsum("mc,mcj->mj", gy, l2p_grad(geo, L0, q))
    GM0 = expand_T(geo, kernel, l2p_T(geo, q, gy), triangular)
    gw, gp = p2m_T(geo, GM0, p, w)
    return y, gw, gp, gq


# ----------------------------------------------------------------------------- sampled

def moments_all_levels(geo: Geometry, p, w) -> List[np.ndarray]:
    Ms = [p2m(geo, p, w)]
    for lv in range(geo.levels - 1):
        Ms.append(m2m(geo, lv, Ms[-1]))
    return Ms


def locals_at_cells(geo: Geometry, kernel: Kernel, Ms: List[np.ndarray],
                    cells: np.ndarray, triangular: bool = False) -> np.ndarray:
    """L_0 at selected finest cells only, one cell at a time from the moment pyramid:
    the M2L sum at each ancestor, shifted down to the cell by L2L.  Returns [C, S, P].
    Used for spot checks at sizes where the full expansion is too slow in numpy."""
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, geo.dim)
    C = Ms[0].shape[0]
    out = np.zeros((C, len(cells), geo.P))
    tcache = {}
    for si, c in enumerate(cells):
        acc = np.zeros((C, geo.P))
        for lv in range(geo.levels - 1, -1, -1):
            anc = c >> lv
            n_l = geo.cells(lv)
            if lv < geo.levels - 1:
                # shift the parent's locals to this ancestor: L_child = L_parent @ S(e)
                b = anc & 1
                e = (b - 0.5) * geo.h(lv)
                acc = acc @ shift_matrix(e, geo.idx)
            for o in offsets(geo.dim):
                if not in_window(o, lv == 0):
                    continue
                ok = True
                for j in range(geo.dim):
                    ij, oj = int(anc[j]), o[j]
                    lo_, hi_ = (-2, 3) if ij % 2 == 0 else (-3, 2)
                    if not (lo_ <= oj <= hi_ and 0 <= ij + oj < n_l):
                        ok = False
                if not ok:
                    continue
                key = (lv, o)
                if key not in tcache:
                    tcache[key] = m2l_tensor(kernel, geo, lv, o, triangular)
                src = tuple(int(anc[j] + o[j]) for j in range(geo.dim))
                acc = acc + Ms[lv][(slice(None),) + src + (slice(None),)] @ tcache[key].T
        out[:, si, :] = acc
    return out


def local_cotangent_pyramid(geo: Geometry, G_L0: np.ndarray) -> List[np.ndarray]:
    """[G_L0, G_L1, ...]: the cotangents of every level's locals (transpose of the L2L chain)."""
    GLs = [G_L0]
    for lv in range(geo.levels - 1):
        GLs.append(l2l_T(geo, lv, GLs[-1]))
    return GLs


def moment_cotangents_at_cells(geo: Geometry, kernel: Kernel, GLs: List[np.ndarray],
                               cells: np.ndarray, triangular: bool = False) -> np.ndarray:
    """The cotangent of the finest moments at selected finest cells only, [C, S, P]: at each
    ancestor J of a cell, the transposed M2L sum over the targets I = J - o that receive J
    (G_M[J] += G_L[I] T(o), the same admissible pairs as the forward), then shifted down the
    ancestor chain by the transpose of M2M (G_child = G_parent S(e)).  The transpose of
    locals_at_cells; for spot checks of the backward at full size."""
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, geo.dim)
    C = GLs[0].shape[0]
    out = np.zeros((C, len(cells), geo.P))
    tcache = {}
    for si, c in enumerate(cells):
        acc = np.zeros((C, geo.P))
        for lv in range(geo.levels - 1, -1, -1):
            anc = c >> lv
            n_l = geo.cells(lv)
            if lv < geo.levels - 1:
                b = anc & 1
                e = (b - 0.5) * geo.h(lv)
                acc = acc @ shift_matrix(e, geo.idx)
            for o in offsets(geo.dim):
                if not in_window(o, lv == 0):
                    continue
                tgt = [int(anc[j] - o[j]) for j in range(geo.dim)]
                ok = True
                for j in range(geo.dim):
                    lo_, hi_ = (-2, 3) if tgt[j] % 2 == 0 else (-3, 2)
                    if not (0 <= tgt[j] < n_l and lo_ <= o[j] <= hi_):
                        ok = False
                if not ok:
                    continue
                key = (lv, o)
                if key not in tcache:
                    tcache[key] = m2l_tensor(kernel, geo, lv, o, triangular)
                acc = acc + GLs[lv][(slice(None),) + tuple(tgt) + (slice(None),)] @ tcache[key]
        out[:, si, :] = acc
    return out


def p2m_T_rows(geo: Geometry, rows: np.ndarray, p: np.ndarray, w: np.ndarray):
    """p2m_T for sources whose cells' moment cotangents are given row by row ([C, N, P], row s
    for source s): (w_bar, p_bar) of those sources."""
    w = np.asarray(w, dtype=np.float64).reshape(len(p), -1)
    cell = geo.cell_index(p)
    dvec = np.asarray(p, dtype=np.float64) - geo.centre(0, cell)
    gw = np.einsum("cnp,np->nc", rows, monomials(dvec, geo.idx))
    gp = np.einsum("cnp,npj,nc->nj", rows, monomial_grads(dvec, geo.idx), w)
    return gw, gp

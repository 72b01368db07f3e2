"""Algorithmic work of the expansion (flop and byte counts used for roofline figures).

Counts are of what the method must do, not of what a kernel happens to do: unpadded
multi-index counts P, the exact number of admissible (target cell, source cell) pairs at
each level (parity window minus the near-field hole, clipped at the grid boundary), and
each grid read or written once per pass.
"""
from __future__ import annotations

from math import comb


def n_terms(dim: int, K: int) -> int:
    return comb(K + dim, dim)


def _window_pairs_1d(n: int) -> int:
    """sum over cells i of the offsets o in i's parity window with 0 <= i + o < n."""
    tot = 0
    for i in range(n):
        lo, hi = (-2, 3) if i % 2 == 0 else (-3, 2)
        tot += sum(1 for o in range(lo, hi + 1) if 0 <= i + o < n)
    return tot


def _hole_pairs_1d(n: int) -> int:
    return sum(1 for i in range(n) for o in (-1, 0, 1) if 0 <= i + o < n)


def m2l_pairs(dim: int, n_level: int, finest: bool) -> int:
    """Admissible (target, source) cell pairs of one level."""
    pairs = _window_pairs_1d(n_level) ** dim
    if not finest:
        pairs -= _hole_pairs_1d(n_level) ** dim
    return pairs


def levels_of(n: int) -> int:
    lv = 0
    while (2 << lv) < n:
        lv += 1
    return lv


def m2l_flops(dim: int, n: int, K: int, channels: int = 1, level: int | None = None) -> int:
    """Multiply-add flops (2 per term) of the forward M2L, one level or all levels."""
    P = n_terms(dim, K)
    lvls = range(levels_of(n)) if level is None else [level]
    return sum(2 * P * P * channels * m2l_pairs(dim, n >> l, l == 0) for l in lvls)


def grid_bytes(dim: int, n_level: int, K: int, channels: int = 1, itemsize: int = 4) -> int:
    return channels * n_level ** dim * n_terms(dim, K) * itemsize


def mfma_padding(dim: int, K: int) -> float:
    """Issued / useful flops of the 16x16x32 MFMA tiling: in-channels padded to a multiple
    of 8, out-channels to a multiple of 16."""
    P = n_terms(dim, K)
    p8 = (P + 7) // 8 * 8
    p16 = (P + 15) // 16 * 16
    return p8 * p16 / (P * P)


def p_pad(dim: int, K: int) -> int:
    return (n_terms(dim, K) + 3) // 4 * 4


def stage_bytes(stage: str, dim: int, n: int, K: int, N: int = 0, M: int = 0, itemsize: int = 4,
                channels: int = 1) -> int:
    """Algorithmic HBM bytes of one call of a single-kernel stage: every point record and
    every finest-grid row it must touch, once.  Backward outputs are counted as written, not
    updated (the step overwrites its gradient buffers).

    per source / query (es = itemsize, d = dim):
      p2m    sorted p, w read (once, contiguous)        (d + 1) es
      l2p    q read, y written                          (d + 1) es
      l2p_T  sorted q, gy read (once, contiguous)       (d + 1) es
      qgrad  q, gy read, q_bar written                  (2 d + 1) es
      p2m_T  p, w read, p_bar, w_bar written            2 (d + 1) es
      l2p_sorted     sorted q, cell, index read; y written          d es + 12
      l2p_T_sorted   sorted q, index, gy read; q_bar written         (2 d + 1) es + 4
    per finest cell (R = P_pad es channels, one row):
      p2m    cell start read, moment row written        4 + R
      l2p    local row read                             R
      l2p_T  cell start read, cotangent row written     4 + R
      qgrad  local row read                             R
      p2m_T  moment-cotangent row read                  R
      l2p_sorted     local row read                     R
      l2p_T_sorted   cell start read, local row read, cotangent row written   4 + 2 R
    """
    d, es, G = dim, itemsize, n ** dim
    R = p_pad(dim, K) * es * channels
    if stage == "p2m":
        return N * (d + 1) * es + G * (4 + R)
    if stage == "l2p":
        return M * (d + 1) * es + G * R
    if stage == "l2p_T":
        return M * (d + 1) * es + G * (4 + R)
    if stage == "qgrad":
        return M * (2 * d + 1) * es + G * R
    if stage == "p2m_T":
        return N * 2 * (d + 1) * es + G * R
    if stage == "l2p_sorted":
        return M * (d * es + 12) + G * R
    if stage == "l2p_T_sorted":
        return M * ((2 * d + 1) * es + 4) + G * (4 + 2 * R)
    raise ValueError(stage)


# ---- M2L work that actually runs when tiles with nothing to contribute are skipped

# Target tile of one MFMA M2L workgroup (cells per dimension).
def m2l_tile(dim: int, K: int):
    if dim == 2:
        return (16, 8)
    return (16, 8, 4) if n_terms(3, K) <= 35 else (16, 8, 8)


def _window_counts_1d(n: int):
    """Per cell i: offsets of its parity window inside the grid, and hole offsets inside."""
    import numpy as np
    i = np.arange(n)
    lo = np.where(i % 2 == 0, -2, -3)
    hi = lo + 5
    w = np.minimum(i + hi, n - 1) - np.maximum(i + lo, 0) + 1
    h = np.minimum(i + 1, n - 1) - np.maximum(i - 1, 0) + 1
    return w, h


def occupancy_pyramid(x, lo: float, hi: float, n: int, dim: int):
    """Occupancy of every level: finest cells by the kernels' FP32 index formula, then any()
    over the 2^d children."""
    import numpy as np
    xs = np.asarray(x, dtype=np.float32)
    scale = np.float32(n / (hi - lo))
    u = (xs - np.float32(lo)) * scale
    idx = np.clip(np.floor(u).astype(np.int64), 0, n - 1)
    occ = np.zeros((n,) * dim, dtype=bool)
    occ[tuple(idx[:, j] for j in range(dim))] = True
    levels = [occ]
    while levels[-1].shape[0] > 4:
        o = levels[-1]
        m = o.shape[0] // 2
        o = o.reshape(sum(((m, 2) for _ in range(dim)), ()))
        levels.append(o.any(axis=tuple(range(1, 2 * dim, 2))))
    return levels


def m2l_flops_executed(dim: int, K: int, occ_levels, transpose: bool, channels: int = 1) -> int:
    """Useful flops (2 per term, unpadded P) of the M2L tiles that run: the forward skips a tile
    whose source region (targets +- 2..3 cells) holds no occupied cell, the transpose one none
    of whose outputs is occupied."""
    import numpy as np
    P = n_terms(dim, K)
    tile = m2l_tile(dim, K)
    total = 0
    for lvl, occ in enumerate(occ_levels):
        n_l = occ.shape[0]
        w, h = _window_counts_1d(n_l)
        pairs = np.ones((n_l,) * dim, dtype=np.int64)
        holes = np.ones((n_l,) * dim, dtype=np.int64)
        for d in range(dim):
            shape = [1] * dim
            shape[d] = n_l
            pairs = pairs * w.reshape(shape)
            holes = holes * h.reshape(shape)
        if lvl > 0:
            pairs = pairs - holes
        run = np.zeros((n_l,) * dim, dtype=bool)
        ntiles = [(n_l + t - 1) // t for t in tile]
        for t_idx in np.ndindex(*ntiles):
            tgt = tuple(slice(t_idx[d] * tile[d], min((t_idx[d] + 1) * tile[d], n_l)) for d in range(dim))
            if transpose:
                live = occ[tgt].any()
            else:
                src = tuple(slice(max(t_idx[d] * tile[d] - 2, 0), min((t_idx[d] + 1) * tile[d] + 2, n_l))
                            for d in range(dim))
                live = occ[src].any()
            if live:
                run[tgt] = True
        total += int(pairs[run].sum())
    return 2 * P * P * channels * total


# ---- separable M2L (Gaussian): one-dimensional passes over intermediate index sets

def _sep_sets(dim: int, K: int):
    """Index sets of the pass chain: S0 (|v| <= K), A and, in 3-D, B."""
    r = range(K + 1)
    if dim == 2:
        S0 = [(a, b) for a in r for b in r if a + b <= K]
        return S0, [(a, b) for a in r for b in r], None
    S0 = [(a, b, c) for a in r for b in r for c in r if a + b + c <= K]
    A = [(a, b, c) for a in r for b in r for c in r if b + c <= K]
    B = [(a, b, c) for a in r for b in r for c in r if a + b <= K]
    return S0, A, B


def _pass_entries(src, dst, axis: int, K: int) -> int:
    """Multiply-adds per cell and offset of one pass: for every output tuple, the input tuples
    equal to it except at the contracted axis."""
    have = set(src)
    tot = 0
    for t in dst:
        for v in range(K + 1):
            u = list(t)
            u[axis] = v
            tot += tuple(u) in have
    return tot


def sep_pass_entries(dim: int, K: int):
    """Per forward pass (x, y[, z]) the multiply-adds per cell and offset."""
    S0, A, B = _sep_sets(dim, K)
    if dim == 2:
        return [_pass_entries(S0, A, 0, K), _pass_entries(A, S0, 1, K)]
    return [_pass_entries(S0, A, 0, K), _pass_entries(A, B, 1, K), _pass_entries(B, S0, 2, K)]


def m2l_flops_separable(dim: int, n: int, K: int, channels: int = 1) -> int:
    """Flops (2 per multiply-add) of the separable M2L at every level: each pass runs the
    window chain (per cell the in-grid offsets of its one-dimensional parity window) and, above
    the finest level, the hole chain (offsets -1..1).  The transpose does the same work."""
    ents = sep_pass_entries(dim, K)
    total = 0
    for l in range(levels_of(n)):
        n_l = n >> l
        per_axis = _window_pairs_1d(n_l) + (_hole_pairs_1d(n_l) if l > 0 else 0)
        total += sum(ents) * n_l ** (dim - 1) * per_axis
    return 2 * channels * total


def m2l_bytes_separable(dim: int, n: int, K: int, itemsize: int = 4, channels: int = 1) -> int:
    """HBM bytes of the separable M2L at every level: every pass reads its input rows and
    writes its output rows once per chain (the first pass reads the moment row once for both
    chains, the last writes one local row: window minus hole)."""
    S0, A, B = _sep_sets(dim, K)
    sizes = [len(A)] if dim == 2 else [len(A), len(B)]
    R = p_pad(dim, K)
    total = 0
    for l in range(levels_of(n)):
        chains = 1 if l == 0 else 2
        per_cell = R + R + 2 * chains * sum(sizes)   # first read, last write, each intermediate out and in
        total += (n >> l) ** dim * per_cell
    return total * itemsize * channels


# ---- whole-step roofline of the explicit layer (forward + backward)

def key_passes(G: int) -> int:
    """8-bit radix passes of a sort by finest cell (keys 0..G, G marking unused records)."""
    bits = max(1, int(G).bit_length())
    return (bits + 7) // 8


def sort_bytes(count: int, dim: int, G: int, payload_words: int, itemsize: int = 4) -> int:
    """Algorithmic bytes of one sort of `count` points by cell: the cell key computed from the
    coordinates (read d coordinates, write one key), every radix pass reading and writing key and
    index, the payload words read once and written once in sorted order (the last pass gathers
    them by original index), and the cell starts written."""
    per_pass = 2 * 8
    return (count * (dim * itemsize + 4) + key_passes(G) * count * per_pass + 2 * 4 * payload_words * count
            + (G + 1) * 4)


def pyramid_rows(dim: int, n: int) -> list:
    return [(n >> l) ** dim for l in range(levels_of(n))]


def explicit_step_model(dim: int, n: int, K: int, N: int, M: int, m2l_flops_fwd: int, m2l_flops_T: int,
                        itemsize: int = 4, carried: bool = True, sorted_queries: bool = True) -> dict:
    """Per stage of one explicit-layer step (expand, eval, eval_backward, expand_backward) the
    algorithmic HBM bytes and flops, grouped as the library's stage timing groups its launches.
    M2L flops are passed in (useful flops of the tiles that run).  sorted_queries: the step of
    eval_sorted / eval_backward_sorted (queries sorted once with their coordinates, L2P from the
    sorted records, q_bar fused into the transpose of L2P); otherwise eval / eval_backward."""
    G = n ** dim
    R = p_pad(dim, K) * itemsize
    rows = pyramid_rows(dim, n)
    pw = dim + 1 if carried else 0
    pq = dim if sorted_queries else pw
    sort = sort_bytes(N, dim, G, pw, itemsize) + sort_bytes(M, dim, G, pq, itemsize) + N * dim * itemsize + G
    up = sum(rows) * R                         # read the finest grid, write every coarser one
    down = sum(rows) * R + rows[0] * R         # read every grid, write the finest
    m2l_io = 2 * sum(rows) * R                 # moments (or local cotangents) in, locals out
    return {
        "sort": {"bytes": sort, "flops": 0},
        "p2m": {"bytes": stage_bytes("p2m", dim, n, K, N=N, itemsize=itemsize), "flops": 0},
        "shift_up": {"bytes": 2 * up, "flops": 0},
        "m2l": {"bytes": m2l_io, "flops": m2l_flops_fwd},
        "shift_down": {"bytes": 2 * down, "flops": 0},
        "l2p": {"bytes": stage_bytes("l2p_sorted" if sorted_queries else "l2p", dim, n, K, M=M, itemsize=itemsize),
                "flops": 0},
        "l2p_T": {"bytes": stage_bytes("l2p_T_sorted" if sorted_queries else "l2p_T", dim, n, K, M=M,
                                       itemsize=itemsize), "flops": 0},
        "qgrad": {"bytes": 0 if sorted_queries else stage_bytes("qgrad", dim, n, K, M=M, itemsize=itemsize),
                  "flops": 0},
        "m2l_T": {"bytes": m2l_io, "flops": m2l_flops_T},
        "p2m_T": {"bytes": stage_bytes("p2m_T", dim, n, K, N=N, itemsize=itemsize), "flops": 0},
    }


def stage_roof_us(stage: dict, hbm_GBps: float, peak_TFLOPs: float) -> float:
    """max(bytes / HBM peak, flops / compute peak) in microseconds."""
    return max(stage["bytes"] / (hbm_GBps * 1e3), stage["flops"] / (peak_TFLOPs * 1e6))

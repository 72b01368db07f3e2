// Separable M2L for the Gaussian kernel (§3.4.1: decomposable kernels).
//
// psi(x) = exp(-|x|^2 / (2 sigma^2)) is a product of one-dimensional factors g(x_d), so every
// derivative factors, d^a psi(x) = prod_d g^(a_d)(x_d), and so does the cell-scaled M2L tensor:
//   T[k][n](o) = prod_d tau[k_d][n_d](o_d),  tau[a][b](o) = h^(a+b) (-1)^b g^(a+b)(-o h).
// The window (per dimension [-2, 3] for an even target index, [-3, 2] for an odd one) and the
// near-field hole H = [-1, 1]^d are products of one-dimensional sets as well.  At the finest
// level every offset of the window counts; above it the admissible offsets W \ H split into
// disjoint products (a_1, a_2, ... the axes in pass order, W_a and H_a their one-dimensional sets)
//   (W_a1 \ H_a1) x W_a2 x W_a3  u  H_a1 x (W_a2 \ H_a2) x W_a3  u  H_a1 x H_a2 x (W_a3 \ H_a3),
// so every pass carries two streams, P (already outside the hole along an earlier axis) and Q
// (inside it along every earlier axis):
//   first:  P = (W \ H)(M),          Q = H(M)
//   middle: P = W(P) + (W \ H)(Q),   Q = H(Q)
//   last:   L = W(P) + (W \ H)(Q)
// where each operator sums one offset component against tau.  Subtracting a hole sum from a
// window sum instead would cancel near-field terms that dwarf the far field when sigma is
// small against the cell.  After the passes over the axes in C the rows are indexed by
//   S(C) = {t : sum_{d not in C} t_d <= K and sum_{d in C} t_d <= K}
// (uncontracted components still hold the input index, contracted ones the output index);
// S({}) = S(all) is the set |v| <= K.  M is zero outside it and only outputs inside it are
// kept, so the partial sums give exactly the square-truncated contraction.  The transpose runs
// the same chain with the roles of k and n swapped and the offset reflected.
//
// Axis order: the first pass contracts the last axis (the rows of neighbouring cells are
// contiguous, so the input tile with its halo is one block of memory staged in LDS); in 3-D the
// middle pass contracts axis 0 (each lane walks a column of cells, keeping the halo in
// registers) and the last pass axis 1; in 2-D the last pass contracts axis 0.  Intermediate
// rows are stored as planes [index][cell], so a wave's loads and stores are contiguous.  Lanes
// are cells and every loop (group, input component, offset, output component) is uniform, so
// the coefficients are scalar operands.  Each pass covers every level and both streams in one
// launch; the intermediates live in the caller's workspace.
#include <math.h>

#include <map>
#include <vector>

#include "plan.h"

using namespace fc2t2;

namespace {

constexpr int kSepLanes = 64;    // cells (columns) of a workgroup, one per lane
constexpr int kSepWaves = 4;     // waves of a workgroup: the same cells, groups split between them
constexpr int kSepThreads = kSepLanes * kSepWaves;
constexpr int kSepMaxK1 = 7;     // K + 1 <= 7
constexpr int kSepCol = 4;       // cells per lane along axis 0 in the middle (3-D) pass
constexpr int kHalo = 3;

// Rows that share every index component except the contracted one form a group: the pass maps
// its nv inputs (contracted component v = 0 .. nv-1) to its nu outputs (u = 0 .. nu-1).
struct SepGroup {
  int nv, nu;
  int in_idx[kSepMaxK1];    // position of component v in the input row (AoS column or plane)
  int out_idx[kSepMaxK1];   // position of component u in the output row
};

struct SepLevel {
  const void* in_w;   // first pass: AoS rows [G][Ppad]; later passes: planes [nin][G]
  const void* in_h;   // Q planes (later passes above the finest level), else null
  void* out_w;        // P planes [nout][G]; last pass: AoS rows [G][Ppad]
  void* out_h;        // Q planes (first and middle passes above the finest level), else null
  int64_t G;
  int64_t tau_off;    // this level's coefficients [v][u][o + 3] in the table
  int n, block_begin, hole;
};

struct SepBatch {
  SepLevel lv[kMaxLevels];
  int nlev, ngroups, nin, nout, Ppad, K1;
};

__device__ __forceinline__ int sep_level(const SepBatch& b) {
  int lvl = b.nlev - 1;
  while (lvl > 0 && (int)blockIdx.x < b.lv[lvl].block_begin) --lvl;
  return lvl;
}

// o in -3..3 usable at own coordinate i along the axis: inside the grid, and o = +3 only at an
// even i, o = -3 only at an odd one (the parity window; for the transpose with the offset
// reflected the condition is the same).
__device__ __forceinline__ bool sep_offset_ok(int i, int o, int n) {
  if (i + o < 0 || i + o >= n) return false;
  if (o == 3) return !(i & 1);
  if (o == -3) return (i & 1);
  return true;
}

// Every kernel computes all K1 outputs of a group with straight-line code (the coefficient table
// covers every output component; outputs beyond the group's nu are not stored) and loads
// unconditionally from clamped, in-bounds addresses, masking the value afterwards.
template <typename T, int K1>
__device__ __forceinline__ void sep_fma_all(const T* __restrict__ tv, const T (&x)[7], T (&ap)[K1]) {
#pragma unroll
  for (int u = 0; u < K1; ++u) {
    T a = ap[u];
#pragma unroll
    for (int o = 0; o < 7; ++o) a += tv[u * 7 + o] * x[o];
    ap[u] = a;
  }
}
template <typename T, int K1>
__device__ __forceinline__ void sep_fma_split(const T* __restrict__ tv, const T (&x)[7], T (&ap)[K1], T (&aq)[K1]) {
#pragma unroll
  for (int u = 0; u < K1; ++u) {
    const T* t = tv + u * 7;
    ap[u] += t[0] * x[0] + t[1] * x[1] + t[5] * x[5] + t[6] * x[6];
    aq[u] += t[2] * x[2] + t[3] * x[3] + t[4] * x[4];
  }
}

// First pass, along the last axis: AoS input rows of 64 cells and their halo staged in LDS.
// Above the finest level P = (W \ H)(M) and Q = H(M), else P = W(M).
template <int D, typename T, int K1>
__global__ void __launch_bounds__(kSepThreads) sep_first_kernel(const SepBatch b, const SepGroup* __restrict__ groups,
                                                                const T* __restrict__ tau_all) {
  extern __shared__ __align__(16) char sep_smem[];
  T* tile = reinterpret_cast<T*>(sep_smem);
  const int tid = threadIdx.x, lane = tid & (kSepLanes - 1), ch = blockIdx.y;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kSepLanes);
  const SepLevel& L = b.lv[sep_level(b)];
  const int64_t G = L.G;
  const int n = L.n, Ppad = b.Ppad, rs = Ppad + 1;
  const int64_t c0 = (int64_t)(blockIdx.x - L.block_begin) * kSepLanes;
  const T* in = (const T*)L.in_w + (int64_t)ch * G * Ppad;
  // rows c0 - 3 .. c0 + 66, zero outside the grid; contiguous in memory
  const int64_t r0 = c0 - kHalo;
  const int nelem = (kSepLanes + 2 * kHalo) * Ppad;
  for (int e = tid; e < nelem; e += kSepThreads) {
    const int r = e / Ppad, k = e - r * Ppad;
    const int64_t cell = r0 + r;
    tile[r * rs + k] = (cell >= 0 && cell < G) ? in[r0 * Ppad + e] : T(0);
  }
  __syncthreads();
  const int64_t cell = c0 + lane;
  if (cell >= G) return;
  const int i = (int)(cell % n);
  bool ok[7];
#pragma unroll
  for (int o = -3; o <= 3; ++o) ok[o + 3] = sep_offset_ok(i, o, n);
  const bool hole = L.hole;
  const T* tau = tau_all + L.tau_off;
  T* outw = (T*)L.out_w + (int64_t)ch * b.nout * G + cell;
  T* outh = hole ? (T*)L.out_h + (int64_t)ch * b.nout * G + cell : nullptr;
  const T* mine = tile + (lane + kHalo) * rs;
  for (int g = wave; g < b.ngroups; g += kSepWaves) {
    const SepGroup& gr = groups[g];
    T ap[K1], aq[K1];
#pragma unroll
    for (int u = 0; u < K1; ++u) ap[u] = aq[u] = T(0);
    for (int v = 0; v < gr.nv; ++v) {
      const T* row = mine + gr.in_idx[v];   // rows lane .. lane + 6 of the tile: always inside it
      T x[7];
#pragma unroll
      for (int o = 0; o < 7; ++o) {
        const T val = row[(o - kHalo) * rs];
        x[o] = ok[o] ? val : T(0);
      }
      if (hole)
        sep_fma_split<T, K1>(tau + v * K1 * 7, x, ap, aq);
      else
        sep_fma_all<T, K1>(tau + v * K1 * 7, x, ap);
    }
#pragma unroll
    for (int u = 0; u < K1; ++u) {
      if (u < gr.nu) {
        outw[(int64_t)gr.out_idx[u] * G] = ap[u];
        if (hole) outh[(int64_t)gr.out_idx[u] * G] = aq[u];
      }
    }
  }
}

// Middle pass (3-D), along axis 0: each lane walks kSepCol cells of a column; the column's
// inputs and halo are loaded once per input component.  P = W(P) + (W \ H)(Q), Q = H(Q).
template <typename T, int K1>
__global__ void __launch_bounds__(kSepThreads) sep_mid_kernel(const SepBatch b, const SepGroup* __restrict__ groups,
                                                              const T* __restrict__ tau_all) {
  const int tid = threadIdx.x, lane = tid & (kSepLanes - 1), ch = blockIdx.y;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kSepLanes);
  const SepLevel& L = b.lv[sep_level(b)];
  const int64_t G = L.G;
  const int n = L.n;
  const int64_t plane = (int64_t)n * n;
  const int nblk_plane = (int)((plane + kSepLanes - 1) / kSepLanes);
  const int blk = (int)blockIdx.x - L.block_begin;
  const int colblk = blk / nblk_plane;
  const int64_t m = (int64_t)(blk - colblk * nblk_plane) * kSepLanes + lane;
  if (m >= plane) return;
  const int i0 = colblk * kSepCol;   // even: the parity of cell c of the column is c & 1
  const bool hole = L.hole;
  const T* tau = tau_all + L.tau_off;
  const T* inw = (const T*)L.in_w + (int64_t)ch * b.nin * G + m;
  const T* inh = hole ? (const T*)L.in_h + (int64_t)ch * b.nin * G + m : nullptr;
  T* outw = (T*)L.out_w + (int64_t)ch * b.nout * G + m;
  T* outh = hole ? (T*)L.out_h + (int64_t)ch * b.nout * G + m : nullptr;
  // column rows i0 - 3 .. i0 + kSepCol + 2, clamped into the grid; masks for the clamped ones
  int64_t rofs[kSepCol + 2 * kHalo];
  bool rin[kSepCol + 2 * kHalo];
#pragma unroll
  for (int j = 0; j < kSepCol + 2 * kHalo; ++j) {
    const int i = i0 - kHalo + j;
    rin[j] = i >= 0 && i < n;
    rofs[j] = (int64_t)(i < 0 ? 0 : (i >= n ? n - 1 : i)) * plane;
  }
  for (int g = wave; g < b.ngroups; g += kSepWaves) {
    const SepGroup& gr = groups[g];
    T ap[kSepCol][K1], aq[kSepCol][K1];
#pragma unroll
    for (int c = 0; c < kSepCol; ++c)
#pragma unroll
      for (int u = 0; u < K1; ++u) ap[c][u] = aq[c][u] = T(0);
    for (int v = 0; v < gr.nv; ++v) {
      const int64_t pofs = (int64_t)gr.in_idx[v] * G;
      const T* tv = tau + v * K1 * 7;
      T x[kSepCol + 2 * kHalo];
#pragma unroll
      for (int j = 0; j < kSepCol + 2 * kHalo; ++j) {
        const T val = inw[pofs + rofs[j]];
        x[j] = rin[j] ? val : T(0);
      }
#pragma unroll
      for (int u = 0; u < K1; ++u) {
        const T* t = tv + u * 7;
#pragma unroll
        for (int c = 0; c < kSepCol; ++c) {
          T a = ap[c][u];
#pragma unroll
          for (int o = -3; o <= 3; ++o) {
            if (o == 3 && (c & 1)) continue;
            if (o == -3 && !(c & 1)) continue;
            a += t[o + 3] * x[c + kHalo + o];
          }
          ap[c][u] = a;
        }
      }
      if (hole) {
        T z[kSepCol + 2 * kHalo];
#pragma unroll
        for (int j = 0; j < kSepCol + 2 * kHalo; ++j) {
          const T val = inh[pofs + rofs[j]];
          z[j] = rin[j] ? val : T(0);
        }
#pragma unroll
        for (int u = 0; u < K1; ++u) {
          const T* t = tv + u * 7;
#pragma unroll
          for (int c = 0; c < kSepCol; ++c) {
            T a = ap[c][u], q = aq[c][u];
#pragma unroll
            for (int o = -3; o <= 3; ++o) {
              if (o == 3 && (c & 1)) continue;
              if (o == -3 && !(c & 1)) continue;
              if (o < -1 || o > 1)
                a += t[o + 3] * z[c + kHalo + o];
              else
                q += t[o + 3] * z[c + kHalo + o];
            }
            ap[c][u] = a;
            aq[c][u] = q;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < K1; ++u) {
      if (u < gr.nu) {
        const int64_t pofs = (int64_t)gr.out_idx[u] * G;
#pragma unroll
        for (int c = 0; c < kSepCol; ++c) {
          outw[pofs + (i0 + c) * plane] = ap[c][u];
          if (hole) outh[pofs + (i0 + c) * plane] = aq[c][u];
        }
      }
    }
  }
}

// Last pass, along axis 1 (3-D) or 0 (2-D): the neighbour along the axis is n cells away in
// both cases.  L = W(P) + (W \ H)(Q), staged in LDS as AoS rows and written out whole, with
// the row padding zeroed.
template <int D, typename T, int K1>
__global__ void __launch_bounds__(kSepThreads) sep_last_kernel(const SepBatch b, const SepGroup* __restrict__ groups,
                                                               const T* __restrict__ tau_all) {
  extern __shared__ __align__(16) char sep_smem[];
  T* st = reinterpret_cast<T*>(sep_smem);
  const int tid = threadIdx.x, lane = tid & (kSepLanes - 1), ch = blockIdx.y;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kSepLanes);
  const SepLevel& L = b.lv[sep_level(b)];
  const int64_t G = L.G;
  const int n = L.n, Ppad = b.Ppad, rs = Ppad + 1;
  const int64_t c0 = (int64_t)(blockIdx.x - L.block_begin) * kSepLanes;
  for (int e = tid; e < kSepLanes * rs; e += kSepThreads) st[e] = T(0);
  __syncthreads();
  const int64_t cell = c0 + lane;
  if (cell < G) {
    const int i = (int)((cell / n) % n);
    bool ok[7], okq[7];
    int64_t nofs[7];   // neighbour offsets, clamped into the grid
#pragma unroll
    for (int o = -3; o <= 3; ++o) {
      ok[o + 3] = sep_offset_ok(i, o, n);
      okq[o + 3] = ok[o + 3] && (o < -1 || o > 1);
      const int j = i + o < 0 ? 0 : (i + o >= n ? n - 1 : i + o);
      nofs[o + 3] = (int64_t)(j - i) * n;
    }
    const bool hole = L.hole;
    const T* tau = tau_all + L.tau_off;
    const T* inw = (const T*)L.in_w + (int64_t)ch * b.nin * G + cell;
    const T* inh = hole ? (const T*)L.in_h + (int64_t)ch * b.nin * G + cell : nullptr;
    T* mine = st + lane * rs;
    for (int g = wave; g < b.ngroups; g += kSepWaves) {
      const SepGroup& gr = groups[g];
      T ap[K1];
#pragma unroll
      for (int u = 0; u < K1; ++u) ap[u] = T(0);
      for (int v = 0; v < gr.nv; ++v) {
        const int64_t pofs = (int64_t)gr.in_idx[v] * G;
        const T* tv = tau + v * K1 * 7;
        T x[7];
#pragma unroll
        for (int o = 0; o < 7; ++o) {
          const T val = inw[pofs + nofs[o]];
          x[o] = ok[o] ? val : T(0);
        }
        sep_fma_all<T, K1>(tv, x, ap);
        if (hole) {
#pragma unroll
          for (int o = 0; o < 7; ++o) {
            const T val = (o < 2 || o > 4) ? inh[pofs + nofs[o]] : T(0);
            x[o] = okq[o] ? val : T(0);
          }
#pragma unroll
          for (int u = 0; u < K1; ++u) {
            const T* t = tv + u * 7;
            ap[u] += t[0] * x[0] + t[1] * x[1] + t[5] * x[5] + t[6] * x[6];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < K1; ++u)
        if (u < gr.nu) mine[gr.out_idx[u]] = ap[u];
    }
  }
  __syncthreads();
  T* out = (T*)L.out_w + (int64_t)ch * G * Ppad;
  const int64_t rows = G - c0 < kSepLanes ? G - c0 : kSepLanes;
  for (int e = tid; e < rows * Ppad; e += kSepThreads) {
    const int r = e / Ppad, k = e - r * Ppad;
    out[c0 * Ppad + e] = st[r * rs + k];
  }
}

// ---- host: index sets and pass tables
using Tuple = std::vector<int>;

struct IndexSet {
  std::vector<Tuple> items;
  std::map<Tuple, int> pos;   // position in the row layout
};

// S(C) (contracted axes in C): sum over uncontracted components <= K and over contracted ones <= K.
// The AoS sets (C empty or all axes) take the library's graded order, the intermediates their
// enumeration order (plane index).
IndexSet index_set(int D, int K, const std::vector<bool>& contracted) {
  IndexSet s;
  bool any = false, all = true;
  for (int d = 0; d < D; ++d) {
    any = any || contracted[d];
    all = all && contracted[d];
  }
  if (!any || all) {
    std::vector<int> e((size_t)nterms(D, K) * 3);
    mi_fill(D, K, reinterpret_cast<int(*)[3]>(e.data()));
    for (int p = 0; p < nterms(D, K); ++p) {
      Tuple t(e.begin() + 3 * p, e.begin() + 3 * p + D);
      s.pos[t] = p;
      s.items.push_back(t);
    }
    return s;
  }
  Tuple t(D, 0);
  for (;;) {
    int su = 0, sc = 0;
    for (int d = 0; d < D; ++d) (contracted[d] ? sc : su) += t[d];
    if (su <= K && sc <= K) {
      s.pos[t] = (int)s.items.size();
      s.items.push_back(t);
    }
    int d = D - 1;
    while (d >= 0 && t[d] == K) t[d--] = 0;
    if (d < 0) break;
    ++t[d];
  }
  return s;
}

// Groups of the pass from `in` to `out` along `axis`: one per output tuple with a zero component
// at the axis (every output row lies in exactly one group).
void build_groups(const IndexSet& in, const IndexSet& out, int axis, int K, std::vector<SepGroup>& groups) {
  for (const Tuple& t : out.items) {
    if (t[axis] != 0) continue;
    SepGroup g{};
    Tuple u = t;
    for (int c = 0; c <= K; ++c) {
      u[axis] = c;
      auto it = in.pos.find(u);
      if (it != in.pos.end()) g.in_idx[g.nv++] = it->second;
      auto jt = out.pos.find(u);
      if (jt != out.pos.end()) g.out_idx[g.nu++] = jt->second;
    }
    groups.push_back(g);
  }
}

// g^(m)(t) for g(t) = exp(-t^2 / (2 s^2)): (-1)^m s^-m He_m(t / s) g(t), probabilists' Hermite.
double gauss_deriv(int m, double t, double s) {
  const double x = t / s;
  double h0 = 1.0, h1 = x;
  double he = m == 0 ? 1.0 : x;
  for (int j = 1; j < m; ++j) {
    const double h2 = x * h1 - j * h0;
    h0 = h1;
    h1 = h2;
    he = h2;
  }
  return ((m & 1) ? -1.0 : 1.0) * pow(s, -m) * he * exp(-0.5 * x * x);
}

}  // namespace

// Plan-side data (groups of every pass, per-level coefficients) in one device allocation.
struct SepTables {
  int axis[3] = {};          // contracted axis of each pass
  int ngroups[3] = {};
  int group_off[3] = {};     // first group of each pass
  int nset[3] = {};          // row size before each pass: Ppad, |S({a0})|, |S({a0, a1})|
  int nA = 0, nB = 0;
  size_t group_bytes = 0;
  int64_t tau_dir_elems = 0; // coefficients of one direction (all levels)
  void* dev = nullptr;       // [groups][tau forward][tau transpose]
};

namespace fc2t2 {

bool sep_supported(const fc2t2_plan_s* pl) { return pl->kind == FC2T2_GAUSSIAN && pl->K + 1 <= kSepMaxK1; }

fc2t2_status sep_build(fc2t2_plan_s* pl, hipStream_t s) {
  if (!sep_supported(pl)) return FC2T2_EUNSUPPORTED;
  const int D = pl->dim, K = pl->K;
  SepTables* t = new (std::nothrow) SepTables();
  if (!t) return FC2T2_ENOMEM;
  pl->sep = t;
  if (D == 2) {
    t->axis[0] = 1;
    t->axis[1] = 0;
  } else {
    t->axis[0] = 2;
    t->axis[1] = 0;
    t->axis[2] = 1;
  }
  std::vector<bool> con(D, false);
  IndexSet prev = index_set(D, K, con);
  std::vector<SepGroup> groups;
  for (int p = 0; p < D; ++p) {
    con[t->axis[p]] = true;
    IndexSet next = index_set(D, K, con);
    t->group_off[p] = (int)groups.size();
    build_groups(prev, next, t->axis[p], K, groups);
    t->ngroups[p] = (int)groups.size() - t->group_off[p];
    if (p + 1 < D) t->nset[p + 1] = (int)next.items.size();
    prev = std::move(next);
  }
  t->nset[0] = pl->Ppad;
  t->nA = t->nset[1];
  t->nB = D == 3 ? t->nset[2] : 0;
  // coefficients per level, [v][u][o + 3]: forward (v = n, u = k) tau[u][v](o); transpose
  // (v = k, u = n, offset reflected) tau[v][u](-o)
  const int K1 = K + 1;
  const size_t es = io_size(pl);
  t->tau_dir_elems = (int64_t)pl->levels * K1 * K1 * 7;
  std::vector<double> tau(2 * (size_t)t->tau_dir_elems);
  for (int l = 0; l < pl->levels; ++l) {
    const double h = pl->h0 * (double)(1 << l);
    auto coef = [&](int a, int b, int o) {
      return pow(h, a + b) * ((b & 1) ? -1.0 : 1.0) * gauss_deriv(a + b, -o * h, pl->param);
    };
    for (int v = 0; v <= K; ++v)
      for (int u = 0; u <= K; ++u)
        for (int o = -3; o <= 3; ++o) {
          const size_t i = (((size_t)l * K1 + v) * K1 + u) * 7 + (o + 3);
          tau[i] = coef(u, v, o);
          tau[t->tau_dir_elems + i] = coef(v, u, -o);
        }
  }
  t->group_bytes = align256(groups.size() * sizeof(SepGroup));
  const size_t tau_bytes = tau.size() * es;
  if (hipMalloc(&t->dev, t->group_bytes + tau_bytes) != hipSuccess) {
    t->dev = nullptr;
    return FC2T2_ENOMEM;
  }
  char* p = (char*)t->dev;
  if (hipMemcpyAsync(p, groups.data(), groups.size() * sizeof(SepGroup), hipMemcpyHostToDevice, s) != hipSuccess)
    return FC2T2_EHIP;
  std::vector<float> tau32;
  const void* src = tau.data();
  if (pl->io == FC2T2_IO_F32) {
    tau32.assign(tau.begin(), tau.end());
    src = tau32.data();
  }
  if (hipMemcpyAsync(p + t->group_bytes, src, tau_bytes, hipMemcpyHostToDevice, s) != hipSuccess) return FC2T2_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? FC2T2_OK : FC2T2_EHIP;
}

void sep_destroy(fc2t2_plan_s* pl) {
  if (!pl->sep) return;
  if (pl->sep->dev) (void)hipFree(pl->sep->dev);
  delete pl->sep;
  pl->sep = nullptr;
}

// Intermediate planes: per level, A and (3-D) B for the P stream and, above the finest level,
// for the Q stream.
size_t sep_ws_bytes(const fc2t2_plan_s* pl) {
  if (!pl->sep) return 0;
  size_t b = 0;
  const size_t es = io_size(pl);
  for (int l = 0; l < pl->levels; ++l) {
    const int chains = l == 0 ? 1 : 2;
    b += chains * align256((size_t)pl->C * pl->Gl[l] * pl->sep->nA * es);
    if (pl->dim == 3) b += chains * align256((size_t)pl->C * pl->Gl[l] * pl->sep->nB * es);
  }
  return b;
}

template <typename T, int K1>
static fc2t2_status sep_launch(int D, int kind, dim3 grid, size_t lds, hipStream_t s, const SepBatch& b,
                               const SepGroup* gp, const T* tau) {
  const dim3 block(kSepThreads);
  if (kind == 0) {
    if (D == 2)
      hipLaunchKernelGGL((sep_first_kernel<2, T, K1>), grid, block, lds, s, b, gp, tau);
    else
      hipLaunchKernelGGL((sep_first_kernel<3, T, K1>), grid, block, lds, s, b, gp, tau);
  } else if (kind == 2) {
    if (D == 2)
      hipLaunchKernelGGL((sep_last_kernel<2, T, K1>), grid, block, lds, s, b, gp, tau);
    else
      hipLaunchKernelGGL((sep_last_kernel<3, T, K1>), grid, block, lds, s, b, gp, tau);
  } else {
    hipLaunchKernelGGL((sep_mid_kernel<T, K1>), grid, block, 0, s, b, gp, tau);
  }
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

template <typename T>
static fc2t2_status sep_run(const fc2t2_plan_s* pl, const void* const* ins, void* const* outs, bool transpose,
                            void* ws, hipStream_t s) {
  const SepTables* t = pl->sep;
  const int D = pl->dim, K1 = pl->K + 1;
  const size_t es = sizeof(T);
  // per level [A_P, A_Q, B_P, B_Q] (Q planes above the finest level only)
  void* Aw[kMaxLevels] = {};
  void* Ah[kMaxLevels] = {};
  void* Bw[kMaxLevels] = {};
  void* Bh[kMaxLevels] = {};
  char* p = (char*)ws;
  for (int l = 0; l < pl->levels; ++l) {
    const size_t a = align256((size_t)pl->C * pl->Gl[l] * t->nA * es);
    const size_t b = D == 3 ? align256((size_t)pl->C * pl->Gl[l] * t->nB * es) : 0;
    Aw[l] = p;
    p += a;
    if (l > 0) {
      Ah[l] = p;
      p += a;
    }
    if (D == 3) {
      Bw[l] = p;
      p += b;
      if (l > 0) {
        Bh[l] = p;
        p += b;
      }
    }
  }
  const SepGroup* groups = (const SepGroup*)t->dev;
  const T* tau = (const T*)((const char*)t->dev + t->group_bytes) + (transpose ? t->tau_dir_elems : 0);
  void* const* mid_w[2] = {Aw, Bw};
  void* const* mid_h[2] = {Ah, Bh};
  for (int pi = 0; pi < D; ++pi) {
    const bool first = pi == 0, last = pi == D - 1;
    SepBatch b{};
    b.nlev = pl->levels;
    b.ngroups = t->ngroups[pi];
    b.nin = t->nset[pi];
    b.nout = last ? pl->Ppad : t->nset[pi + 1];
    b.Ppad = pl->Ppad;
    b.K1 = K1;
    int blocks = 0;
    for (int l = 0; l < pl->levels; ++l) {
      SepLevel& L = b.lv[l];
      L.in_w = first ? ins[l] : mid_w[pi - 1][l];
      L.in_h = first ? nullptr : mid_h[pi - 1][l];
      L.out_w = last ? outs[l] : mid_w[pi][l];
      L.out_h = last ? nullptr : mid_h[pi][l];
      L.G = pl->Gl[l];
      L.tau_off = (int64_t)l * K1 * K1 * 7;
      L.n = pl->nl[l];
      L.hole = l > 0 ? 1 : 0;
      L.block_begin = blocks;
      if (D == 3 && pi == 1)
        blocks += (int)((L.n / kSepCol) * ceil_div((int64_t)L.n * L.n, kSepLanes));
      else
        blocks += (int)ceil_div(L.G, kSepLanes);
    }
    const dim3 grid((unsigned)blocks, pl->C);
    const SepGroup* gp = groups + t->group_off[pi];
    const int kind = first ? 0 : (last ? 2 : 1);
    const size_t lds = first ? (size_t)(kSepLanes + 2 * kHalo) * (pl->Ppad + 1) * es
                             : (last ? (size_t)kSepLanes * (pl->Ppad + 1) * es : 0);
    fc2t2_status st;
    switch (K1) {
      case 2: st = sep_launch<T, 2>(D, kind, grid, lds, s, b, gp, tau); break;
      case 3: st = sep_launch<T, 3>(D, kind, grid, lds, s, b, gp, tau); break;
      case 4: st = sep_launch<T, 4>(D, kind, grid, lds, s, b, gp, tau); break;
      case 5: st = sep_launch<T, 5>(D, kind, grid, lds, s, b, gp, tau); break;
      case 6: st = sep_launch<T, 6>(D, kind, grid, lds, s, b, gp, tau); break;
      case 7: st = sep_launch<T, 7>(D, kind, grid, lds, s, b, gp, tau); break;
      default: st = FC2T2_EUNSUPPORTED;
    }
    if (st) return st;
  }
  return FC2T2_OK;
}

fc2t2_status launch_m2l_separable(const fc2t2_plan_s* pl, const void* const* ins, void* const* outs, bool transpose,
                                  void* ws, hipStream_t s) {
  if (!pl->sep || !ws) return FC2T2_EUNSUPPORTED;
  return pl->io == FC2T2_IO_F64 ? sep_run<double>(pl, ins, outs, transpose, ws, s)
                                : sep_run<float>(pl, ins, outs, transpose, ws, s);
}

}  // namespace fc2t2

// Grid-to-grid stages of the multilevel expansion (section 3):
//   up-shift    out[I]    = sum_b S_b in[2I + b]     M2M, and the transpose of L2L
//   down-shift  out[2I+b] = S_b^T in[I]              L2L, and the transpose of M2M
// (section 3, the binomial M2M shift and the Taylor L2L shift)
//   M2L         L[i] = sum_o T(o) M[i + o] over the parity window minus the hole
//   M2L^T       G_M[j] = sum_o T(o)^T G_L[j - o] over the same pairs
// S_b are the cell-scaled binomial shift matrices S_b[n][m] = 2^-|n| (b - 1/2)^(n-m)/(n-m)!
// (identical at every level in scaled units), T the per-level derivative tensors.
//
// Admissible offsets o = j - i at a level (target i, source j): per dimension
// o_d in [-2, 3] when i_d is even and [-3, 2] when odd (children of the parent's
// neighbours), j inside the grid, and max |o_d| > 1 above the finest level (the hole is
// filled by the finer levels).
#include <math.h>

#include <vector>

#include "plan.h"

using namespace fc2t2;

namespace {

template <int D>
__device__ __forceinline__ void decode(int64_t lin, int n, int (&c)[3]) {
  c[0] = c[1] = c[2] = 0;
#pragma unroll
  for (int j = D - 1; j >= 0; --j) { c[j] = (int)(lin % n); lin /= n; }
}

template <int D>
__device__ __forceinline__ int64_t encode(const int (&c)[3], int n) {
  int64_t lin = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) lin = lin * n + c[j];
  return lin;
}

// ---------------------------------------------------------------------------------------
// Shifts between a parent and its 2^d children in cell-scaled units.  With the child
// offset e = (b - 1/2) h_child (b in {0,1}^d), the scaled shift matrix factors as
//   S_b[n][m] = c[n][m] * sigma_b(n - m),
//   c[n][m] = 2^(-|n| - |n-m|) / prod_j (n_j - m_j)!,   sigma_b(d) = prod_j (-1)^(d_j (1 - b_j)),
// and sigma depends on d only through its parity pattern pi = d mod 2, so
//   sigma_b(pi) = (-1)^popcount(pi & ~b).
// The sign sums over the children are therefore a Walsh-Hadamard transform of size 2^d:
//   up:   out[n] = sum_{m <= n} c[n][m] H[pi(n-m)][m],  H[pi][m] = sum_b sigma_b(pi) child_b[m]
//   down: child_b[k] = sum_pi sigma_b(pi) G[pi][k],     G[pi][k] = sum_{m >= k, pi(m-k) = pi} c[m][k] in[m]
// which costs one multiply-add per (output, list entry) plus d 2^(d-1) butterflies per
// coefficient, instead of 2^d multiply-adds per list entry.
//
// Several levels run in one launch: a block owns a tile of 2^f x .. x 2^f cells at the
// finer level l0 and the 2^(f-j)-wide tiles above it at levels l0 + j (the subtree of one
// cell at level l0 + f); the intermediate tiles stay in LDS.

struct ShiftEntry {
  double c;
  int m;
  int pi;
};

struct LevelPtrs {
  void* p[kMaxLevels];
  uint8_t* occ[kMaxLevels];   // per-level occupancy (up chain only; null entries: not tracked)
  int has_occ;
  int gen;                     // occupied <=> byte == gen
};

constexpr int kShiftThreads = 256;
constexpr int kMaxShiftEntries = 2048;
constexpr size_t kShiftLds = 64 * 1024;

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// x[pi] <- sum_b (-1)^popcount(pi & b) x[b]  (Sylvester-ordered Hadamard butterflies)
template <int D, typename T>
__device__ __forceinline__ void hadamard(T (&x)[1 << D]) {
#pragma unroll
  for (int st = 1; st < (1 << D); st <<= 1)
#pragma unroll
    for (int i = 0; i < (1 << D); ++i)
      if (!(i & st)) {
        const T a = x[i], b = x[i | st];
        x[i] = a + b;
        x[i | st] = a - b;
      }
}

// The same transform across the NB = 2^D consecutive lanes of a group, one value per lane:
// lane pi of the group ends with sum_q (-1)^popc(pi & q) x_q.  Every lane of the wave must
// take part (groups are aligned and whole).
template <int D, typename T>
__device__ __forceinline__ T hadamard_lanes(T v, int pi) {
#pragma unroll
  for (int st = 1; st < (1 << D); st <<= 1) {
    const T o = __shfl_xor(v, st);
    v = (pi & st) ? o - v : v + o;
  }
  return v;
}

// Coordinates of local index p in a tile of side 2^lg (last dimension fastest).
template <int D>
__device__ __forceinline__ void tile_coords(uint32_t p, int lg, uint32_t (&c)[3]) {
  const uint32_t mask = (1u << lg) - 1u;
  c[0] = c[1] = c[2] = 0;
#pragma unroll
  for (int j = D - 1; j >= 0; --j) { c[j] = p & mask; p >>= lg; }
}
template <int D>
__device__ __forceinline__ uint32_t tile_lin(const uint32_t (&c)[3], int lg) {
  uint32_t lin = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) lin = (lin << lg) | c[j];
  return lin;
}
// Child b of a cell with coordinates c (bit D-1-j of b is the offset along dimension j).
template <int D>
__device__ __forceinline__ void child_coords(const uint32_t (&c)[3], int b, uint32_t (&cc)[3]) {
  cc[0] = cc[1] = cc[2] = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) cc[j] = 2 * c[j] + ((b >> (D - 1 - j)) & 1);
}

// Up-shift chain: levels l0+1 .. l0+f from level l0.  grids.p[l] is the level-l grid
// [C][G_l][P_pad]; lg0 = log2 of the level-l0 side.  Every produced level is written out
// (padding coefficients as zero).
template <class S, typename T>
__global__ void __launch_bounds__(kShiftThreads) upchain_kernel(LevelPtrs grids, const ShiftEntry* __restrict__ tab,
                                                                const int* __restrict__ beg, int n_entries, int l0,
                                                                int f, int lg0) {
  constexpr int D = S::D, P = S::P, PP = S::Ppad, NB = 1 << D;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  T* s_coef = reinterpret_cast<T*>(smem);
  int* s_off = reinterpret_cast<int*>(s_coef + n_entries);
  int* s_beg = s_off + n_entries;
  T* hbuf = reinterpret_cast<T*>(smem + align16((size_t)n_entries * (sizeof(T) + sizeof(int)) + (P + 1) * sizeof(int)));
  T* obuf = hbuf + ((size_t)PP << (f * D));
  uint8_t* s_occ = reinterpret_cast<uint8_t*>(obuf + ((size_t)PP << ((f - 1) * D)));   // 2 x 2^((f-1)D) bytes
  const uint32_t occ_half = 1u << ((f - 1) * D);
  const int tid = threadIdx.x, ch = blockIdx.y;
  for (int i = tid; i < n_entries; i += kShiftThreads) {
    const ShiftEntry e = tab[i];
    s_coef[i] = (T)e.c;
    s_off[i] = e.pi * PP + e.m;
  }
  for (int i = tid; i <= P; i += kShiftThreads) s_beg[i] = beg[i];
  uint32_t tc[3];
  tile_coords<D>(blockIdx.x, lg0 - f, tc);
  for (int j = 1; j <= f; ++j) {
    const int lgp = f - j;                         // log2 parent tile side
    const uint32_t npar = 1u << (lgp * D);
    const int lgn_c = lg0 - j + 1, lgn_p = lg0 - j;  // log2 level sides (children, parents)
    const T* cin = (const T*)grids.p[l0 + j - 1] + ((size_t)ch << (lgn_c * D)) * PP;
    // stage H[p][pi][m]
    for (uint32_t idx = tid; idx < npar * PP; idx += kShiftThreads) {
      const uint32_t p = idx / PP, m = idx - p * PP;
      uint32_t pc[3], cc[3];
      tile_coords<D>(p, lgp, pc);
      T x[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        child_coords<D>(pc, b, cc);
        T v;
        if (j == 1) {
          uint32_t gc[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) gc[d] = (tc[d] << (lgp + 1)) + cc[d];
          v = cin[(size_t)tile_lin<D>(gc, lgn_c) * PP + m];
        } else {
          v = obuf[(size_t)tile_lin<D>(cc, lgp + 1) * PP + m];
        }
        x[NB - 1 - b] = v;
      }
      hadamard<D>(x);
#pragma unroll
      for (int pi = 0; pi < NB; ++pi) hbuf[((size_t)p * NB + pi) * PP + m] = x[pi];
    }
    if (grids.has_occ && ch == 0) {
      // occupancy of the parents: OR over their children
      const uint8_t* prev = s_occ + ((j + 1) & 1) * occ_half;
      uint8_t* cur = s_occ + (j & 1) * occ_half;
      for (uint32_t p = tid; p < npar; p += kShiftThreads) {
        uint32_t pc[3], cc[3], gc[3];
        tile_coords<D>(p, lgp, pc);
        uint8_t o = 0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          child_coords<D>(pc, b, cc);
          if (j == 1) {
#pragma unroll
            for (int d = 0; d < 3; ++d) gc[d] = (tc[d] << (lgp + 1)) + cc[d];
            o |= grids.occ[l0][tile_lin<D>(gc, lgn_c)] == grids.gen ? 1 : 0;
          } else {
            o |= prev[tile_lin<D>(cc, lgp + 1)];
          }
        }
        cur[p] = o;
#pragma unroll
        for (int d = 0; d < 3; ++d) gc[d] = (tc[d] << lgp) + pc[d];
        grids.occ[l0 + j][tile_lin<D>(gc, lgn_p)] = o ? (uint8_t)grids.gen : (uint8_t)0;
      }
    }
    __syncthreads();
    T* out = (T*)grids.p[l0 + j] + ((size_t)ch << (lgn_p * D)) * PP;
    for (uint32_t idx = tid; idx < npar * PP; idx += kShiftThreads) {
      const uint32_t p = idx / PP, n = idx - p * PP;
      T acc = T(0);
      if (n < P) {
        const T* h = hbuf + (size_t)p * NB * PP;
        for (int e = s_beg[n]; e < s_beg[n + 1]; ++e) acc += s_coef[e] * h[s_off[e]];
      }
      if (j < f) obuf[idx] = acc;
      uint32_t pc[3], gc[3];
      tile_coords<D>(p, lgp, pc);
#pragma unroll
      for (int d = 0; d < 3; ++d) gc[d] = (tc[d] << lgp) + pc[d];
      out[(size_t)tile_lin<D>(gc, lgn_p) * PP + n] = acc;
    }
    __syncthreads();
  }
}

// Down-shift chain: from level l0+f down to level l0, each finer level accumulating onto what
// its grid holds: grid[l] <- grid[l] + down-shift(grid[l+1]).  Only level l0 is written; the
// intermediate levels stay in LDS.  beg holds NB+1 list offsets per k (lists grouped by pi).
// The block first loads the top cell and the tile's rows of every level below it (what the
// finer levels already hold) into LDS in one pass, so the level steps touch no global memory
// until the final write.
//
// Levels above l0+f (up to l_top, the coarsest) are not taken from a previous launch: each
// block first walks its own ancestor chain down from l_top, one cell per level, so the whole
// down pass is one launch.
template <class S, typename T>
__global__ void __launch_bounds__(kShiftThreads) downchain_kernel(LevelPtrs grids, const ShiftEntry* __restrict__ tab,
                                                                  const int* __restrict__ beg, int n_entries, int l0,
                                                                  int f, int lg0, int l_top) {
  constexpr int D = S::D, P = S::P, PP = S::Ppad, NB = 1 << D;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  T* s_coef = reinterpret_cast<T*>(smem);
  int* s_m = reinterpret_cast<int*>(s_coef + n_entries);
  int* s_beg = s_m + n_entries;
  T* buf0 = reinterpret_cast<T*>(smem + align16((size_t)n_entries * (sizeof(T) + sizeof(int)) + P * (NB + 1) * sizeof(int)));
  const size_t buf_elems = (size_t)PP << ((f - 1) * D);
  T* buf1 = buf0 + buf_elems;
  T* own = buf1 + buf_elems;   // rows of levels l0+f-1 .. l0 of the tile, level by level
  const int tid = threadIdx.x, ch = blockIdx.y;
  for (int i = tid; i < n_entries; i += kShiftThreads) {
    const ShiftEntry e = tab[i];
    s_coef[i] = (T)e.c;
    s_m[i] = e.m;
  }
  for (int i = tid; i < P * (NB + 1); i += kShiftThreads) s_beg[i] = beg[i];
  uint32_t tc[3];
  tile_coords<D>(blockIdx.x, lg0 - f, tc);
  {
    // the tile's top cell at level l0 + f, or its ancestor at l_top to walk down from
    const int la = l_top > l0 + f ? l_top : l0 + f;
    const int lgn = lg0 - la;
    uint32_t ac[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) ac[d] = tc[d] >> (la - l0 - f);
    const T* top = (const T*)grids.p[la] + (((size_t)ch << (lgn * D)) + tile_lin<D>(ac, lgn)) * PP;
    for (int i = tid; i < PP; i += kShiftThreads) buf0[i] = top[i];
  }
  // ancestor walk: buf0 holds the final row of the ancestor at level l+1; make level l's
  for (int l = l_top - 1; l >= l0 + f; --l) {
    __syncthreads();
    const int lgn = lg0 - l;
    uint32_t ac[3];
    int b = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) ac[d] = tc[d] >> (l - l0 - f);
#pragma unroll
    for (int d = 0; d < D; ++d) b = (b << 1) | (int)(ac[d] & 1u);
    const T* own_row = (const T*)grids.p[l] + (((size_t)ch << (lgn * D)) + tile_lin<D>(ac, lgn)) * PP;
    // thread (k, pi): one parity pattern's sum; the lanes' transform gives the child's value
    // in lane NB - 1 - b of the group
    constexpr int kRounds = (P * NB + kShiftThreads - 1) / kShiftThreads;
    T v[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int t = tid + r * kShiftThreads;
      const int pi = t & (NB - 1), k = t / NB;
      T a = T(0);
      if (k < P)
        for (int e = s_beg[k * (NB + 1) + pi]; e < s_beg[k * (NB + 1) + pi + 1]; ++e) a += s_coef[e] * buf0[s_m[e]];
      a = hadamard_lanes<D>(a, pi);
      v[r] = (k < P && pi == NB - 1 - b) ? own_row[k] + a : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int t = tid + r * kShiftThreads;
      const int pi = t & (NB - 1), k = t / NB;
      if (k < P && pi == NB - 1 - b) buf0[k] = v[r];
    }
  }
  {
    size_t off = 0;
    for (int j = 1; j <= f; ++j) {
      const int lgn_c = lg0 - f + j;
      const T* src = (const T*)grids.p[l0 + f - j] + ((size_t)ch << (lgn_c * D)) * PP;
      const uint32_t cnt = (1u << (j * D)) * PP;
#pragma unroll 4
      for (uint32_t idx = tid; idx < cnt; idx += kShiftThreads) {
        const uint32_t c = idx / PP, k = idx - c * PP;
        uint32_t cc[3], gc[3];
        tile_coords<D>(c, j, cc);
#pragma unroll
        for (int d = 0; d < 3; ++d) gc[d] = (tc[d] << j) + cc[d];
        own[off + idx] = src[(size_t)tile_lin<D>(gc, lgn_c) * PP + k];
      }
      off += cnt;
    }
  }
  __syncthreads();
  size_t own_off = 0;
  for (int j = 1; j <= f; ++j) {
    const int lgp = j - 1;                          // log2 parent tile side
    const uint32_t npar = 1u << (lgp * D);
    const int lc = l0 + f - j;                      // child level
    const int lgn_c = lg0 - f + j;
    const T* pin = (j & 1) ? buf0 : buf1;
    T* cout_lds = (j & 1) ? buf1 : buf0;
    const T* cown = own + own_off;
    T* cg = (T*)grids.p[lc] + ((size_t)ch << (lgn_c * D)) * PP;
    // thread (p, k, pi): one parity pattern's sum over the parent row; after the lanes'
    // transform, lane pi holds the value of child NB - 1 - pi.  The trip count is uniform so
    // every lane takes part in the exchange.
    const uint32_t work = npar * P * NB;
    for (uint32_t t0 = 0; t0 < work; t0 += kShiftThreads) {
      const uint32_t t = t0 + tid;
      const bool valid = t < work;
      const int pi = (int)(t & (NB - 1));
      const uint32_t pk = t / NB;
      const uint32_t p = pk / P, k = pk - p * P;
      T a = T(0);
      if (valid) {
        const T* row = pin + (size_t)p * PP;
        for (int e = s_beg[k * (NB + 1) + pi]; e < s_beg[k * (NB + 1) + pi + 1]; ++e) a += s_coef[e] * row[s_m[e]];
      }
      a = hadamard_lanes<D>(a, pi);
      if (valid) {
        uint32_t pc[3], cc[3];
        tile_coords<D>(p, lgp, pc);
        child_coords<D>(pc, NB - 1 - pi, cc);
        const uint32_t cl = tile_lin<D>(cc, lgp + 1);
        const T v = cown[(size_t)cl * PP + k] + a;
        if (j < f) {
          cout_lds[(size_t)cl * PP + k] = v;
        } else {
          uint32_t gc[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) gc[d] = (tc[d] << (lgp + 1)) + cc[d];
          cg[(size_t)tile_lin<D>(gc, lgn_c) * PP + k] = v;
        }
      }
    }
    own_off += (size_t)(1u << (j * D)) * PP;
    __syncthreads();
  }
}

__device__ __forceinline__ bool offset_ok(int i, int o, int n_l) {
  const bool in_win = (i & 1) ? (o >= -3 && o <= 2) : (o >= -2 && o <= 3);
  return in_win && i + o >= 0 && i + o < n_l;
}

// L[ch][i][k] (+)= sum_o sum_n T[o][n][k] M[ch][i+o][n]; one thread per (target, k).
template <int D, typename T>
__global__ void __launch_bounds__(256) m2l_kernel(const T* __restrict__ M, T* __restrict__ L,
                                                  const T* __restrict__ Tl, int P, int Ppad, int n_l,
                                                  int64_t G_l, int finest, int accumulate) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= G_l * Ppad) return;
  const int ch = blockIdx.y;
  const int k = (int)(tid % Ppad);
  const int64_t i = tid / Ppad;
  T acc = T(0);
  if (k < P) {
    int ci[3];
    decode<D>(i, n_l, ci);
    const int z_lo = D == 3 ? -3 : 0, z_hi = D == 3 ? 3 : 0;
    for (int o0 = -3; o0 <= 3; ++o0) {
      if (!offset_ok(ci[0], o0, n_l)) continue;
      for (int o1 = -3; o1 <= 3; ++o1) {
        if (!offset_ok(ci[1], o1, n_l)) continue;
        for (int o2 = z_lo; o2 <= z_hi; ++o2) {
          if (D == 3 && !offset_ok(ci[2], o2, n_l)) continue;
          const int am = max(max(abs(o0), abs(o1)), abs(o2));
          if (!finest && am <= 1) continue;
          int cj[3] = {ci[0] + o0, ci[1] + o1, ci[2] + o2};
          const int oi = D == 2 ? (o0 + 3) * 7 + (o1 + 3) : ((o0 + 3) * 7 + (o1 + 3)) * 7 + (o2 + 3);
          const T* __restrict__ src = M + ((int64_t)ch * G_l + encode<D>(cj, n_l)) * Ppad;
          const T* __restrict__ To = Tl + (int64_t)oi * P * Ppad + k;
          for (int nn = 0; nn < P; ++nn) acc += To[(int64_t)nn * Ppad] * src[nn];
        }
      }
    }
  }
  T* dst = L + ((int64_t)ch * G_l + i) * Ppad + k;
  if (accumulate) *dst += acc; else *dst = acc;
}

// GM[ch][j][n] (+)= sum_o sum_k T[o][n][k] GL[ch][j-o][k]; one thread per (source, n).
template <int D, typename T>
__global__ void __launch_bounds__(256) m2l_T_kernel(const T* __restrict__ GL, T* __restrict__ GM,
                                                    const T* __restrict__ Tl, int P, int Ppad, int n_l,
                                                    int64_t G_l, int finest, int accumulate) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= G_l * Ppad) return;
  const int ch = blockIdx.y;
  const int nn = (int)(tid % Ppad);
  const int64_t j = tid / Ppad;
  T acc = T(0);
  if (nn < P) {
    int cj[3];
    decode<D>(j, n_l, cj);
    const int z_lo = D == 3 ? -3 : 0, z_hi = D == 3 ? 3 : 0;
    for (int o0 = -3; o0 <= 3; ++o0) {
      const int i0 = cj[0] - o0;
      if (i0 < 0 || i0 >= n_l || !offset_ok(i0, o0, n_l)) continue;
      for (int o1 = -3; o1 <= 3; ++o1) {
        const int i1 = cj[1] - o1;
        if (i1 < 0 || i1 >= n_l || !offset_ok(i1, o1, n_l)) continue;
        for (int o2 = z_lo; o2 <= z_hi; ++o2) {
          const int i2 = cj[2] - o2;
          if (D == 3 && (i2 < 0 || i2 >= n_l || !offset_ok(i2, o2, n_l))) continue;
          const int am = max(max(abs(o0), abs(o1)), abs(o2));
          if (!finest && am <= 1) continue;
          int ci[3] = {i0, i1, D == 3 ? i2 : 0};
          const int oi = D == 2 ? (o0 + 3) * 7 + (o1 + 3) : ((o0 + 3) * 7 + (o1 + 3)) * 7 + (o2 + 3);
          const T* __restrict__ src = GL + ((int64_t)ch * G_l + encode<D>(ci, n_l)) * Ppad;
          const T* __restrict__ To = Tl + ((int64_t)oi * P + nn) * Ppad;
          for (int k = 0; k < P; ++k) acc += To[k] * src[k];
        }
      }
    }
  }
  T* dst = GM + ((int64_t)ch * G_l + j) * Ppad + nn;
  if (accumulate) *dst += acc; else *dst = acc;
}

template <typename T>
const T* level_tensor(const fc2t2_plan_s* pl, int lvl) {
  return (const T*)pl->m2l_T + (size_t)lvl * pl->n_off * pl->P * pl->Ppad;
}

}  // namespace

namespace fc2t2 {

// Host: the sparse shift lists (see above), laid out as [up lists | down lists] entries
// followed by the begin offsets of both.
fc2t2_status build_shift_tables(fc2t2_plan_s* pl, hipStream_t s) {
  const int P = pl->P, dim = pl->dim;
  std::vector<int> e((size_t)P * 3);
  mi_fill(dim, pl->K, reinterpret_cast<int(*)[3]>(e.data()));
  std::vector<ShiftEntry> up, down;
  std::vector<int> beg_up(P + 1), beg_down((size_t)P * ((1 << dim) + 1));
  auto le = [&](int a, int c) {   // multi-index c <= a componentwise
    return e[3 * c] <= e[3 * a] && e[3 * c + 1] <= e[3 * a + 1] && e[3 * c + 2] <= e[3 * a + 2];
  };
  auto coef = [&](int hi, int lo) {
    double v = 1.0;
    int tot = 0;
    for (int j = 0; j < 3; ++j) {
      const int d = e[3 * hi + j] - e[3 * lo + j];
      for (int i = 2; i <= d; ++i) v /= i;
      tot += e[3 * hi + j] + d;
    }
    return ldexp(v, -tot);
  };
  auto parity = [&](int hi, int lo) {
    int pi = 0;
    for (int j = 0; j < dim; ++j) pi = (pi << 1) | ((e[3 * hi + j] - e[3 * lo + j]) & 1);
    return pi;
  };
  for (int n = 0; n < P; ++n) {
    beg_up[n] = (int)up.size();
    for (int m = 0; m < P; ++m)
      if (le(n, m)) up.push_back(ShiftEntry{coef(n, m), m, parity(n, m)});
  }
  beg_up[P] = (int)up.size();
  const int NB = 1 << dim;
  for (int k = 0; k < P; ++k) {
    for (int pi = 0; pi < NB; ++pi) {
      beg_down[k * (NB + 1) + pi] = (int)down.size();
      for (int m = 0; m < P; ++m)
        if (le(m, k) && parity(m, k) == pi) down.push_back(ShiftEntry{coef(m, k), m, pi});
    }
    beg_down[k * (NB + 1) + NB] = (int)down.size();
  }
  std::vector<ShiftEntry> all(up);
  all.insert(all.end(), down.begin(), down.end());
  pl->shift_n_up = (int)up.size();
  pl->shift_n_down = (int)down.size();
  if (up.size() > (size_t)kMaxShiftEntries || down.size() > (size_t)kMaxShiftEntries) return FC2T2_EUNSUPPORTED;
  std::vector<int> begs(beg_up);
  begs.insert(begs.end(), beg_down.begin(), beg_down.end());
  const size_t tab_bytes = align256(all.size() * sizeof(ShiftEntry));
  const size_t bytes = tab_bytes + align256(begs.size() * sizeof(int));
  if (hipMalloc(&pl->shift, bytes) != hipSuccess) { pl->shift = nullptr; return FC2T2_ENOMEM; }
  if (hipMemcpyAsync(pl->shift, all.data(), all.size() * sizeof(ShiftEntry), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync((char*)pl->shift + tab_bytes, begs.data(), begs.size() * sizeof(int), hipMemcpyHostToDevice, s) !=
          hipSuccess)
    return FC2T2_EHIP;
  pl->shift_beg_off = tab_bytes;
  return hipStreamSynchronize(s) == hipSuccess ? FC2T2_OK : FC2T2_EHIP;
}

}  // namespace fc2t2

namespace {

struct ShiftSeg {
  int l0, f;
  int l_top = 0;   // down pass: level the blocks start from (above l0 + f: ancestor walk)
};

size_t upchain_lds(const fc2t2_plan_s* pl, int f) {
  const int D = pl->dim;
  const size_t es = io_size(pl);
  return align16((size_t)pl->shift_n_up * (es + sizeof(int)) + (pl->P + 1) * sizeof(int)) +
         (((size_t)pl->Ppad << (f * D)) + ((size_t)pl->Ppad << ((f - 1) * D))) * es + (size_t(2) << ((f - 1) * D));
}
size_t downchain_lds(const fc2t2_plan_s* pl, int f) {
  const int D = pl->dim;
  const size_t es = io_size(pl);
  size_t own = 0;
  for (int j = 1; j <= f; ++j) own += (size_t)pl->Ppad << (j * D);
  return align16((size_t)pl->shift_n_down * (es + sizeof(int)) + (size_t)pl->P * ((1 << D) + 1) * sizeof(int)) +
         (2 * ((size_t)pl->Ppad << ((f - 1) * D)) + own) * es;
}

// Level segments [l0, l0 + f] of the pyramid, one launch each.  A small level (at most 4096
// cells) finishes the pyramid in one launch; below that, a segment is as deep as the LDS
// budget allows while leaving at least 1024 tiles (four per compute unit).
int shift_segments(const fc2t2_plan_s* pl, ShiftSeg* seg) {
  const int D = pl->dim, L = pl->levels;
  auto fits = [&](int f) { return upchain_lds(pl, f) <= kShiftLds && downchain_lds(pl, f) <= kShiftLds; };
  int ns = 0, l0 = 0;
  while (l0 + 1 < L) {
    const int rem = L - 1 - l0, lgn = lg2i(pl->nl[l0]);
    int f = 0;
    if (pl->Gl[l0] <= 4096 && rem <= lgn && fits(rem)) {
      f = rem;
    } else {
      for (int g = 1; g <= rem && g <= lgn && fits(g); ++g) {
        if (((int64_t)1 << ((lgn - g) * D)) < 1024) break;
        f = g;
      }
      if (f == 0) f = 1;
    }
    seg[ns++] = ShiftSeg{l0, f, l0 + f};
    l0 += f;
  }
  return ns;
}

template <class S, typename T>
fc2t2_status chain_launch(const fc2t2_plan_s* pl, const ShiftSeg& sg, void* const* grids, bool up, hipStream_t s,
                          uint8_t* const* occ, uint8_t gen) {
  LevelPtrs g{};
  for (int l = 0; l < pl->levels; ++l) {
    g.p[l] = grids[l];
    g.occ[l] = occ ? occ[l] : nullptr;
  }
  g.has_occ = (up && occ) ? 1 : 0;
  g.gen = gen;
  const int lgn = lg2i(pl->nl[sg.l0]);
  const dim3 grid(1u << ((lgn - sg.f) * S::D), pl->C);
  const int* begs = (const int*)((const char*)pl->shift + pl->shift_beg_off);
  const ShiftEntry* tab = (const ShiftEntry*)pl->shift;
  if (up) {
    const size_t smem = upchain_lds(pl, sg.f);
    hipLaunchKernelGGL((upchain_kernel<S, T>), grid, dim3(kShiftThreads), smem, s, g, tab, begs, pl->shift_n_up, sg.l0,
                       sg.f, lgn);
  } else {
    const size_t smem = downchain_lds(pl, sg.f);
    hipLaunchKernelGGL((downchain_kernel<S, T>), grid, dim3(kShiftThreads), smem, s, g, tab + pl->shift_n_up,
                       begs + (pl->P + 1), pl->shift_n_down, sg.l0, sg.f, lgn, sg.l_top);
  }
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

fc2t2_status shift_pyramid(const fc2t2_plan_s* pl, void* const* grids, bool up, hipStream_t s,
                           uint8_t* const* occ, uint8_t gen) {
  ShiftSeg seg[kMaxLevels];
  int ns = shift_segments(pl, seg);
  int walk_from = -1;   // down pass: segment whose blocks walk their ancestors up to the top
  if (!up) {
    // the coarsest segments fold into the first one (from the top) with at most 4096 blocks:
    // its blocks each recompute their single-cell ancestor chain instead of a launch per segment
    for (int i = 0; i < ns; ++i) {
      const int64_t blocks = (int64_t)1 << ((lg2i(pl->nl[seg[i].l0]) - seg[i].f) * pl->dim);
      if (blocks <= 4096) {
        walk_from = i;
        break;
      }
    }
    if (walk_from >= 0) ns = walk_from + 1;
  }
  for (int i = 0; i < ns; ++i) {
    ShiftSeg sg = seg[up ? i : ns - 1 - i];
    sg.l_top = (!up && walk_from >= 0 && (ns - 1 - i) == walk_from) ? pl->levels - 1 : sg.l0 + sg.f;
    if ((up ? upchain_lds(pl, sg.f) : downchain_lds(pl, sg.f)) > kShiftLds) return FC2T2_EUNSUPPORTED;
    fc2t2_status st = FC2T2_EUNSUPPORTED;
    dispatch_shape(pl->dim, pl->K, [&](auto sh) {
      using S = decltype(sh);
      st = pl->io == FC2T2_IO_F64 ? chain_launch<S, double>(pl, sg, grids, up, s, occ, gen)
                                  : chain_launch<S, float>(pl, sg, grids, up, s, occ, gen);
    });
    if (st) return st;
  }
  return FC2T2_OK;
}

}  // namespace

namespace fc2t2 {

// Up-shift pass: grids[l + 1] = up-shift(grids[l]) for l = 0 .. levels-2.
fc2t2_status upshift_pyramid(const fc2t2_plan_s* pl, void* const* grids, hipStream_t s, uint8_t* const* occ,
                             uint8_t gen) {
  return shift_pyramid(pl, grids, true, s, occ, gen);
}

// Down-shift pass: grids[l] += down-shift(grids[l + 1]) for l = levels-2 .. 0.
fc2t2_status downshift_pyramid(const fc2t2_plan_s* pl, void* const* grids, hipStream_t s) {
  return shift_pyramid(pl, grids, false, s, nullptr, 0);
}

fc2t2_status launch_m2l(const fc2t2_plan_s* pl, int lvl, const void* M, void* L, bool accumulate,
                        hipStream_t s) {
  if (m2l_is_mfma(pl)) {
    const void* ins[kMaxLevels] = {};
    void* outs[kMaxLevels] = {};
    ins[lvl] = M;
    outs[lvl] = L;
    return launch_m2l_mfma(pl, lvl, lvl + 1, ins, outs, accumulate, false, s);
  }
  const int64_t work = pl->Gl[lvl] * pl->Ppad;
  const dim3 grid((unsigned)ceil_div(work, 256), pl->C);
  const int fin = lvl == 0, acc = accumulate ? 1 : 0;
  if (pl->io == FC2T2_IO_F64) {
    if (pl->dim == 2)
      hipLaunchKernelGGL((m2l_kernel<2, double>), grid, dim3(256), 0, s, (const double*)M, (double*)L, level_tensor<double>(pl, lvl), pl->P, pl->Ppad, pl->nl[lvl], pl->Gl[lvl], fin, acc);
    else
      hipLaunchKernelGGL((m2l_kernel<3, double>), grid, dim3(256), 0, s, (const double*)M, (double*)L, level_tensor<double>(pl, lvl), pl->P, pl->Ppad, pl->nl[lvl], pl->Gl[lvl], fin, acc);
  } else {
    if (pl->dim == 2)
      hipLaunchKernelGGL((m2l_kernel<2, float>), grid, dim3(256), 0, s, (const float*)M, (float*)L, level_tensor<float>(pl, lvl), pl->P, pl->Ppad, pl->nl[lvl], pl->Gl[lvl], fin, acc);
    else
      hipLaunchKernelGGL((m2l_kernel<3, float>), grid, dim3(256), 0, s, (const float*)M, (float*)L, level_tensor<float>(pl, lvl), pl->P, pl->Ppad, pl->nl[lvl], pl->Gl[lvl], fin, acc);
  }
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

fc2t2_status launch_m2l_T(const fc2t2_plan_s* pl, int lvl, const void* GL, void* GM, bool accumulate,
                          hipStream_t s) {
  if (m2l_is_mfma(pl)) {
    const void* ins[kMaxLevels] = {};
    void* outs[kMaxLevels] = {};
    ins[lvl] = GL;
    outs[lvl] = GM;
    return launch_m2l_mfma(pl, lvl, lvl + 1, ins, outs, accumulate, true, s);
  }
  const int64_t work = pl->Gl[lvl] * pl->Ppad;
  const dim3 grid((unsigned)ceil_div(work, 256), pl->C);
  const int fin = lvl == 0, acc = accumulate ? 1 : 0;
  if (pl->io == FC2T2_IO_F64) {
    if (pl->dim == 2)
      hipLaunchKernelGGL((m2l_T_kernel<2, double>), grid, dim3(256), 0, s, (const double*)GL, (double*)GM, level_tensor<double>(pl, lvl), pl->P, pl->Ppad, pl->nl[lvl], pl->Gl[lvl], fin, acc);
    else
      hipLaunchKernelGGL((m2l_T_kernel<3, double>), grid, dim3(256), 0, s, (const double*)GL, (double*)GM, level_tensor<double>(pl, lvl), pl->P, pl->Ppad, pl->nl[lvl], pl->Gl[lvl], fin, acc);
  } else {
    if (pl->dim == 2)
      hipLaunchKernelGGL((m2l_T_kernel<2, float>), grid, dim3(256), 0, s, (const float*)GL, (float*)GM, level_tensor<float>(pl, lvl), pl->P, pl->Ppad, pl->nl[lvl], pl->Gl[lvl], fin, acc);
    else
      hipLaunchKernelGGL((m2l_T_kernel<3, float>), grid, dim3(256), 0, s, (const float*)GL, (float*)GM, level_tensor<float>(pl, lvl), pl->P, pl->Ppad, pl->nl[lvl], pl->Gl[lvl], fin, acc);
  }
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

fc2t2_status launch_m2l_all(const fc2t2_plan_s* pl, const void* const* ins, void* const* outs, bool transpose,
                            hipStream_t s, const uint8_t* const* occ, uint8_t gen, void* sep_ws) {
  if (m2l_is_mfma(pl))
    return launch_m2l_mfma(pl, 0, pl->levels, ins, outs, false, transpose, s, occ, gen);
  if (pl->prec == FC2T2_M2L_SEPARABLE) return launch_m2l_separable(pl, ins, outs, transpose, sep_ws, s);
  for (int l = 0; l < pl->levels; ++l) {
    const fc2t2_status st = transpose ? launch_m2l_T(pl, l, ins[l], outs[l], false, s)
                                      : launch_m2l(pl, l, ins[l], outs[l], false, s);
    if (st) return st;
  }
  return FC2T2_OK;
}

}  // namespace fc2t2

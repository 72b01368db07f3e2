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
// and sigma depends on d only through its parity pattern pi = d mod 2.  The plan holds,
// for every multi-index, the sparse list of its (partner multi-index, parity pattern, c)
// entries: for the up-shift, n's list runs over m <= n; for the down-shift, k's list runs
// over m >= k.  One thread computes one output coefficient by walking its list and
// combining the 2^d children with the signs sigma_b(pi).

struct ShiftEntry {
  double c;
  int m;
  int pi;
};

__device__ __forceinline__ float sigma_sign(int pi, int b) {
  // (-1)^(number of dimensions j with pi_j = 1 and b_j = 0)
  return (__popc(pi & ~b) & 1) ? -1.0f : 1.0f;
}

template <int D>
__device__ __forceinline__ int64_t child_cell(const int (&pc)[3], int b, int n_child) {
  int64_t lin = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) lin = lin * n_child + (2 * pc[j] + ((b >> (D - 1 - j)) & 1));
  return lin;
}

// Both shifts run in blocks of 256 threads covering NPB = 256 / P_pad parents: the block first
// copies the sparse lists and its parents' (or children's) rows into LDS with coalesced loads,
// then each thread computes one coefficient from LDS, and the results are written coalesced.
constexpr int kShiftThreads = 256;
constexpr int kMaxShiftEntries = 2048;

template <typename T>
__device__ __forceinline__ void copy_rows_to_lds(const T* __restrict__ src, T* dst, int count) {
  for (int i = threadIdx.x; i < count; i += kShiftThreads) dst[i] = src[i];
}

// out[ch][I][n] = sum_b sum_{m <= n} S_b[n][m] in[ch][2I+b][m]; one thread per (parent, n).
template <int D, typename T>
__global__ void __launch_bounds__(kShiftThreads) upshift_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                                const ShiftEntry* __restrict__ tab,
                                                                const int* __restrict__ beg, int n_entries, int P,
                                                                int Ppad, int lg_par, uint32_t G_par,
                                                                uint32_t G_child) {
  constexpr int NB = 1 << D;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  ShiftEntry* s_tab = reinterpret_cast<ShiftEntry*>(smem);
  int* s_beg = reinterpret_cast<int*>(s_tab + n_entries);
  T* s_rows = reinterpret_cast<T*>(smem + (((size_t)n_entries * sizeof(ShiftEntry) + (P + 1) * sizeof(int) + 15) & ~size_t(15)));
  const int npb = kShiftThreads / Ppad;
  const int ch = blockIdx.y;
  const uint32_t I0 = blockIdx.x * npb;
  const int tid = threadIdx.x;
  for (int i = tid; i < n_entries; i += kShiftThreads) s_tab[i] = tab[i];
  for (int i = tid; i <= P; i += kShiftThreads) s_beg[i] = beg[i];
  // children rows of the block's parents: s_rows[p][b][:]
  const uint32_t mask = (1u << lg_par) - 1u;
  const int lg_child = lg_par + 1;
  for (int idx = tid; idx < npb * NB * Ppad; idx += kShiftThreads) {
    const int pb = idx / Ppad, k = idx - pb * Ppad;
    const int p = pb / NB, b = pb % NB;
    const uint32_t I = I0 + p;
    if (I >= G_par) continue;
    uint32_t r = I, lin = 0, pc[3] = {0, 0, 0};
#pragma unroll
    for (int j = D - 1; j >= 0; --j) { pc[j] = r & mask; r >>= lg_par; }
#pragma unroll
    for (int j = 0; j < D; ++j) lin = (lin << lg_child) | (2 * pc[j] + ((b >> (D - 1 - j)) & 1));
    s_rows[idx] = in[((size_t)ch * G_child + lin) * Ppad + k];
  }
  __syncthreads();
  const int p = tid / Ppad, nn = tid - p * Ppad;
  if (p >= npb) return;
  const uint32_t I = I0 + p;
  if (I >= G_par) return;
  T acc = T(0);
  if (nn < P) {
    const T* rows = s_rows + (size_t)p * NB * Ppad;
    for (int e = s_beg[nn]; e < s_beg[nn + 1]; ++e) {
      const ShiftEntry en = s_tab[e];
      T h = T(0);
#pragma unroll
      for (int b = 0; b < NB; ++b) h += (T)sigma_sign(en.pi, b) * rows[b * Ppad + en.m];
      acc += (T)en.c * h;
    }
  }
  out[((size_t)ch * G_par + I) * Ppad + nn] = acc;
}

// out[ch][2I+b][k] (+)= sum_{m >= k} S_b[m][k] in[ch][I][m]; one thread per (parent, k)
// producing coefficient k of all 2^d children.
template <int D, typename T>
__global__ void __launch_bounds__(kShiftThreads) downshift_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                                  const ShiftEntry* __restrict__ tab,
                                                                  const int* __restrict__ beg, int n_entries, int P,
                                                                  int Ppad, int lg_par, uint32_t G_par,
                                                                  uint32_t G_child, int accumulate) {
  constexpr int NB = 1 << D;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  ShiftEntry* s_tab = reinterpret_cast<ShiftEntry*>(smem);
  int* s_beg = reinterpret_cast<int*>(s_tab + n_entries);
  T* s_rows = reinterpret_cast<T*>(smem + (((size_t)n_entries * sizeof(ShiftEntry) + (P + 1) * sizeof(int) + 15) & ~size_t(15)));
  const int npb = kShiftThreads / Ppad;
  const int ch = blockIdx.y;
  const uint32_t I0 = blockIdx.x * npb;
  const int tid = threadIdx.x;
  for (int i = tid; i < n_entries; i += kShiftThreads) s_tab[i] = tab[i];
  for (int i = tid; i <= P; i += kShiftThreads) s_beg[i] = beg[i];
  {
    // the block's parent rows are contiguous in memory
    const uint32_t nrows = (I0 + npb <= G_par) ? (uint32_t)npb : (G_par - I0);
    copy_rows_to_lds(in + ((size_t)ch * G_par + I0) * Ppad, s_rows, (int)(nrows * Ppad));
  }
  __syncthreads();
  const int p = tid / Ppad, k = tid - p * Ppad;
  if (p >= npb) return;
  const uint32_t I = I0 + p;
  if (I >= G_par) return;
  T acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = T(0);
  if (k < P) {
    const T* row = s_rows + (size_t)p * Ppad;
    for (int e = s_beg[k]; e < s_beg[k + 1]; ++e) {
      const ShiftEntry en = s_tab[e];
      const T v = (T)en.c * row[en.m];
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] += (T)sigma_sign(en.pi, b) * v;
    }
  }
  const uint32_t mask = (1u << lg_par) - 1u;
  uint32_t r = I, pc[3] = {0, 0, 0};
#pragma unroll
  for (int j = D - 1; j >= 0; --j) { pc[j] = r & mask; r >>= lg_par; }
  const int lg_child = lg_par + 1;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    uint32_t lin = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) lin = (lin << lg_child) | (2 * pc[j] + ((b >> (D - 1 - j)) & 1));
    T* dst = out + ((size_t)ch * G_child + lin) * Ppad + k;
    if (accumulate) *dst += acc[b]; else *dst = acc[b];
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
  std::vector<int> beg_up(P + 1), beg_down(P + 1);
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
  for (int k = 0; k < P; ++k) {
    beg_down[k] = (int)down.size();
    for (int m = 0; m < P; ++m)
      if (le(m, k)) down.push_back(ShiftEntry{coef(m, k), m, parity(m, k)});
  }
  beg_down[P] = (int)down.size();
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

template <int D, typename T>
fc2t2_status shift_launch(const fc2t2_plan_s* pl, int lvl_child, const void* in, void* out, bool up,
                          bool accumulate, hipStream_t s) {
  const int lp = lvl_child + 1;
  const int npb = kShiftThreads / pl->Ppad;
  const int n_up = pl->shift_n_up, n_down = pl->shift_n_down;
  const int n_entries = up ? n_up : n_down;
  const ShiftEntry* tab = (const ShiftEntry*)pl->shift + (up ? 0 : n_up);
  const int* beg0 = (const int*)((const char*)pl->shift + pl->shift_beg_off);
  // the down-shift list offsets are stored after the up lists; rebase them to its own table
  const int* beg = up ? beg0 : beg0 + (pl->P + 1);
  const size_t rows = (size_t)npb * (up ? (1 << D) : 1) * pl->Ppad;
  const size_t smem = (((size_t)n_entries * sizeof(ShiftEntry) + (pl->P + 1) * sizeof(int) + 15) & ~size_t(15)) +
                      rows * sizeof(T);
  const dim3 grid((unsigned)ceil_div(pl->Gl[lp], npb), pl->C);
  if (up)
    hipLaunchKernelGGL((upshift_kernel<D, T>), grid, dim3(kShiftThreads), smem, s, (const T*)in, (T*)out, tab, beg,
                       n_entries, pl->P, pl->Ppad, lg2i(pl->nl[lp]), (uint32_t)pl->Gl[lp], (uint32_t)pl->Gl[lvl_child]);
  else
    hipLaunchKernelGGL((downshift_kernel<D, T>), grid, dim3(kShiftThreads), smem, s, (const T*)in, (T*)out, tab, beg,
                       n_entries, pl->P, pl->Ppad, lg2i(pl->nl[lp]), (uint32_t)pl->Gl[lp], (uint32_t)pl->Gl[lvl_child],
                       accumulate ? 1 : 0);
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

fc2t2_status launch_upshift(const fc2t2_plan_s* pl, int lvl_child, const void* in, void* out,
                            hipStream_t s) {
  if (pl->io == FC2T2_IO_F64)
    return pl->dim == 2 ? shift_launch<2, double>(pl, lvl_child, in, out, true, false, s)
                        : shift_launch<3, double>(pl, lvl_child, in, out, true, false, s);
  return pl->dim == 2 ? shift_launch<2, float>(pl, lvl_child, in, out, true, false, s)
                      : shift_launch<3, float>(pl, lvl_child, in, out, true, false, s);
}

fc2t2_status launch_downshift(const fc2t2_plan_s* pl, int lvl_child, const void* in, void* out,
                              bool accumulate, hipStream_t s) {
  if (pl->io == FC2T2_IO_F64)
    return pl->dim == 2 ? shift_launch<2, double>(pl, lvl_child, in, out, false, accumulate, s)
                        : shift_launch<3, double>(pl, lvl_child, in, out, false, accumulate, s);
  return pl->dim == 2 ? shift_launch<2, float>(pl, lvl_child, in, out, false, accumulate, s)
                      : shift_launch<3, float>(pl, lvl_child, in, out, false, accumulate, s);
}

fc2t2_status launch_m2l(const fc2t2_plan_s* pl, int lvl, const void* M, void* L, bool accumulate,
                        hipStream_t s) {
  if (pl->prec >= FC2T2_M2L_BF16) {
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
  if (pl->prec >= FC2T2_M2L_BF16) {
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
                            hipStream_t s) {
  if (pl->prec >= FC2T2_M2L_BF16) return launch_m2l_mfma(pl, 0, pl->levels, ins, outs, false, transpose, s);
  for (int l = 0; l < pl->levels; ++l) {
    const fc2t2_status st = transpose ? launch_m2l_T(pl, l, ins[l], outs[l], false, s)
                                      : launch_m2l(pl, l, ins[l], outs[l], false, s);
    if (st) return st;
  }
  return FC2T2_OK;
}

// Up-shift pass: grids[l + 1] = up-shift(grids[l]) for l = 0 .. levels-2.
fc2t2_status upshift_pyramid(const fc2t2_plan_s* pl, void* const* grids, hipStream_t s) {
  for (int l = 0; l + 1 < pl->levels; ++l) {
    const fc2t2_status st = launch_upshift(pl, l, grids[l], grids[l + 1], s);
    if (st) return st;
  }
  return FC2T2_OK;
}

// Down-shift pass: grids[l] += down-shift(grids[l + 1]) for l = levels-2 .. 0.
fc2t2_status downshift_pyramid(const fc2t2_plan_s* pl, void* const* grids, hipStream_t s) {
  for (int l = pl->levels - 2; l >= 0; --l) {
    const fc2t2_status st = launch_downshift(pl, l, grids[l + 1], grids[l], true, s);
    if (st) return st;
  }
  return FC2T2_OK;
}

}  // namespace fc2t2

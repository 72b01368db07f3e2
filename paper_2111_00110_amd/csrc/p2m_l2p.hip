// Point <-> grid stages (section 3):
//   P2M    M[c, n] = sum_{s in c} w_s u_s^n / n!                 (per-cell segmented sum)
//   L2P    f(q) = sum_k L[c(q), k] u^k / k!, its gradient and Hessian
// and their transposes for the explicit layer's backward pass (section 4.1):
//   L2P^T  G_L[c, k] = sum_{q in c} gy_q u_q^k / k!               (per-cell segmented sum)
//   P2M^T  w_bar_s = <G_M[c(s)], u_s^n / n!>,  p_bar_s = w_s <G_M[c(s)], grad u_s^n / n!>
// with u = (x - centre) / h the cell-scaled offset.
//
// The segmented sums run over points sorted by cell: a group of GROUP lanes owns one cell,
// strides over its points in input order with TwoSum-compensated accumulation, combines
// the lanes with xor shuffles, and writes the cell's row.  No atomics.
#include "plan.h"
#include "segreduce.h"

using namespace fc2t2;

namespace {

template <typename T>
struct Vec4;
template <>
struct Vec4<float> { using type = float4; static constexpr int n = 4; };
template <>
struct Vec4<double> { using type = double2; static constexpr int n = 2; };

// Load a padded row of Ppad values (16-byte aligned) into registers.
template <int Ppad, typename T>
__device__ __forceinline__ void load_row(const T* __restrict__ src, T (&c)[Ppad]) {
  using V = typename Vec4<T>::type;
  constexpr int w = Vec4<T>::n;
  const V* s = reinterpret_cast<const V*>(src);
#pragma unroll
  for (int i = 0; i < Ppad / w; ++i) {
    const V v = s[i];
    if constexpr (w == 4) { c[4 * i] = v.x; c[4 * i + 1] = v.y; c[4 * i + 2] = v.z; c[4 * i + 3] = v.w; }
    else { c[2 * i] = v.x; c[2 * i + 1] = v.y; }
  }
}

template <class S, typename T>
struct PointMonomials {
  const T* __restrict__ x;     // [count][D]
  const T* __restrict__ wt;    // [count][C]
  int C;
  T inv_h;
  __device__ __forceinline__ void operator()(uint32_t idx, const T (&centre)[3], int ch,
                                             T (&v)[S::P], int64_t) const {
    T u[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < S::D; ++j) u[j] = (x[(int64_t)idx * S::D + j] - centre[j]) * inv_h;
    monomials<S>(u, v);
    const T a = wt[(int64_t)idx * C + ch];
#pragma unroll
    for (int k = 0; k < S::P; ++k) v[k] *= a;
  }
};

// The same from records sorted along with their data: pay [count][D + 1] holds each point's
// coordinates and its weight (one channel), indexed by sorted position.
template <class S, typename T>
struct SortedMonomials {
  const T* __restrict__ pay;   // [count][D + C]: coordinates, then the C values
  T inv_h;
  int C;
  __device__ __forceinline__ void operator()(uint32_t r, const T (&centre)[3], int ch, T (&v)[S::P],
                                             int64_t) const {
    const T* rec = pay + (size_t)r * (S::D + C);
    T u[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < S::D; ++j) u[j] = (rec[j] - centre[j]) * inv_h;
    monomials<S>(u, v);
    const T a = rec[S::D + ch];
#pragma unroll
    for (int k = 0; k < S::P; ++k) v[k] *= a;
  }
};

// Transpose of L2P fused with the query gradient (one channel): besides the record's
// monomials times gy, adds gy * grad f(q) to gq[q] using the cell's local row.  Each
// query is one record, so the gq writes do not collide.
template <class S, typename T>
struct QueryMonomialsGrad {
  const T* __restrict__ q;     // [M][D]
  const T* __restrict__ gy;    // [M]
  const T* __restrict__ L;     // [G][Ppad]
  T* __restrict__ gq;          // [M][D]
  T inv_h;
  __device__ __forceinline__ void operator()(uint32_t idx, const T (&centre)[3], int, T (&v)[S::P],
                                             int64_t cell) const {
    T u[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < S::D; ++j) u[j] = (q[(int64_t)idx * S::D + j] - centre[j]) * inv_h;
    T pw[3][S::K + 1];
    power_table<S>(u, pw);
    const T a = gy[idx];
    T row[S::Ppad];
    load_row<S::Ppad>(L + cell * S::Ppad, row);
    T val, g[3], hs[6];
    eval_poly<S, T, true, false>(row, pw, val, g, hs);
#pragma unroll
    for (int j = 0; j < S::D; ++j) gq[(int64_t)idx * S::D + j] += a * g[j] * inv_h;
    monomials<S>(u, v);
#pragma unroll
    for (int k = 0; k < S::P; ++k) v[k] *= a;
  }
};

// Transpose of L2P with q_bar from queries sorted with their coordinates (FP32, one channel):
// record r (sorted position) holds the coordinates (pay [M][D]); its input index perm[r] gives
// the cotangent gy and where q_bar goes.  Each query is one record, so the gq writes do not
// collide.
// q_bar of one query, written (or added) as one vector access of D floats: the queries are
// visited in cell order, so these are scattered, and one request per query instead of D.
template <int D>
struct alignas(4) FloatD {
  float v[D];
};
template <int D>
__device__ __forceinline__ void store_qgrad(float* __restrict__ dst, float s, const float (&g)[3], int accumulate) {
  FloatD<D> o;
#pragma unroll
  for (int j = 0; j < D; ++j) o.v[j] = s * g[j];
  FloatD<D>* p = reinterpret_cast<FloatD<D>*>(dst);
  if (accumulate) {
    const FloatD<D> old = *p;
#pragma unroll
    for (int j = 0; j < D; ++j) o.v[j] += old.v[j];
  }
  *p = o;
}

template <class S>
struct SortedQueryGrad {
  const float* __restrict__ pay;
  const uint32_t* __restrict__ perm;
  const float* __restrict__ gy;    // [M]
  const float* __restrict__ L;     // [G][Ppad]
  float* __restrict__ gq;          // [M][D]
  float inv_h;
  int accumulate;
  __device__ __forceinline__ void operator()(uint32_t r, const float (&centre)[3], int, float (&v)[S::P],
                                             int64_t cell) const {
    constexpr int D = S::D;
    const float* rec = pay + (size_t)r * D;
    float u[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < D; ++j) u[j] = (rec[j] - centre[j]) * inv_h;
    float pw[3][S::K + 1];
    power_table<S>(u, pw);
    const uint32_t i = perm[r];
    const float a = gy[i];
    if (gq) {
      float row[S::Ppad];
      load_row<S::Ppad>(L + cell * S::Ppad, row);
      float val, g[3], hs[6];
      eval_poly<S, float, true, false>(row, pw, val, g, hs);
      store_qgrad<D>(gq + (int64_t)i * D, a * inv_h, g, accumulate);
    }
    monomials<S>(u, v);
#pragma unroll
    for (int k = 0; k < S::P; ++k) v[k] *= a;
  }
};

template <typename T>
fc2t2_status reduce_points(const fc2t2_plan_s* pl, const void* x, const void* wt, int64_t count,
                           const uint32_t* starts, const uint32_t* perm, void* out, bool accumulate,
                           hipStream_t s, uint8_t* occ = nullptr, uint8_t gen = 1) {
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    PointMonomials<S, T> fn{(const T*)x, (const T*)wt, pl->C, (T)(1.0 / pl->h0)};
    st = launch_reduce_cells<S, T>(pl, starts, perm, count, (T*)out, accumulate, fn, s, occ, gen);
  });
  return st;
}

// ---------------------------------------------------------------------------------------
// Gather-evaluate: one thread per point reads its cell's row.
//   mode 0 (L2P):    y = f, grad = grad f / h, hess = H f / h^2     (overwrite)
//   mode 1 (q grad): gq += sum_ch gy[ch] grad_ch f / h              (accumulate)
//   mode 2 (P2M^T):  gw[ch] += f_ch, gp += sum_ch w[ch] grad_ch f / h (accumulate)
template <class S, typename T, int MODE, bool kGrad, bool kHess>
__global__ void __launch_bounds__(256) gather_eval_kernel(const T* __restrict__ grid, const T* __restrict__ x,
                                                          int64_t count, int C, int n, int64_t G, T lo,
                                                          T scale, T h, T inv_h,
                                                          const T* __restrict__ wts,
                                                          T* __restrict__ out_v, T* __restrict__ out_g,
                                                          T* __restrict__ out_h, int accumulate,
                                                          unsigned long long* __restrict__ ood) {
  constexpr int D = S::D, Ppad = S::Ppad;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int ic[3] = {0, 0, 0};
  int64_t cell = 0;
  T u[3] = {T(0), T(0), T(0)};
  bool out = false;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const T xj = x[i * D + j];
    out = out || outside_domain<T>(xj, lo, scale, n);
    ic[j] = cell_coord<T>(xj, lo, scale, n);
    cell = cell * n + ic[j];
    u[j] = (xj - (lo + (T(ic[j]) + T(0.5)) * h)) * inv_h;
  }
  if (ood) count_lanes(out, ood);
  T pw[3][S::K + 1];
  power_table<S>(u, pw);
  T gsum[3] = {T(0), T(0), T(0)};
  for (int ch = 0; ch < C; ++ch) {
    T c[Ppad];
    load_row<Ppad>(grid + ((int64_t)ch * G + cell) * Ppad, c);
    T val, g[3], hs[6];
    eval_poly<S, T, kGrad, kHess>(c, pw, val, g, hs);
    if constexpr (MODE == 0) {
      out_v[i * C + ch] = val;
      if constexpr (kGrad) {
#pragma unroll
        for (int j = 0; j < D; ++j) out_g[(i * C + ch) * D + j] = g[j] * inv_h;
      }
      if constexpr (kHess) {
        constexpr int NH = D == 2 ? 3 : 6;
#pragma unroll
        for (int j = 0; j < NH; ++j) out_h[(i * C + ch) * NH + j] = hs[j] * inv_h * inv_h;
      }
    } else if constexpr (MODE == 1) {
      const T a = wts[i * C + ch];
#pragma unroll
      for (int j = 0; j < D; ++j) gsum[j] += a * g[j];
    } else {
      if (out_v) out_v[i * C + ch] = accumulate ? out_v[i * C + ch] + val : val;
      const T a = wts[i * C + ch];
#pragma unroll
      for (int j = 0; j < D; ++j) gsum[j] += a * g[j];
    }
  }
  if constexpr (MODE != 0) {
    if (out_g) {
#pragma unroll
      for (int j = 0; j < D; ++j) out_g[i * D + j] = accumulate ? out_g[i * D + j] + gsum[j] * inv_h : gsum[j] * inv_h;
    }
  }
}

// q_bar over the queries in sorted order (FP32, one channel): record r holds the query's
// coordinates and cotangent (pay [M][D + 1]), its cell (keys) and input index (perm); queries of
// one cell are neighbours, so their row is read from cache.  gq[perm[r]] = (or +=) gy grad f / h.
template <class S>
__global__ void __launch_bounds__(256) qgrad_sorted_kernel(const float* __restrict__ grid, const float* __restrict__ pay,
                                                           const uint32_t* __restrict__ keys,
                                                           const uint32_t* __restrict__ perm, int64_t count, int n,
                                                           float lo, float h, float inv_h, float* __restrict__ gq,
                                                           int accumulate, const uint32_t* __restrict__ err) {
  constexpr int D = S::D, Ppad = S::Ppad, W = D + 1;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= count || *err) return;   // a failed sort: the records are not valid
  const int64_t cell = keys[r];
  int ic[3];
  decode_cell<D, float>(cell, n, ic);
  const float* rec = pay + r * W;
  float u[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < D; ++j) u[j] = (rec[j] - (lo + (float(ic[j]) + 0.5f) * h)) * inv_h;
  float pw[3][S::K + 1];
  power_table<S>(u, pw);
  float c[Ppad];
  load_row<Ppad>(grid + cell * Ppad, c);
  float val, g[3], hs[6];
  eval_poly<S, float, true, false>(c, pw, val, g, hs);
  const float a = rec[D];
  const int64_t i = perm[r];
  store_qgrad<D>(gq + (int64_t)i * D, a * inv_h, g, accumulate);
}

// L2P over the queries in sorted order (FP32, one channel): record r holds the query's
// coordinates (pay [M][D]), its cell (keys) and input index (perm); queries of one cell are
// neighbours, so their row is read once from memory and then from cache.  y[perm[r]] = f.
template <class S>
__global__ void __launch_bounds__(256) l2p_sorted_kernel(const float* __restrict__ grid, const float* __restrict__ pay,
                                                         const uint32_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ perm, int64_t count, int n,
                                                         float lo, float h, float inv_h, float* __restrict__ y,
                                                         const uint32_t* __restrict__ err) {
  constexpr int D = S::D, Ppad = S::Ppad;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= count || *err) return;   // a failed sort: the records are not valid
  const int64_t cell = keys[r];
  int ic[3];
  decode_cell<D, float>(cell, n, ic);
  const float* rec = pay + r * D;
  float u[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < D; ++j) u[j] = (rec[j] - (lo + (float(ic[j]) + 0.5f) * h)) * inv_h;
  float pw[3][S::K + 1];
  power_table<S>(u, pw);
  float c[Ppad];
  load_row<Ppad>(grid + cell * Ppad, c);
  float val, g[3], hs[6];
  eval_poly<S, float, false, false>(c, pw, val, g, hs);
  y[perm[r]] = val;
}

template <typename T, int MODE>
fc2t2_status gather_eval(const fc2t2_plan_s* pl, const void* grid, const void* x, int64_t count,
                         const void* wts, void* out_v, void* out_g, void* out_h, hipStream_t s,
                         int accumulate = 1, unsigned long long* ood = nullptr) {
  if (count == 0) return FC2T2_OK;
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  const int threads = 256;
  const dim3 blocks((unsigned)ceil_div(count, threads));
  const T lo = (T)pl->lo, scale = (T)(pl->n / (pl->hi - pl->lo)), h = (T)pl->h0, inv_h = (T)(1.0 / pl->h0);
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    if constexpr (MODE == 0) {
      if (out_h)
        hipLaunchKernelGGL((gather_eval_kernel<S, T, 0, true, true>), blocks, dim3(threads), 0, s,
                           (const T*)grid, (const T*)x, count, pl->C, pl->n, pl->G, lo, scale, h, inv_h,
                           (const T*)wts, (T*)out_v, (T*)out_g, (T*)out_h, accumulate, ood);
      else if (out_g)
        hipLaunchKernelGGL((gather_eval_kernel<S, T, 0, true, false>), blocks, dim3(threads), 0, s,
                           (const T*)grid, (const T*)x, count, pl->C, pl->n, pl->G, lo, scale, h, inv_h,
                           (const T*)wts, (T*)out_v, (T*)out_g, (T*)out_h, accumulate, ood);
      else
        hipLaunchKernelGGL((gather_eval_kernel<S, T, 0, false, false>), blocks, dim3(threads), 0, s,
                           (const T*)grid, (const T*)x, count, pl->C, pl->n, pl->G, lo, scale, h, inv_h,
                           (const T*)wts, (T*)out_v, (T*)out_g, (T*)out_h, accumulate, ood);
    } else {
      hipLaunchKernelGGL((gather_eval_kernel<S, T, MODE, true, false>), blocks, dim3(threads), 0, s,
                         (const T*)grid, (const T*)x, count, pl->C, pl->n, pl->G, lo, scale, h, inv_h,
                         (const T*)wts, (T*)out_v, (T*)out_g, (T*)out_h, accumulate, ood);
    }
    st = FC2T2_OK;
  });
  if (st != FC2T2_OK) return st;
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

}  // namespace

namespace fc2t2 {

fc2t2_status launch_p2m(const fc2t2_plan_s* pl, const void* p, const void* w, int64_t N,
                        const uint32_t* starts, const uint32_t* perm, void* M0, hipStream_t s, uint8_t* occ,
                        uint8_t gen) {
  return pl->io == FC2T2_IO_F64 ? reduce_points<double>(pl, p, w, N, starts, perm, M0, false, s, occ, gen)
                                : reduce_points<float>(pl, p, w, N, starts, perm, M0, false, s, occ, gen);
}

// Occupancy of the finest cells from points: occ[cell(x)] = gen.
template <typename T, int D>
__global__ void __launch_bounds__(256) mark_cells_kernel(const T* __restrict__ x, int64_t N, T lo, T scale, int n,
                                                         uint8_t* __restrict__ occ, uint8_t gen) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int64_t cell = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) cell = cell * n + cell_coord<T>(x[i * D + j], lo, scale, n);
  occ[cell] = gen;
}

__global__ void __launch_bounds__(256) clear_bytes_kernel(uint8_t* __restrict__ p, int64_t n) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
  if (i + 16 <= n) {
    *reinterpret_cast<uint4*>(p + i) = uint4{0u, 0u, 0u, 0u};
  } else {
    for (int64_t j = i; j < n; ++j) p[j] = 0;
  }
}

fc2t2_status launch_mark_cells(const fc2t2_plan_s* pl, const void* x, int64_t N, uint8_t* occ, uint8_t gen,
                               hipStream_t s) {
  // cleared first: workspace bytes left by earlier calls would match the stamp now and then
  // and disable skips
  hipLaunchKernelGGL(clear_bytes_kernel, dim3((unsigned)ceil_div(ceil_div(pl->G, 16), 256)), dim3(256), 0, s, occ,
                     pl->G);
  FC2T2_LAUNCH_CHECK();
  if (N == 0) return FC2T2_OK;
  const dim3 grid((unsigned)ceil_div(N, 256));
  const double scale = pl->n / (pl->hi - pl->lo);
  if (pl->io == FC2T2_IO_F64) {
    if (pl->dim == 2)
      hipLaunchKernelGGL((mark_cells_kernel<double, 2>), grid, dim3(256), 0, s, (const double*)x, N, pl->lo, scale, pl->n, occ, gen);
    else
      hipLaunchKernelGGL((mark_cells_kernel<double, 3>), grid, dim3(256), 0, s, (const double*)x, N, pl->lo, scale, pl->n, occ, gen);
  } else {
    if (pl->dim == 2)
      hipLaunchKernelGGL((mark_cells_kernel<float, 2>), grid, dim3(256), 0, s, (const float*)x, N, (float)pl->lo, (float)scale, pl->n, occ, gen);
    else
      hipLaunchKernelGGL((mark_cells_kernel<float, 3>), grid, dim3(256), 0, s, (const float*)x, N, (float)pl->lo, (float)scale, pl->n, occ, gen);
  }
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

fc2t2_status launch_reduce_sorted(const fc2t2_plan_s* pl, const void* pay, int64_t count, const uint32_t* starts,
                                  void* out, bool accumulate, hipStream_t s, uint8_t* occ, uint8_t gen) {
  if (pl->io != FC2T2_IO_F32 || pl->C > 4) return FC2T2_EUNSUPPORTED;
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    SortedMonomials<S, float> fn{(const float*)pay, (float)(1.0 / pl->h0), pl->C};
    // sources (the call that records occupancy) may crowd a few cells: let waves take those
    st = occ ? launch_reduce_cells<S, float, decltype(fn), true>(pl, starts, nullptr, count, (float*)out, accumulate,
                                                                  fn, s, occ, gen)
             : launch_reduce_cells<S, float>(pl, starts, nullptr, count, (float*)out, accumulate, fn, s, occ, gen);
  });
  return st;
}

fc2t2_status launch_l2p_T(const fc2t2_plan_s* pl, const void* q, const void* gy, int64_t M,
                          const uint32_t* starts, const uint32_t* perm, void* gL, hipStream_t s, bool accumulate) {
  return pl->io == FC2T2_IO_F64 ? reduce_points<double>(pl, q, gy, M, starts, perm, gL, accumulate, s)
                                : reduce_points<float>(pl, q, gy, M, starts, perm, gL, accumulate, s);
}

template <typename T>
fc2t2_status l2p_T_qgrad_t(const fc2t2_plan_s* pl, const void* L, const void* q, const void* gy, int64_t M,
                           const uint32_t* starts, const uint32_t* perm, void* gL, void* gq, hipStream_t s,
                           bool accumulate) {
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    QueryMonomialsGrad<S, T> fn{(const T*)q, (const T*)gy, (const T*)L, (T*)gq, (T)(1.0 / pl->h0)};
    st = launch_reduce_cells<S, T>(pl, starts, perm, M, (T*)gL, accumulate, fn, s);
  });
  return st;
}

fc2t2_status launch_l2p_T_qgrad(const fc2t2_plan_s* pl, const void* L, const void* q, const void* gy, int64_t M,
                                const uint32_t* starts, const uint32_t* perm, void* gL, void* gq, hipStream_t s,
                                bool accumulate) {
  if (pl->C != 1) return FC2T2_EUNSUPPORTED;
  return pl->io == FC2T2_IO_F64 ? l2p_T_qgrad_t<double>(pl, L, q, gy, M, starts, perm, gL, gq, s, accumulate)
                                : l2p_T_qgrad_t<float>(pl, L, q, gy, M, starts, perm, gL, gq, s, accumulate);
}

fc2t2_status launch_l2p(const fc2t2_plan_s* pl, const void* L, const void* q, int64_t M, void* y,
                        void* grad, void* hess, hipStream_t s) {
  return pl->io == FC2T2_IO_F64 ? gather_eval<double, 0>(pl, L, q, M, nullptr, y, grad, hess, s, 1, pl->ood)
                                : gather_eval<float, 0>(pl, L, q, M, nullptr, y, grad, hess, s, 1, pl->ood);
}

fc2t2_status launch_l2p_qgrad(const fc2t2_plan_s* pl, const void* L, const void* q, int64_t M,
                              const void* gy, void* gq, hipStream_t s, bool accumulate) {
  const int acc = accumulate ? 1 : 0;
  return pl->io == FC2T2_IO_F64 ? gather_eval<double, 1>(pl, L, q, M, gy, nullptr, gq, nullptr, s, acc)
                                : gather_eval<float, 1>(pl, L, q, M, gy, nullptr, gq, nullptr, s, acc);
}

fc2t2_status launch_p2m_T(const fc2t2_plan_s* pl, const void* GM0, const void* p, const void* w,
                          int64_t N, void* gp, void* gw, hipStream_t s, bool accumulate) {
  const int acc = accumulate ? 1 : 0;
  return pl->io == FC2T2_IO_F64 ? gather_eval<double, 2>(pl, GM0, p, N, w, gw, gp, nullptr, s, acc)
                                : gather_eval<float, 2>(pl, GM0, p, N, w, gw, gp, nullptr, s, acc);
}

fc2t2_status launch_qgrad_sorted(const fc2t2_plan_s* pl, const void* L, const void* pay, const uint32_t* keys,
                                 const uint32_t* perm, int64_t M, void* gq, hipStream_t s, bool accumulate,
                                 const uint32_t* err) {
  if (pl->io != FC2T2_IO_F32 || pl->C != 1) return FC2T2_EUNSUPPORTED;
  if (M == 0) return FC2T2_OK;
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  const dim3 grid((unsigned)ceil_div(M, 256));
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    hipLaunchKernelGGL((qgrad_sorted_kernel<S>), grid, dim3(256), 0, s, (const float*)L, (const float*)pay, keys, perm,
                       M, pl->n, (float)pl->lo, (float)pl->h0, (float)(1.0 / pl->h0), (float*)gq, accumulate ? 1 : 0,
                       err);
    st = FC2T2_OK;
  });
  if (st != FC2T2_OK) return st;
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

fc2t2_status launch_l2p_sorted(const fc2t2_plan_s* pl, const void* L, const void* pay, const uint32_t* keys,
                               const uint32_t* perm, int64_t M, void* y, hipStream_t s, const uint32_t* err) {
  if (pl->io != FC2T2_IO_F32 || pl->C != 1) return FC2T2_EUNSUPPORTED;
  if (M == 0) return FC2T2_OK;
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  const dim3 grid((unsigned)ceil_div(M, 256));
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    hipLaunchKernelGGL((l2p_sorted_kernel<S>), grid, dim3(256), 0, s, (const float*)L, (const float*)pay, keys, perm,
                       M, pl->n, (float)pl->lo, (float)pl->h0, (float)(1.0 / pl->h0), (float*)y, err);
    st = FC2T2_OK;
  });
  if (st != FC2T2_OK) return st;
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

fc2t2_status launch_l2p_T_qgrad_sorted(const fc2t2_plan_s* pl, const void* L, const void* pay, const uint32_t* starts,
                                       const uint32_t* perm, const void* gy, int64_t M, void* gL, void* gq,
                                       hipStream_t s, bool accumulate) {
  if (pl->io != FC2T2_IO_F32 || pl->C != 1) return FC2T2_EUNSUPPORTED;
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    SortedQueryGrad<S> fn{(const float*)pay, perm, (const float*)gy, (const float*)L, (float*)gq,
                          (float)(1.0 / pl->h0), accumulate ? 1 : 0};
    st = launch_reduce_cells<S, float>(pl, starts, nullptr, M, (float*)gL, accumulate, fn, s);
  });
  return st;
}

template <typename T>
__global__ void __launch_bounds__(256) zero_kernel(T* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

fc2t2_status launch_zero(const fc2t2_plan_s* pl, void* p, int64_t elems, hipStream_t s) {
  if (elems <= 0) return FC2T2_OK;
  const dim3 grid((unsigned)ceil_div(elems, 256));
  if (pl->io == FC2T2_IO_F64)
    hipLaunchKernelGGL(zero_kernel<double>, grid, dim3(256), 0, s, (double*)p, elems);
  else
    hipLaunchKernelGGL(zero_kernel<float>, grid, dim3(256), 0, s, (float*)p, elems);
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

}  // namespace fc2t2

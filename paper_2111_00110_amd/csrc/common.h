// Shared device/host helpers of the FC^2T^2 HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <type_traits>
#include <utility>

#include "fc2t2.h"

namespace fc2t2 {

// ----------------------------------------------------------------------------- limits
constexpr int kMaxLevels = 12;          // n <= 2^13
constexpr int kWave = 64;               // CDNA wavefront

// ----------------------------------------------------------------------------- status
#define FC2T2_HIP_CHECK(expr)                                        \
  do {                                                               \
    hipError_t _e = (expr);                                          \
    if (_e != hipSuccess) return FC2T2_EHIP;                         \
  } while (0)

#define FC2T2_LAUNCH_CHECK()                                         \
  do {                                                               \
    hipError_t _e = hipGetLastError();                               \
    if (_e != hipSuccess) return FC2T2_EHIP;                         \
  } while (0)

// ----------------------------------------------------------------------------- multi-indices
// Graded order: total degree t ascending; inside a degree the first component descending,
// then the second.  Position of (a0, a1) with t = a0 + a1: t(t+1)/2 + (t - a0).
// Position of (a0, a1, a2) with t = a0 + a1 + a2:
//   t(t+1)(t+2)/6 + (t - a0)(t - a0 + 1)/2 + (t - a0 - a1).
__host__ __device__ constexpr int nterms(int D, int K) {
  return D == 2 ? (K + 1) * (K + 2) / 2 : (K + 1) * (K + 2) * (K + 3) / 6;
}
__host__ __device__ constexpr int mi_pos2(int a0, int a1) {
  return (a0 + a1) * (a0 + a1 + 1) / 2 + a1;
}
__host__ __device__ constexpr int mi_pos3(int a0, int a1, int a2) {
  return (a0 + a1 + a2) * (a0 + a1 + a2 + 1) * (a0 + a1 + a2 + 2) / 6 +
         (a1 + a2) * (a1 + a2 + 1) / 2 + a2;
}
template <int D>
__host__ __device__ constexpr int mi_pos(int a0, int a1, int a2) {
  return D == 2 ? mi_pos2(a0, a1) : mi_pos3(a0, a1, a2);
}
__host__ __device__ constexpr int pad4(int P) { return (P + 3) & ~3; }

// Runtime enumeration (host and device): fill exps[P][3] in graded order.
__host__ __device__ inline void mi_fill(int D, int K, int (*exps)[3]) {
  int idx = 0;
  for (int t = 0; t <= K; ++t) {
    if (D == 2) {
      for (int a = t; a >= 0; --a) { exps[idx][0] = a; exps[idx][1] = t - a; exps[idx][2] = 0; ++idx; }
    } else {
      for (int a = t; a >= 0; --a)
        for (int b = t - a; b >= 0; --b) {
          exps[idx][0] = a; exps[idx][1] = b; exps[idx][2] = t - a - b; ++idx;
        }
    }
  }
}

// ----------------------------------------------------------------------------- compile-time shapes
template <int D_, int K_>
struct Shape {
  static constexpr int D = D_;
  static constexpr int K = K_;
  static constexpr int P = nterms(D_, K_);
  static constexpr int Ppad = pad4(nterms(D_, K_));
};

// Monomials u^a / a! for every multi-index, in graded order, from per-dimension power
// tables.  All loops unroll, so every index is a compile-time constant.
template <class S, typename T>
__device__ __forceinline__ void monomials(const T (&u)[3], T (&out)[S::P]) {
  constexpr int D = S::D, K = S::K;
  T pw[D][K + 1];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    pw[j][0] = T(1);
#pragma unroll
    for (int a = 1; a <= K; ++a) pw[j][a] = pw[j][a - 1] * u[j] * (T(1) / T(a));
  }
#pragma unroll
  for (int t = 0; t <= K; ++t) {
#pragma unroll
    for (int a = t; a >= 0; --a) {
      if constexpr (D == 2) {
        out[mi_pos2(a, t - a)] = pw[0][a] * pw[1][t - a];
      } else {
#pragma unroll
        for (int b = t - a; b >= 0; --b)
          out[mi_pos3(a, b, t - a - b)] = pw[0][a] * pw[1][b] * pw[2][t - a - b];
      }
    }
  }
}

// Low-degree monomials (|a| <= K - drop) of the same point, reusing a power table.
template <class S, typename T>
__device__ __forceinline__ void power_table(const T (&u)[3], T (&pw)[3][S::K + 1]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    pw[j][0] = T(1);
#pragma unroll
    for (int a = 1; a <= S::K; ++a) pw[j][a] = pw[j][a - 1] * (j < S::D ? u[j] : T(0)) * (T(1) / T(a));
  }
}

// Value, gradient and Hessian of sum_k c[k] u^k / k! (all in u-units) from a power table.
// grad_j = sum_{|m| <= K-1} c[m + e_j] u^m / m!, hess_ab = sum_{|m| <= K-2} c[m+e_a+e_b] u^m/m!.
template <class S, typename T, bool kGrad, bool kHess>
__device__ __forceinline__ void eval_poly(const T* c, const T (&pw)[3][S::K + 1], T& val,
                                          T (&grad)[3], T (&hess)[6]) {
  constexpr int D = S::D, K = S::K;
  val = T(0);
#pragma unroll
  for (int j = 0; j < 3; ++j) grad[j] = T(0);
#pragma unroll
  for (int j = 0; j < 6; ++j) hess[j] = T(0);
#pragma unroll
  for (int t = 0; t <= K; ++t) {
#pragma unroll
    for (int a = t; a >= 0; --a) {
#pragma unroll
      for (int b = (D == 2 ? t - a : t - a); b >= (D == 2 ? t - a : 0); --b) {
        const int cc = (D == 2) ? 0 : t - a - b;
        const T m = (D == 2) ? pw[0][a] * pw[1][b] : pw[0][a] * pw[1][b] * pw[2][cc];
        val += c[mi_pos<D>(a, b, cc)] * m;
        if constexpr (kGrad) {
          if (t + 1 <= K) {
            grad[0] += c[mi_pos<D>(a + 1, b, cc)] * m;
            grad[1] += c[mi_pos<D>(a, b + 1, cc)] * m;
            if constexpr (D == 3) grad[2] += c[mi_pos<D>(a, b, cc + 1)] * m;
          }
        }
        if constexpr (kHess) {
          if (t + 2 <= K) {
            if constexpr (D == 2) {
              hess[0] += c[mi_pos<D>(a + 2, b, 0)] * m;
              hess[1] += c[mi_pos<D>(a + 1, b + 1, 0)] * m;
              hess[2] += c[mi_pos<D>(a, b + 2, 0)] * m;
            } else {
              hess[0] += c[mi_pos<D>(a + 2, b, cc)] * m;
              hess[1] += c[mi_pos<D>(a + 1, b + 1, cc)] * m;
              hess[2] += c[mi_pos<D>(a + 1, b, cc + 1)] * m;
              hess[3] += c[mi_pos<D>(a, b + 2, cc)] * m;
              hess[4] += c[mi_pos<D>(a, b + 1, cc + 1)] * m;
              hess[5] += c[mi_pos<D>(a, b, cc + 2)] * m;
            }
          }
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------- compensated sums
// Knuth's TwoSum: s + x = t + e exactly; the error is kept in a running compensation.
template <typename T>
__device__ __forceinline__ void acc2(T& s, T& c, T x) {
  const T t = s + x;
  const T bp = t - s;
  const T e = (s - (t - bp)) + (x - bp);
  s = t;
  c += e;
}

// ----------------------------------------------------------------------------- cell index
// i = clamp(floor((x - lo) * scale), 0, n - 1) with one rounding per operation in T.
template <typename T>
__device__ __forceinline__ int cell_coord(T x, T lo, T scale, int n) {
  T u = (x - lo);
  u = u * scale;
  int i = (int)floor(u);
  // NaN and huge values land on a boundary cell
  if (!(u >= T(0))) i = 0;
  if (u >= T(n)) i = n - 1;
  return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

// Whether x lies outside [lo, hi] (hi = lo + n / scale), by the cell formula's own rounding;
// NaN counts as outside.
template <typename T>
__device__ __forceinline__ bool outside_domain(T x, T lo, T scale, int n) {
  T u = (x - lo);
  u = u * scale;
  return !(u >= T(0) && u <= T(n));
}

// Adds the number of active lanes with `flag` set to *ctr: one vector atomic per wave.
__device__ __forceinline__ void count_lanes(bool flag, unsigned long long* ctr) {
  const unsigned long long m = __ballot(flag);
  if (m && (int)(threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicAdd(ctr, (unsigned long long)__popcll(m));
}

// ----------------------------------------------------------------------------- dispatch
// Calls f(Shape<D,K>{}) for the supported (D, K) pairs; returns false otherwise.
template <class F>
bool dispatch_shape(int D, int K, F&& f) {
  if (D == 2) {
    switch (K) {
      case 1: f(Shape<2, 1>{}); return true;
      case 2: f(Shape<2, 2>{}); return true;
      case 3: f(Shape<2, 3>{}); return true;
      case 4: f(Shape<2, 4>{}); return true;
      case 5: f(Shape<2, 5>{}); return true;
      case 6: f(Shape<2, 6>{}); return true;
    }
  } else if (D == 3) {
    switch (K) {
      case 1: f(Shape<3, 1>{}); return true;
      case 2: f(Shape<3, 2>{}); return true;
      case 3: f(Shape<3, 3>{}); return true;
      case 4: f(Shape<3, 4>{}); return true;
      case 5: f(Shape<3, 5>{}); return true;
    }
  }
  return false;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int lg2i(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace fc2t2

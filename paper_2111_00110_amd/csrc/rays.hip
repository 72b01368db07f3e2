// Ray layers on the finest-level local expansions (dim 3):
//   line integral        y = integral over t of f(o + t r)            (section 6.1.1)
//   ray insertion        G_L[c] += gy * int_0^s (d + r v)^k / k! dv   (section 6.2.1)
//   first level crossing of f along the ray and its IFT backward     (sections 5.1, 5.2)
//
// Traversal: the ray is clipped to the domain and [t0, t1], then walked cell by cell with
// an incremental 3-D DDA in FP64 whose plane crossings are recomputed from the plane
// position at every step (lo + k h - o) / r, so they do not drift.  Inside a cell with
// centre c the expansion restricted to the segment is a polynomial in v = t - t_a with
// u(v) = (o + t_a r - c) / h + v r / h (line to polynomial, section 5.1.1).
//
// MI355X note: without packed FP32 the vector FP32 and FP64 rates are equal, so the
// per-segment polynomial work (line integrals, root isolation) runs in FP64; only the
// expansion rows are FP32.
#include <math.h>

#include <mutex>

#include "plan.h"
#include "raywalk.h"
#include "segreduce.h"

using namespace fc2t2;

// Scratch of fc2t2_ray_root_backward_noalloc: a fixed array in device memory, one copy per
// GPU (the code object's data segment), held until the process ends.  Host code never uses
// this name as an address: the device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) char scratch[FC2T2_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kRaySaved = FC2T2_ROOT_SAVED;

// The root's finest cell travels in a slot of the saved record as the bits of an integer
// (32 bits in an FP32 record, 64 in an FP64 one), never as a floating-point value.
__device__ __forceinline__ void put_cell(float& slot, int64_t c) { slot = __uint_as_float((uint32_t)c); }
__device__ __forceinline__ void put_cell(double& slot, int64_t c) { slot = __longlong_as_double((long long)c); }
__device__ __forceinline__ int64_t get_cell(float slot) { return (int64_t)__float_as_uint(slot); }
__device__ __forceinline__ int64_t get_cell(double slot) { return (int64_t)__double_as_longlong(slot); }

// Three-point Gauss-Legendre rule on [0, s]: nodes s (1 + x_i) / 2 with x = 0, +-sqrt(3/5),
// weights (s / 2) * (8/9, 5/9, 5/9).  Exact for polynomials of degree <= 5, so for every
// monomial of an expansion with K <= 5 it gives the segment integral exactly (up to
// rounding) -- the same value as integrating the line polynomial term by term.
__device__ __forceinline__ void gl3(double s, double (&v)[3], double (&wt)[3]) {
  const double x = 0.7745966692414833770;   // sqrt(3/5)
  v[0] = 0.5 * s;
  v[1] = 0.5 * s * (1.0 - x);
  v[2] = 0.5 * s * (1.0 + x);
  wt[0] = 0.5 * s * (8.0 / 9.0);
  wt[1] = 0.5 * s * (5.0 / 9.0);
  wt[2] = wt[1];
}

// ---------------------------------------------------------------------------------------
template <class S, typename T>
__device__ __forceinline__ void load_row_f64(const T* __restrict__ src, double (&c)[S::P]) {
#pragma unroll
  for (int k = 0; k < S::P; ++k) c[k] = (double)src[k];
}

// Line integral: kRayLanes lanes per ray, each over its sub-range of the clipped ray; each
// piece's integral is the three-point Gauss-Legendre sum of the cell polynomial (exact for
// K <= 5), accumulated in FP64, and the lanes' sums are added by a butterfly.
template <class S, typename T>
__global__ void __launch_bounds__(64) ray_integral_kernel(const T* __restrict__ L, const T* __restrict__ O,
                                                          const T* __restrict__ Rd, int64_t R, double t0,
                                                          double t1, double lo, double hi, double h, int n,
                                                          int64_t G, T* __restrict__ y, int C) {
  static_assert(S::K <= 5, "three Gauss-Legendre nodes integrate degree <= 5 exactly");
  constexpr int P = S::P, Ppad = S::Ppad, K = S::K;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ray = gid / kRayLanes;
  const int l = (int)(gid % kRayLanes);
  const int ch = blockIdx.y;
  double acc = 0.0;
  double o[3], r[3], ta_r, tb_r;
  if (ray < R) {
    load3(O, ray, o);
    load3(Rd, ray, r);
  }
  if (ray < R && ray_range(o, r, t0, t1, lo, hi, ta_r, tb_r)) {
    Dda dda;
    dda.init(o, r, lane_cut(ta_r, tb_r, l), lane_cut(ta_r, tb_r, l + 1), lo, hi, h, n);
    const double ih = 1.0 / h;
    const double q[3] = {r[0] * ih, r[1] * ih, r[2] * ih};
    const T* __restrict__ Lc = L + (int64_t)ch * G * Ppad;
    int64_t cell;
    int cc[3];
    double ta, tb;
    while (dda.next(cell, cc, ta, tb)) {
      double row[P];
      load_row_f64<S>(Lc + cell * Ppad, row);
      double d[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) d[j] = (o[j] + ta * r[j] - (lo + (cc[j] + 0.5) * h)) * ih;
      double nodes[3], wt[3];
      gl3(tb - ta, nodes, wt);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double u[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) u[j] = d[j] + q[j] * nodes[i];
        double pw[3][K + 1];
        power_table<S>(u, pw);
        double val, g[3], hs[6];
        eval_poly<S, double, false, false>(row, pw, val, g, hs);
        acc += wt[i] * val;
      }
    }
  }
#pragma unroll
  for (int off = kRayLanes / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, kRayLanes);
  if (ray < R && l == 0) y[ray * C + ch] = (T)acc;
}

// ---------------------------------------------------------------------------------------
// Ray insertion records: lane l of ray i writes its pieces to its own slots (ray_slot; the cell
// as the sort key, [ta, tb] as payload); unused slots get the key G (sorted after every cell).
// The ray of a slot is slot / maxseg with maxseg = kRayLanes perlane.
template <typename T>
__global__ void __launch_bounds__(256) ray_records_kernel(const T* __restrict__ O, const T* __restrict__ Rd,
                                                          int64_t R, double t0, double t1, double lo, double hi,
                                                          double h, int n, int64_t G, int perlane,
                                                          uint32_t* __restrict__ keys, double2* __restrict__ rec) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ray = gid / kRayLanes;
  const int l = (int)(gid % kRayLanes);
  if (ray >= R) return;
  double o[3], r[3], ta_r, tb_r;
  load3(O, ray, o);
  load3(Rd, ray, r);
  int j = 0;
  if (ray_range(o, r, t0, t1, lo, hi, ta_r, tb_r)) {
    Dda dda;
    dda.init(o, r, lane_cut(ta_r, tb_r, l), lane_cut(ta_r, tb_r, l + 1), lo, hi, h, n);
    int64_t cell;
    int cc[3];
    double ta, tb;
    while (j < perlane && dda.next(cell, cc, ta, tb)) {
      const int64_t slot = ray_slot(ray, l, j, perlane);
      keys[slot] = (uint32_t)cell;
      rec[slot] = make_double2(ta, tb);
      ++j;
    }
  }
  for (; j < perlane; ++j) keys[ray_slot(ray, l, j, perlane)] = (uint32_t)G;
}

template <class S, typename T>
struct SegmentInsert {
  static_assert(S::K <= 5, "three Gauss-Legendre nodes integrate degree <= 5 exactly");
  const T* __restrict__ O;
  const T* __restrict__ Rd;
  const double2* __restrict__ rec;
  const T* __restrict__ gy;
  int maxseg, C;
  double ih;   // 1 / h
  __device__ __forceinline__ void operator()(uint32_t slot, const T (&centre)[3], int ch, T (&v)[S::P],
                                             int64_t) const {
    const int64_t ray = slot / maxseg;
    double o[3], r[3];
    load3(O, ray, o);
    load3(Rd, ray, r);
    const double2 tt = rec[slot];
    double d[3], q[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      d[j] = (o[j] + tt.x * r[j] - (double)centre[j]) * ih;
      q[j] = r[j] * ih;
    }
    double nodes[3], wt[3];
    gl3(tt.y - tt.x, nodes, wt);
    const double g = (double)gy[ray * C + ch];
#pragma unroll
    for (int k = 0; k < S::P; ++k) v[k] = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T u[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) u[j] = (T)(d[j] + q[j] * nodes[i]);
      T m[S::P];
      monomials<S>(u, m);
      const T a = (T)(g * wt[i]);
#pragma unroll
      for (int k = 0; k < S::P; ++k) v[k] += a * m[k];
    }
  }
};

// ---------------------------------------------------------------------------------------
// Real-root isolation for polynomials of degree <= 5 on [a, b] (FP64): the roots of the
// derivative split [a, b] into monotone pieces; each piece with a sign change holds one
// root, found by Newton steps safeguarded by bisection.
template <int DEG>
__device__ __forceinline__ double peval(const double (&c)[6], double x) {
  double v = c[DEG];
#pragma unroll
  for (int m = DEG - 1; m >= 0; --m) v = v * x + c[m];
  return v;
}

template <int DEG>
__device__ double solve_monotone(const double (&c)[6], double lo, double hi, double flo, double x0 = -1.0) {
  double dc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int m = 0; m < DEG; ++m) dc[m] = (m + 1) * c[m + 1];
  double x = (x0 > lo && x0 < hi) ? x0 : 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    const double fx = peval<DEG>(c, x);
    if (fx == 0.0) return x;
    if ((fx < 0.0) == (flo < 0.0)) { lo = x; flo = fx; } else { hi = x; }
    const double dfx = peval<(DEG >= 1 ? DEG - 1 : 0)>(dc, x);
    double xn = x - fx / dfx;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    const double tol = 4e-16 * fmax(1.0, fabs(x));
    if (fabs(xn - x) <= tol || hi - lo <= tol) return xn;
    x = xn;
  }
  return x;
}

// Sign-changing roots of c (degree <= DEG) in [a, b], ascending.  Returns the count.
template <int DEG>
__device__ int real_roots(const double (&c)[6], double a, double b, double (&out)[5]) {
  if constexpr (DEG <= 0) {
    return 0;
  } else {
    if (c[DEG] == 0.0) return real_roots<DEG - 1>(c, a, b, out);
    if constexpr (DEG == 1) {
      const double x = -c[0] / c[1];
      if (a <= x && x <= b) { out[0] = x; return 1; }
      return 0;
    } else {
      double dc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int m = 0; m < DEG; ++m) dc[m] = (m + 1) * c[m + 1];
      double crit[5];
      const int nc = real_roots<DEG - 1>(dc, a, b, crit);
      double pts[7];
      int np = 0;
      pts[np++] = a;
      for (int i = 0; i < nc; ++i)
        if (crit[i] > a && crit[i] < b && crit[i] > pts[np - 1]) pts[np++] = crit[i];
      pts[np++] = b;
      int cnt = 0;
      double f0 = peval<DEG>(c, pts[0]);
      for (int i = 0; i + 1 < np; ++i) {
        const double f1 = peval<DEG>(c, pts[i + 1]);
        if (f0 == 0.0) {
          if (cnt == 0 || out[cnt - 1] != pts[i]) out[cnt++] = pts[i];
        } else if ((f0 < 0.0) != (f1 < 0.0) && f1 != 0.0) {
          out[cnt++] = solve_monotone<DEG>(c, pts[i], pts[i + 1], f0);
        }
        f0 = f1;
      }
      if (f0 == 0.0 && (cnt == 0 || out[cnt - 1] != b)) out[cnt++] = b;
      return cnt;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Closed-form roots for degree <= 4 (section 5.1: the paper finds the roots of a box's quartic
// with Ferrari's method): the quadratic formula in its cancellation-free form, Cardano's
// formula for the cubic (trigonometric form when all three roots are real), and Ferrari's
// reduction of the quartic to two quadratics through a positive root of its resolvent cubic.
// Every real root is polished by three Newton steps on the original polynomial.  A leading
// coefficient below 1e-8 of the largest other one is dropped first (on [0, 1] its term moves a
// root of the rest by a relative 1e-8 at most, which the polish removes).  The closed forms are
// used only where they are well conditioned on [0, 1]: a leading coefficient between 1e-8 and
// 1e-2 of the largest other one (the roots that matter would sit behind the cancellation of
// huge normalised coefficients), or a polished root that does not zero the polynomial to
// 1e-9 of its coefficient sum, makes the caller use the derivative cascade instead.
template <int DEG>
__device__ __forceinline__ void newton_polish(const double (&c)[6], double& x) {
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    double v = c[DEG], d = 0.0;
#pragma unroll
    for (int m = DEG - 1; m >= 0; --m) { d = d * x + v; v = v * x + c[m]; }
    if (d != 0.0) {
      const double xn = x - v / d;
      if (isfinite(xn)) x = xn;
    }
  }
}

// Real roots of x^2 + b x + c (appended to r at n).
__device__ __forceinline__ void quad_roots(double b, double c, double* r, int& n) {
  const double disc = b * b - 4.0 * c;
  if (disc < 0.0) return;
  const double q = -0.5 * (b + copysign(sqrt(disc), b));
  if (q != 0.0) {
    r[n++] = q;
    r[n++] = c / q;
  } else {
    r[n++] = 0.0;   // b = c = 0
  }
}

// Real roots of x^3 + a x^2 + b x + c; returns the count, the largest first when all are real.
__device__ __forceinline__ int cubic_roots(double a, double b, double c, double* r) {
  const double a3 = a / 3.0;
  const double p = b - a * a3, q = (2.0 * a3 * a3 - b) * a3 + c;   // t^3 + p t + q, x = t - a/3
  const double hq = 0.5 * q, tp = p / 3.0;
  const double disc = hq * hq + tp * tp * tp;
  if (disc > 0.0) {
    // one real root: t = u - tp / u with u^3 = -q/2 - sign(q) sqrt(disc) (no cancellation)
    const double u = cbrt(-hq - copysign(sqrt(disc), hq));
    r[0] = (u != 0.0 ? u - tp / u : 0.0) - a3;
    return 1;
  }
  if (tp == 0.0) {   // p = q = 0: a triple root
    r[0] = -a3;
    return 1;
  }
  const double m = sqrt(-tp);
  const double arg = fmin(1.0, fmax(-1.0, -hq / (m * m * m)));
  const double phi = acos(arg) / 3.0;
  const double two_pi_3 = 2.0943951023931954923;
  r[0] = 2.0 * m * cos(phi) - a3;
  r[1] = 2.0 * m * cos(phi - two_pi_3) - a3;
  r[2] = 2.0 * m * cos(phi + two_pi_3) - a3;
  return 3;
}

// All real roots of the polynomial c of degree <= DEG (DEG <= 4), unsorted, unpolished; -1 where
// the closed forms are not well conditioned.
template <int DEG>
__device__ int closed_form_roots_raw(const double (&c)[6], double (&r)[4]) {
  static_assert(DEG <= 4, "closed forms exist up to degree 4");
  if constexpr (DEG <= 0) {
    return 0;
  } else {
    double big = 0.0;
#pragma unroll
    for (int m = 0; m < DEG; ++m) big = fmax(big, fabs(c[m]));
    if (!(fabs(c[DEG]) > 1e-8 * big)) return closed_form_roots_raw<DEG - 1>(c, r);
    if (!(fabs(c[DEG]) >= 1e-2 * big)) return -1;
    int n = 0;
    const double inv = 1.0 / c[DEG];
    if constexpr (DEG == 1) {
      r[n++] = -c[0] * inv;
    } else if constexpr (DEG == 2) {
      quad_roots(c[1] * inv, c[0] * inv, r, n);
    } else if constexpr (DEG == 3) {
      n = cubic_roots(c[2] * inv, c[1] * inv, c[0] * inv, r);
    } else {
      // Ferrari: x = y - a/4 gives y^4 + p y^2 + q y + s
      const double a = c[3] * inv, b = c[2] * inv, cc = c[1] * inv, d = c[0] * inv;
      const double a4 = 0.25 * a, aa = a4 * a4;
      const double p = b - 6.0 * aa;
      const double q = cc - 2.0 * b * a4 + 8.0 * aa * a4;
      const double sq = d - cc * a4 + b * aa - 3.0 * aa * aa;
      if (fabs(q) <= 1e-14 * (fabs(p) * fabs(p) + fabs(sq) + 1e-300)) {
        // biquadratic: y^2 = z with z^2 + p z + s = 0
        double z[2];
        int nz = 0;
        quad_roots(p, sq, z, nz);
        for (int i = 0; i < nz; ++i)
          if (z[i] >= 0.0) {
            const double y = sqrt(z[i]);
            r[n++] = y - a4;
            if (n < 4 && y != 0.0) r[n++] = -y - a4;
          }
      } else {
        // resolvent 8 m^3 + 8 p m^2 + (2 p^2 - 8 s) m - q^2 = 0 has a root m > 0 (its largest)
        double mr[3];
        const int nm = cubic_roots(p, 0.25 * p * p - sq, -0.125 * q * q, mr);
        double m = mr[0];
        for (int i = 1; i < nm; ++i) m = fmax(m, mr[i]);
        if (m > 0.0) {
          // y^4 + p y^2 + q y + s = (y^2 + p/2 + m)^2 - (w y - q / (2 w))^2 with w = sqrt(2 m)
          const double w = sqrt(2.0 * m);
          const double h0 = 0.5 * p + m, h1 = 0.5 * q / w;
          double y[4];
          int ny = 0;
          quad_roots(w, h0 - h1, y, ny);
          quad_roots(-w, h0 + h1, y, ny);
          for (int i = 0; i < ny; ++i) r[n++] = y[i] - a4;
        }
      }
    }
    return n;
  }
}

// The same, each root polished by Newton steps on the full polynomial; -1 where the closed
// forms are not well conditioned or a polished root fails the residual check.
template <int DEG>
__device__ int closed_form_roots(const double (&c)[6], double (&r)[4]) {
  const int n = closed_form_roots_raw<DEG>(c, r);
  double sum = 0.0;
#pragma unroll
  for (int m = 0; m <= DEG; ++m) sum += fabs(c[m]);
  for (int i = 0; i < n; ++i) {
    newton_polish<DEG>(c, r[i]);
    if (!(fabs(peval<DEG>(c, r[i])) <= 1e-9 * sum)) return -1;
  }
  return n;
}

// Real roots of c (degree <= DEG <= 4) strictly inside (a, b), ascending: the split points of
// [a, b] into monotone pieces when c is a derivative.
// Where the closed forms are not usable, or miss a sign change (an odd number of sign-changing
// roots is needed when c changes sign over [a, b]), the derivative cascade answers.
template <int DEG>
__device__ int interior_roots_cf(const double (&c)[6], double a, double b, double (&out)[5]) {
  double r[4];
  const int n = closed_form_roots<DEG>(c, r);
  if (n < 0) return real_roots<DEG>(c, a, b, out);
  int cnt = 0;
  for (int i = 0; i < n; ++i)
    if (r[i] > a && r[i] < b) {
      // insertion into the ascending list
      int j = cnt++;
      while (j > 0 && out[j - 1] > r[i]) { out[j] = out[j - 1]; --j; }
      out[j] = r[i];
    }
  const double ca = peval<DEG>(c, a), cb = peval<DEG>(c, b);
  if ((ca < 0.0 && cb > 0.0) || (ca > 0.0 && cb < 0.0)) {
    // an odd number of sign changes inside: count the found roots that change sign
    int changes = 0;
    for (int i = 0; i < cnt; ++i) {
      const double lo = 0.5 * ((i > 0 ? out[i - 1] : a) + out[i]);
      const double hi = 0.5 * (out[i] + (i + 1 < cnt ? out[i + 1] : b));
      if ((peval<DEG>(c, lo) < 0.0) != (peval<DEG>(c, hi) < 0.0)) ++changes;
    }
    if ((changes & 1) == 0) return real_roots<DEG>(c, a, b, out);
  }
  return cnt;
}

// Upper bound of the polynomial a on [0, s]: a_0 + sum_{m >= 1} max(0, a_m) s^m.
template <int K>
__device__ __forceinline__ double upper_bound(const double (&a)[6], double s) {
  double ub = a[0], sp = 1.0;
#pragma unroll
  for (int m = 1; m <= K; ++m) { sp *= s; ub += fmax(a[m], 0.0) * sp; }
  return ub;
}

// Called only for the few segments the bounds cannot rule out: kept out of line so that the
// root cascade does not raise the register pressure of the traversal loop.
// With closed_form the critical points (roots of the derivative, degree K - 1 <= 4) come from
// the closed forms, else from the derivative cascade.
template <class S>
__device__ __noinline__ double seg_max(const double (&a)[6], double s, int closed_form) {
  constexpr int K = S::K;
  double best = fmax(peval<K>(a, 0.0), peval<K>(a, s));
  double da[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int m = 0; m < K; ++m) da[m] = (m + 1) * a[m + 1];
  double crit[5];
  int nc;
  if constexpr (K <= 5) {
    nc = closed_form ? interior_roots_cf<K - 1>(da, 0.0, s, crit) : real_roots<K - 1>(da, 0.0, s, crit);
  } else {
    nc = real_roots<K - 1>(da, 0.0, s, crit);
  }
  for (int i = 0; i < nc; ++i) best = fmax(best, peval<K>(a, crit[i]));
  return best;
}

// First v in (0, s] where g = a - tau goes from < 0 to >= 0 on a monotone piece; -1 if none.
// With closed_form: the critical points from the closed forms (degree K - 1 <= 4), and for
// K <= 4 the root on the piece too (polished, it starts the safeguarded Newton iteration, which
// then ends at once); for K = 5 the piece's root comes from the safeguarded iteration alone.
template <class S>
__device__ __noinline__ double first_upward(const double (&g)[6], double s, int closed_form) {
  constexpr int K = S::K;
  double dg[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int m = 0; m < K; ++m) dg[m] = (m + 1) * g[m + 1];
  double crit[5];
  int nc;
  if constexpr (K <= 5) {
    nc = closed_form ? interior_roots_cf<K - 1>(dg, 0.0, s, crit) : real_roots<K - 1>(dg, 0.0, s, crit);
  } else {
    nc = real_roots<K - 1>(dg, 0.0, s, crit);
  }
  double pts[7];
  int np = 0;
  pts[np++] = 0.0;
  for (int i = 0; i < nc; ++i)
    if (crit[i] > 0.0 && crit[i] < s && crit[i] > pts[np - 1]) pts[np++] = crit[i];
  pts[np++] = s;
  double f0 = peval<K>(g, 0.0);
  for (int i = 0; i + 1 < np; ++i) {
    const double f1 = peval<K>(g, pts[i + 1]);
    if (f0 < 0.0 && f1 >= 0.0) {
      if (f1 == 0.0) return pts[i + 1];
      if constexpr (K <= 4) {
        if (closed_form) {
          double r[4];
          const int n = closed_form_roots<K>(g, r);
          for (int k = 0; k < n; ++k)   // (n = -1: no candidate; the bracketed iteration alone)
            if (r[k] > pts[i] && r[k] < pts[i + 1]) return solve_monotone<K>(g, pts[i], pts[i + 1], f0, r[k]);
        }
      }
      return solve_monotone<K>(g, pts[i], pts[i + 1], f0);
    }
    f0 = f1;
  }
  return -1.0;
}

// Ray root.  Each ray's clipped parameter interval is split into SUB equal sub-intervals,
// one per lane of a SUB-lane group (SUB divides the wavefront); splitting a cell's segment
// changes neither the maximum nor the crossings.
//  pass 1: each lane's maximum of f over its pieces; the group's maximum gives tau.
//  pass 2: each lane walks its pieces in order for the first upward crossing of tau (with the
//          face rule between consecutive pieces); an event at the start of lane j (j >= 1)
//          occurs when lane j-1 ends below tau and lane j starts at or above it (a face
//          crossing, or a crossing exactly at the split) and belongs to lane j-1's last cell.
//  The ray's root is the earliest event; the ray is dead when f >= tau at its entry point.
// grad f and (H r) at the root (physical units) from the cell's row; out of line, once per ray.
template <class S, typename T>
__device__ __forceinline__ void root_gradients(const T* __restrict__ row_ptr, const double (&u)[3], const double (&r)[3],
                                            double ih, double (&gout)[3], double (&hr)[3]) {
  constexpr int P = S::P, K = S::K;
  double row[P];
#pragma unroll
  for (int k = 0; k < P; ++k) row[k] = (double)row_ptr[k];
  double pw[3][K + 1];
  power_table<S>(u, pw);
  double val, g[3], hs[6];
  eval_poly<S, double, true, true>(row, pw, val, g, hs);
#pragma unroll
  for (int j = 0; j < 3; ++j) gout[j] = g[j] * ih;
  const double H[3][3] = {{hs[0], hs[1], hs[2]}, {hs[1], hs[3], hs[4]}, {hs[2], hs[4], hs[5]}};
#pragma unroll
  for (int j = 0; j < 3; ++j) hr[j] = (H[j][0] * r[0] + H[j][1] * r[1] + H[j][2] * r[2]) * ih * ih;
}

constexpr int kRootSub = 8;
// Root finding: closed forms (1, the default: every polynomial of degree <= 4, i.e. the roots of
// g for K <= 4 and the critical points for K <= 5) or the derivative cascade throughout (0, a test
// aid set by fc2t2_debug_root_cascade, so that the two can be compared on the same rays).
int g_root_closed_form = 1;
constexpr int kRootSmooth = FC2T2_ROOT_SMOOTH, kRootFace = FC2T2_ROOT_FACE, kRootGrazing = FC2T2_ROOT_GRAZING;

// Bounds of each finest cell's polynomial over the whole cell: with u in [-1/2, 1/2]^3,
// |f(u) - L_0| <= B = sum_{k != 0} |L_k| prod_j (1/2)^{k_j} / k_j!.  Stored as the float pair
// (L_0 - B, L_0 + B), widened by a relative 1e-6 and rounded outward, so that a segment of the
// cell can be ruled out (entirely below or above a level) without building its polynomial.
template <class S, typename T>
__global__ void __launch_bounds__(256) cell_bounds_kernel(const T* __restrict__ L, int64_t G,
                                                          float2* __restrict__ out) {
  constexpr int P = S::P, Ppad = S::Ppad;
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= G) return;
  double half[P];
  const double hu[3] = {0.5, 0.5, 0.5};
  monomials<S>(hu, half);
  const T* row = L + cell * Ppad;
  const double l0 = (double)row[0];
  double B = 0.0;
#pragma unroll
  for (int k = 1; k < P; ++k) B += fabs((double)row[k]) * half[k];
  const double pad = 1e-6 * (fabs(l0) + B) + 1e-30;
  float lo_b = (float)(l0 - B - pad), hi_b = (float)(l0 + B + pad);
  lo_b = nextafterf(lo_b, -INFINITY);
  hi_b = nextafterf(hi_b, INFINITY);
  out[cell] = make_float2(lo_b, hi_b);
}

template <class S, typename T>
__global__ void __launch_bounds__(64) ray_root_kernel(const T* __restrict__ L, const T* __restrict__ O,
                                                      const T* __restrict__ Rd, int64_t R, double t0, double t1,
                                                      double lo, double hi, double h, int n, double frac,
                                                      T* __restrict__ t_out, T* __restrict__ normal,
                                                      int32_t* __restrict__ hit, T* __restrict__ saved,
                                                      const float2* __restrict__ bounds,
                                                      unsigned long long* __restrict__ grazing,
                                                      const T* __restrict__ tau_in, int closed_form) {
  constexpr int P = S::P, Ppad = S::Ppad, K = S::K, SUB = kRootSub;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ray = gtid / SUB;
  const int part = (int)(gtid % SUB);
  const bool active = ray < R;
  const int64_t rr = active ? ray : 0;
  double o[3], r[3];
  load3(O, rr, o);
  load3(Rd, rr, r);
  const double ih = 1.0 / h;
  const double q[3] = {r[0] * ih, r[1] * ih, r[2] * ih};
  // the ray's clipped interval, then this lane's sub-interval [e0, e1]
  double ta_ray = t0, tb_ray = t1;
  bool live = active;
  {
    Dda clip;
    clip.init(o, r, t0, t1, lo, hi, h, n);
    ta_ray = clip.t;
    tb_ray = clip.t_end;
    live = live && clip.live;
  }
  const double step = (tb_ray - ta_ray) / SUB;
  const double e0 = part == 0 ? ta_ray : ta_ray + part * step;
  const double e1 = part == SUB - 1 ? tb_ray : ta_ray + (part + 1) * step;
  int64_t cell;
  int cc[3];
  double ta, tb;
  // ---- pass 0: a value the ray's maximum surely reaches: the largest value of f at a segment
  // midpoint (evaluated only where the cell's upper bound exceeds the largest so far).  Passes 0
  // and 1 only serve the level frac * max f; given levels skip them.
  const bool find_max = live && tau_in == nullptr;
  double lb = -INFINITY;
  if (find_max) {
    Dda dda;
    dda.init(o, r, e0, e1, lo, hi, h, n);
    while (dda.next(cell, cc, ta, tb)) {
      if ((double)bounds[cell].y <= lb) continue;
      const T* row = L + cell * Ppad;
      const double tm = 0.5 * (ta + tb);
      double u[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) u[j] = (o[j] + tm * r[j] - (lo + (cc[j] + 0.5) * h)) * ih;
      lb = fmax(lb, cell_eval<S>(row, u));
    }
  }
#pragma unroll
  for (int off = SUB / 2; off >= 1; off >>= 1) lb = fmax(lb, __shfl_xor(lb, off));
  // ---- pass 1.  The running maximum starts at lb, a value f takes on the ray: the maximum
  // over the segments is at least lb, so starting there changes nothing but skips the exact
  // maximisation of every segment whose bound stays below it.
  double fmax_v = lb;
  if (find_max) {
    Dda dda;
    dda.init(o, r, e0, e1, lo, hi, h, n);
    while (dda.next(cell, cc, ta, tb)) {
      // no value in this cell can exceed the running maximum (at least lb, a value the ray
      // surely reaches)
      if ((double)bounds[cell].y <= fmax_v) continue;
      T row[P];
#pragma unroll
      for (int k = 0; k < P; ++k) row[k] = L[cell * Ppad + k];
      double d[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) d[j] = (o[j] + ta * r[j] - (lo + (cc[j] + 0.5) * h)) * ih;
      double a[6];
      segment_poly<S>(row, d, q, tb - ta, a);
      // the exact segment maximum only matters when the segment can beat the best so far
      if (upper_bound<K>(a, 1.0) > fmax_v) fmax_v = fmax(fmax_v, seg_max<S>(a, 1.0, closed_form));
    }
  }
#pragma unroll
  for (int off = SUB / 2; off >= 1; off >>= 1) fmax_v = fmax(fmax_v, __shfl_xor(fmax_v, off));
  const double tau = tau_in ? (double)tau_in[rr] : frac * fmax_v;
  // ---- pass 2
  bool found = false, have_piece = false, ev_face = false;
  double t_ev = INFINITY, first_start = 0.0, last_end = 0.0, last_tb = 0.0;
  int64_t ev_cell = 0, last_cell = 0, first_cell = -1;
  int ev_c[3] = {0, 0, 0}, last_c[3] = {0, 0, 0};
  if (live && (tau_in != nullptr || fmax_v > -INFINITY)) {
    Dda dda;
    dda.init(o, r, e0, e1, lo, hi, h, n);
    double prev_end = 0.0;
    while (dda.next(cell, cc, ta, tb)) {
      // a cell entirely below or above the level is settled by its bounds: its piece has one
      // sign throughout, so it holds no crossing and only its sign matters at the faces
      const float2 bd = bounds[cell];
      const double side = (double)bd.y < tau ? -1.0 : ((double)bd.x > tau ? 1.0 : 0.0);
      if (side != 0.0) {
        if (!have_piece) {
          first_start = side;
          first_cell = cell;
          have_piece = true;
        } else if (!found && prev_end < 0.0 && side > 0.0) {   // crossing on a face
          t_ev = last_tb;
          ev_cell = last_cell;
          ev_c[0] = last_c[0]; ev_c[1] = last_c[1]; ev_c[2] = last_c[2];
          found = true;
          ev_face = true;
        }
        prev_end = side;
        last_end = side;
        last_tb = tb;
        last_cell = cell;
        last_c[0] = cc[0]; last_c[1] = cc[1]; last_c[2] = cc[2];
        if (found) break;
        continue;
      }
      T row[P];
#pragma unroll
      for (int k = 0; k < P; ++k) row[k] = L[cell * Ppad + k];
      double d[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) d[j] = (o[j] + ta * r[j] - (lo + (cc[j] + 0.5) * h)) * ih;
      double g[6];
      const double sl = tb - ta;
      segment_poly<S>(row, d, q, sl, g);
      g[0] -= tau;
      const double g0 = peval<K>(g, 0.0);
      if (!have_piece) {
        first_start = g0;
        first_cell = cell;
        have_piece = true;
      } else if (!found && prev_end < 0.0 && g0 >= 0.0) {   // crossing on a face: earlier piece
        t_ev = last_tb;
        ev_cell = last_cell;
        ev_c[0] = last_c[0]; ev_c[1] = last_c[1]; ev_c[2] = last_c[2];
        found = true;
        ev_face = true;
      }
      if (!found) {
        const double v = upper_bound<K>(g, 1.0) < 0.0 ? -1.0 : first_upward<S>(g, 1.0, closed_form);
        if (v >= 0.0) {
          t_ev = ta + sl * v;
          ev_cell = cell;
          ev_c[0] = cc[0]; ev_c[1] = cc[1]; ev_c[2] = cc[2];
          found = true;
        }
      }
      prev_end = peval<K>(g, 1.0);
      last_end = prev_end;
      last_tb = tb;
      last_cell = cell;
      last_c[0] = cc[0]; last_c[1] = cc[1]; last_c[2] = cc[2];
      if (found) break;
    }
  }
  // boundary event at the start of this lane: previous lane ends below, this lane starts at or above
  const int lane = threadIdx.x & 63;
  const int src = lane - 1;
  const double prev_last_end = __shfl(last_end, src < 0 ? 0 : src);
  const int prev_have = __shfl((int)have_piece, src < 0 ? 0 : src);
  const int64_t prev_last_cell = __shfl(last_cell, src < 0 ? 0 : src);
  const int pc0 = __shfl(last_c[0], src < 0 ? 0 : src), pc1 = __shfl(last_c[1], src < 0 ? 0 : src),
            pc2 = __shfl(last_c[2], src < 0 ? 0 : src);
  const double prev_last_tb = __shfl(last_tb, src < 0 ? 0 : src);
  if (part > 0 && have_piece && prev_have && prev_last_end < 0.0 && first_start >= 0.0) {
    // an event at this lane's start precedes any event inside it; it is a face crossing when
    // the two lanes' pieces there belong to different cells, else a root of one cell's
    // polynomial at the split point
    t_ev = prev_last_tb;
    ev_cell = prev_last_cell;
    ev_c[0] = pc0; ev_c[1] = pc1; ev_c[2] = pc2;
    found = true;
    ev_face = prev_last_cell != first_cell;
  }
  // the earliest event of the group (lowest lane on ties)
  double tmin = found ? t_ev : INFINITY;
#pragma unroll
  for (int off = SUB / 2; off >= 1; off >>= 1) tmin = fmin(tmin, __shfl_xor(tmin, off));
  const int group0 = lane & ~(SUB - 1);
  const uint64_t winners = __ballot(found && t_ev == tmin) >> group0;
  const int win = (int)__ffsll((unsigned long long)(winners & ((1ull << SUB) - 1))) - 1;
  const int64_t wcell = __shfl(ev_cell, group0 + (win < 0 ? 0 : win));
  const int w0 = __shfl(ev_c[0], group0 + (win < 0 ? 0 : win)), w1 = __shfl(ev_c[1], group0 + (win < 0 ? 0 : win)),
            w2 = __shfl(ev_c[2], group0 + (win < 0 ? 0 : win));
  const int wface = __shfl((int)ev_face, group0 + (win < 0 ? 0 : win));
  // dead ray: at or above the level at the entry point (lane 0's first piece)
  const double entry = __shfl(first_start, group0);
  const int entry_have = __shfl((int)have_piece, group0);
  const bool ray_hit = win >= 0 && entry_have && entry < 0.0;
  if (!active || part != 0) return;
  double gout[3] = {0.0, 0.0, 0.0}, hr[3] = {0.0, 0.0, 0.0}, qs[3] = {0.0, 0.0, 0.0}, rdg = 0.0;
  const double t_star = ray_hit ? tmin : NAN;
  if (ray_hit) {
    const int wc[3] = {w0, w1, w2};
    double u[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      qs[j] = o[j] + t_star * r[j];
      u[j] = (qs[j] - (lo + (wc[j] + 0.5) * h)) * ih;
    }
    root_gradients<S>(L + wcell * Ppad, u, r, ih, gout, hr);
    rdg = r[0] * gout[0] + r[1] * gout[1] + r[2] * gout[2];
  }
  // kind of the hit for the backward pass: the implicit function theorem needs r . grad f != 0
  int kind = kRootSmooth;
  if (ray_hit && wface) {
    kind = kRootFace;
  } else if (ray_hit) {
    const double gg = sqrt(gout[0] * gout[0] + gout[1] * gout[1] + gout[2] * gout[2]);
    const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (fabs(rdg) <= FC2T2_GRAZE_COS * rn * gg) {
      kind = kRootGrazing;
      atomicAdd(grazing, 1ull);
    }
  }
  t_out[ray] = (T)t_star;
  hit[ray] = ray_hit ? 1 : 0;
#pragma unroll
  for (int j = 0; j < 3; ++j) normal[ray * 3 + j] = (T)gout[j];
  T* sv = saved + ray * kRaySaved;
  sv[0] = (T)qs[0]; sv[1] = (T)qs[1]; sv[2] = (T)qs[2];
  put_cell(sv[3], ray_hit ? wcell : 0);
  sv[4] = (T)rdg;
  sv[5] = (T)hr[0]; sv[6] = (T)hr[1]; sv[7] = (T)hr[2];
  sv[8] = (T)tau;
  sv[9] = (T)t_star;
  sv[10] = (T)kind;
  sv[11] = T(0);
}

// Root insertion records: key = the root's cell for rays that hit, G otherwise.
template <typename T>
__global__ void __launch_bounds__(256) root_keys_kernel(const T* __restrict__ saved, const int32_t* __restrict__ hit,
                                                        int64_t R, int64_t G, uint32_t* __restrict__ keys) {
  const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ray >= R) return;
  const int64_t c = get_cell(saved[ray * kRaySaved + 3]);
  keys[ray] = (hit[ray] && c >= 0 && c < G) ? (uint32_t)c : (uint32_t)G;
}

template <class S, typename T>
struct RootInsert {
  const T* __restrict__ saved;
  const T* __restrict__ gt;
  const T* __restrict__ gn;
  double h;
  __device__ __forceinline__ void operator()(uint32_t ray, const T (&centre)[3], int, T (&v)[S::P],
                                             int64_t) const {
    constexpr int K = S::K;
    const T* sv = saved + (int64_t)ray * kRaySaved;
    double u[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) u[j] = ((double)sv[j] - (double)centre[j]) / h;
    const double rdg = (double)sv[4];
    double gnv[3] = {0.0, 0.0, 0.0};
    if (gn) {
#pragma unroll
      for (int j = 0; j < 3; ++j) gnv[j] = (double)gn[(int64_t)ray * 3 + j];
    }
    const double gtv = gt ? (double)gt[ray] : 0.0;
    // a face crossing or a grazing root inserts only the dipole term: at a face the root does
    // not move with L, at a grazing root its sensitivity is unbounded
    const double a = (int)sv[10] != kRootSmooth
                         ? 0.0
                         : -(gtv + gnv[0] * (double)sv[5] + gnv[1] * (double)sv[6] + gnv[2] * (double)sv[7]) / rdg;
    const double ih = 1.0 / h;
    double pw[3][K + 1];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      pw[j][0] = 1.0;
#pragma unroll
      for (int m = 1; m <= K; ++m) pw[j][m] = pw[j][m - 1] * u[j] / m;
    }
#pragma unroll
    for (int t = 0; t <= K; ++t)
#pragma unroll
      for (int p0 = t; p0 >= 0; --p0)
#pragma unroll
        for (int p1 = t - p0; p1 >= 0; --p1) {
          const int p2 = t - p0 - p1;
          double val = a * pw[0][p0] * pw[1][p1] * pw[2][p2];
          if (p0 >= 1) val += gnv[0] * ih * pw[0][p0 - 1] * pw[1][p1] * pw[2][p2];
          if (p1 >= 1) val += gnv[1] * ih * pw[0][p0] * pw[1][p1 - 1] * pw[2][p2];
          if (p2 >= 1) val += gnv[2] * ih * pw[0][p0] * pw[1][p1] * pw[2][p2 - 1];
          v[mi_pos3(p0, p1, p2)] = (T)val;
        }
  }
};

}  // namespace

namespace fc2t2 {

size_t ray_integral_bwd_ws(const fc2t2_plan_s* pl, int64_t R) {
  Carve c(nullptr);
  carve_records(c, pl, R * maxseg_for(pl), 1);
  return c.off;
}

size_t ray_root_bwd_ws(const fc2t2_plan_s* pl, int64_t R) {
  Carve c(nullptr);
  carve_records(c, pl, R, 0);
  return c.off;
}

fc2t2_status launch_ray_integral(const fc2t2_plan_s* pl, const void* L, const void* o, const void* r, double t0,
                                 double t1, int64_t R, void* y, hipStream_t s) {
  if (R == 0) return FC2T2_OK;
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  const dim3 grid((unsigned)ceil_div(R * kRayLanes, 64), pl->C);
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    if constexpr (S::D == 3) {
      if (pl->io == FC2T2_IO_F64)
        hipLaunchKernelGGL((ray_integral_kernel<S, double>), grid, dim3(64), 0, s, (const double*)L,
                           (const double*)o, (const double*)r, R, t0, t1, pl->lo, pl->hi, pl->h0, pl->n, pl->G,
                           (double*)y, pl->C);
      else
        hipLaunchKernelGGL((ray_integral_kernel<S, float>), grid, dim3(64), 0, s, (const float*)L,
                           (const float*)o, (const float*)r, R, t0, t1, pl->lo, pl->hi, pl->h0, pl->n, pl->G,
                           (float*)y, pl->C);
      st = FC2T2_OK;
    }
  });
  if (st) return st;
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

template <typename T>
fc2t2_status ray_integral_backward_t(const fc2t2_plan_s* pl, const T* o, const T* r, double t0, double t1,
                                     int64_t R, const T* gy, T* gL, void* ws, hipStream_t s) {
  const int maxseg = maxseg_for(pl);
  const int64_t slots = R * maxseg;
  Carve c(ws);
  RecordBufs b = carve_records(c, pl, slots, 1);
  hipLaunchKernelGGL((ray_records_kernel<T>), dim3((unsigned)ceil_div(R * kRayLanes, 256)), dim3(256), 0, s, o, r, R,
                     t0, t1, pl->lo, pl->hi, pl->h0, pl->n, pl->G, perlane_for(pl), b.keys, b.rec);
  FC2T2_LAUNCH_CHECK();
  fc2t2_status st = radix_sort_pairs(b.keys, b.keys_sorted, b.perm, slots, key_bits_for(pl->G + 1), b.scratch, s,
                                          (uint32_t)pl->G);
  if (st) return st;
  st = launch_cell_starts(b.keys_sorted, slots, pl->G, b.starts, s, sort_err_word(b.scratch, slots), pl->sort_fail);
  if (st) return st;
  st = FC2T2_EUNSUPPORTED;
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    if constexpr (S::D == 3) {
      SegmentInsert<S, T> fn{o, r, b.rec, gy, maxseg, pl->C, 1.0 / pl->h0};
      // records per occupied cell are few (a ray crosses a cell once): the number of real
      // segments is about 2.3 n per ray; below 12 per cell on average, two lanes per cell (a
      // shorter butterfly) are faster than four
      const int64_t recs = R * 2 * pl->n;
      st = recs < 12 * pl->G ? launch_reduce_cells_g<S, T, 2, false>(pl, b.starts, b.perm, gL, true, fn, s, nullptr, 0)
                             : launch_reduce_cells<S, T>(pl, b.starts, b.perm, recs, gL, true, fn, s);
    }
  });
  return st;
}

fc2t2_status ray_integral_backward(const fc2t2_plan_s* pl, const void* o, const void* r, double t0, double t1,
                                   int64_t R, const void* gy, void* gL, void* ws, hipStream_t s) {
  if (R == 0) return FC2T2_OK;
  return pl->io == FC2T2_IO_F64
             ? ray_integral_backward_t<double>(pl, (const double*)o, (const double*)r, t0, t1, R, (const double*)gy,
                                               (double*)gL, ws, s)
             : ray_integral_backward_t<float>(pl, (const float*)o, (const float*)r, t0, t1, R, (const float*)gy,
                                              (float*)gL, ws, s);
}

fc2t2_status launch_ray_root(const fc2t2_plan_s* pl, const void* L, const void* o, const void* r, double t0, double t1,
                             int64_t R, double frac, void* t, void* normal, int32_t* hit, void* saved, hipStream_t s,
                             const void* tau_in) {
  if (R == 0) return FC2T2_OK;
  if (!pl->cell_bounds) return FC2T2_EUNSUPPORTED;
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  const dim3 grid((unsigned)ceil_div(R * kRootSub, 64));
  const dim3 bgrid((unsigned)ceil_div(pl->G, 256));
  float2* bounds = (float2*)pl->cell_bounds;
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    if constexpr (S::D == 3) {
      if (pl->io == FC2T2_IO_F64) {
        hipLaunchKernelGGL((cell_bounds_kernel<S, double>), bgrid, dim3(256), 0, s, (const double*)L, pl->G, bounds);
        hipLaunchKernelGGL((ray_root_kernel<S, double>), grid, dim3(64), 0, s, (const double*)L, (const double*)o,
                           (const double*)r, R, t0, t1, pl->lo, pl->hi, pl->h0, pl->n, frac, (double*)t,
                           (double*)normal, hit, (double*)saved, bounds, pl->grazing, (const double*)tau_in,
                           g_root_closed_form);
      } else {
        hipLaunchKernelGGL((cell_bounds_kernel<S, float>), bgrid, dim3(256), 0, s, (const float*)L, pl->G, bounds);
        hipLaunchKernelGGL((ray_root_kernel<S, float>), grid, dim3(64), 0, s, (const float*)L, (const float*)o,
                           (const float*)r, R, t0, t1, pl->lo, pl->hi, pl->h0, pl->n, frac, (float*)t,
                           (float*)normal, hit, (float*)saved, bounds, pl->grazing, (const float*)tau_in,
                           g_root_closed_form);
      }
      st = FC2T2_OK;
    }
  });
  if (st) return st;
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

template <typename T>
fc2t2_status ray_root_backward_t(const fc2t2_plan_s* pl, const T* saved, const int32_t* hit, int64_t R, const T* gt,
                                 const T* gn, T* gL, void* ws, hipStream_t s) {
  Carve c(ws);
  RecordBufs b = carve_records(c, pl, R, 0);
  hipLaunchKernelGGL((root_keys_kernel<T>), dim3((unsigned)ceil_div(R, 256)), dim3(256), 0, s, saved, hit, R, pl->G,
                     b.keys);
  FC2T2_LAUNCH_CHECK();
  fc2t2_status st = radix_sort_pairs(b.keys, b.keys_sorted, b.perm, R, key_bits_for(pl->G + 1), b.scratch, s,
                                          (uint32_t)pl->G);
  if (st) return st;
  st = launch_cell_starts(b.keys_sorted, R, pl->G, b.starts, s, sort_err_word(b.scratch, R), pl->sort_fail);
  if (st) return st;
  st = FC2T2_EUNSUPPORTED;
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    if constexpr (S::D == 3) {
      RootInsert<S, T> fn{saved, gt, gn, pl->h0};
      st = launch_reduce_cells<S, T>(pl, b.starts, b.perm, R, gL, true, fn, s);
    }
  });
  return st;
}

void noalloc_setup(fc2t2_plan_s* pl) {
  static std::mutex mu;
  static void* addr[64] = {};
  pl->noalloc_scratch = nullptr;
  if (pl->device < 0 || pl->device >= 64) return;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[pl->device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return;
    addr[pl->device] = p;
  }
  pl->noalloc_scratch = addr[pl->device];
}

fc2t2_status ray_root_backward(const fc2t2_plan_s* pl, const void* saved, const int32_t* hit, int64_t R, const void* gt,
                               const void* gn, void* gL, void* ws, hipStream_t s) {
  if (R == 0) return FC2T2_OK;
  return pl->io == FC2T2_IO_F64
             ? ray_root_backward_t<double>(pl, (const double*)saved, hit, R, (const double*)gt, (const double*)gn,
                                           (double*)gL, ws, s)
             : ray_root_backward_t<float>(pl, (const float*)saved, hit, R, (const float*)gt, (const float*)gn,
                                          (float*)gL, ws, s);
}

}  // namespace fc2t2

extern "C" {

void fc2t2_debug_root_cascade(int enable) { g_root_closed_form = enable ? 0 : 1; }

static bool bad_rays(int64_t R) { return R < 0 || R > 0x7FFFFFFFll; }

fc2t2_status fc2t2_ray_integral(fc2t2_plan plan, const void* L, const void* o, const void* r, double t0, double t1,
                                int64_t R, void* y, hipStream_t stream) {
  if (!plan || !L || bad_rays(R) || !isfinite(t0) || !isfinite(t1)) return FC2T2_EINVAL;
  if (R > 0 && (!o || !r || !y)) return FC2T2_EINVAL;
  if (!rays_ok(plan)) return FC2T2_EUNSUPPORTED;
  StageScope tm(plan, FC2T2_STAGE_RAY, stream);
  return launch_ray_integral(plan, L, o, r, t0, t1, R, y, stream);
}

fc2t2_status fc2t2_ray_integral_backward(fc2t2_plan plan, const void* o, const void* r, double t0, double t1,
                                         int64_t R, const void* gy, void* gL, void* ws, size_t ws_bytes,
                                         hipStream_t stream) {
  if (!plan || !gL || bad_rays(R) || !isfinite(t0) || !isfinite(t1)) return FC2T2_EINVAL;
  if (R > 0 && (!o || !r || !gy)) return FC2T2_EINVAL;
  if (!rays_ok(plan)) return FC2T2_EUNSUPPORTED;
  if (R * (int64_t)maxseg_for(plan) > 0xFFFFFFFFll) return FC2T2_EUNSUPPORTED;
  if (R == 0) return FC2T2_OK;
  if (!ws || ws_bytes < ray_integral_bwd_ws(plan, R)) return FC2T2_EWORKSPACE;
  StageScope tm(plan, FC2T2_STAGE_RAY_T, stream);
  return ray_integral_backward(plan, o, r, t0, t1, R, gy, gL, ws, stream);
}

fc2t2_status fc2t2_ray_root(fc2t2_plan plan, const void* L, const void* o, const void* r, double t0, double t1,
                            int64_t R, double level_frac, void* t, void* normal, int32_t* hit, void* saved,
                            hipStream_t stream) {
  if (!plan || !L || bad_rays(R) || !isfinite(t0) || !isfinite(t1) || !isfinite(level_frac)) return FC2T2_EINVAL;
  if (R > 0 && (!o || !r || !t || !normal || !hit || !saved)) return FC2T2_EINVAL;
  if (!rays_ok(plan) || plan->C != 1) return FC2T2_EUNSUPPORTED;
  if (plan->G > 0xFFFFFFFFll) return FC2T2_EUNSUPPORTED;
  StageScope tm(plan, FC2T2_STAGE_RAY, stream);
  return launch_ray_root(plan, L, o, r, t0, t1, R, level_frac, t, normal, hit, saved, stream, nullptr);
}

fc2t2_status fc2t2_ray_root_at(fc2t2_plan plan, const void* L, const void* o, const void* r, double t0, double t1,
                               int64_t R, const void* tau, void* t, void* normal, int32_t* hit, void* saved,
                               hipStream_t stream) {
  if (!plan || !L || bad_rays(R) || !isfinite(t0) || !isfinite(t1)) return FC2T2_EINVAL;
  if (R > 0 && (!o || !r || !tau || !t || !normal || !hit || !saved)) return FC2T2_EINVAL;
  if (!rays_ok(plan) || plan->C != 1) return FC2T2_EUNSUPPORTED;
  if (plan->G > 0xFFFFFFFFll) return FC2T2_EUNSUPPORTED;
  StageScope tm(plan, FC2T2_STAGE_RAY, stream);
  return launch_ray_root(plan, L, o, r, t0, t1, R, 0.0, t, normal, hit, saved, stream, tau);
}

fc2t2_status fc2t2_ray_root_backward_noalloc(fc2t2_plan plan, const void* saved, const int32_t* hit, int64_t R,
                                             const void* gt, const void* gn, void* gL, hipStream_t stream) {
  if (!plan || !gL || bad_rays(R)) return FC2T2_EINVAL;
  if (R > 0 && (!saved || !hit)) return FC2T2_EINVAL;
  if (!rays_ok(plan) || plan->C != 1) return FC2T2_EUNSUPPORTED;
  if (R == 0 || (!gt && !gn)) return FC2T2_OK;
  if (ray_root_bwd_ws(plan, R) > (size_t)FC2T2_NOALLOC_SCRATCH_BYTES) return FC2T2_ESCRATCH;
  if (!plan->noalloc_scratch) return FC2T2_EHIP;
  return ray_root_backward(plan, saved, hit, R, gt, gn, gL, plan->noalloc_scratch, stream);
}

fc2t2_status fc2t2_ray_root_backward(fc2t2_plan plan, const void* saved, const int32_t* hit, int64_t R, const void* gt,
                                     const void* gn, void* gL, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!plan || !gL || bad_rays(R)) return FC2T2_EINVAL;
  if (R > 0 && (!saved || !hit)) return FC2T2_EINVAL;
  if (!rays_ok(plan) || plan->C != 1) return FC2T2_EUNSUPPORTED;
  if (R == 0 || (!gt && !gn)) return FC2T2_OK;
  if (!ws || ws_bytes < ray_root_bwd_ws(plan, R)) return FC2T2_EWORKSPACE;
  StageScope tm(plan, FC2T2_STAGE_RAY_T, stream);
  return ray_root_backward(plan, saved, hit, R, gt, gn, gL, ws, stream);
}

}  // extern "C"

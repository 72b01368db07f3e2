// Volumetric rendering on the finest-level local expansions (section 6.1.2) and its backward
// (section 6.2.2); dim 3, four channels: density sigma (channel 0) and colour c = (R, G, B)
// (channels 1..3).
//
// Along a ray, y = int T sigma c dt + bg T_end with T = mexp(S) and S the optical depth from
// the entry point; mexp is the degree-4 polynomial closest to exp(-x) in L2 on [0, 5].  Inside
// one cell every factor is a polynomial of the normalised segment parameter x in [0, 1]:
// sigma and c of degree K (line to polynomial, section 5.1.1), S of degree K + 1 and T of
// degree 4 (K + 1), so c sigma T has degree 6K + 4 and the N = 3K + 3 point Gauss-Legendre
// rule integrates it exactly (up to rounding): no sampling along the ray.  The walk stops
// after the first cell whose exit depth exceeds 4.5 (the fit is used below 5 only); then
// T_end = 0, else T_end = mexp(D_end).
//
// Backward: the exact derivative of this forward.  Colour channel k receives
//   y_bar_k int mono sigma T dt,
// the density channel int mono H dt with
//   H(t) = c_y(t) T(t) + E - Gb - int_{t_a}^t c_y sigma mexp'(S),    c_y = sum_k y_bar_k c_k,
// E = int over the whole walk of c_y sigma mexp'(S), plus (y_bar . bg) mexp'(D_end) when the
// walk did not stop, and Gb the same integral up to the cell's entry: a change of sigma at t
// changes S at every later point.  mono = u^k / k! in cell units u = (q - centre) / h, so the
// output is the cotangent of the cell-scaled rows.  The stop decision is not differentiated.
//
// Records: one per piece of the walk (a cell's segment, or its part on one of the lanes that
// share a ray; cell as the sort key; [ta, tb] and the piece's weights at K + 1 points as payload,
// see below), sorted by cell and reduced per cell into the four rows.  Every per-piece quantity
// runs in FP64 (the vector FP64 and FP32 rates are equal without packed FP32); only the
// expansion rows and the output rows use the IO type.
#include <math.h>

#include <vector>

#include "plan.h"
#include "raywalk.h"
#include "segreduce.h"

using namespace fc2t2;

namespace {

constexpr int kMaxNodes = 18;        // 3K + 3 for K <= 5
constexpr double kStopDepth = FC2T2_VOLUME_STOP_DEPTH;
constexpr double kMexpRange = 5.0;   // mexp fits exp(-x) on [0, kMexpRange]

struct VolumeConsts {
  double m[5];                         // mexp, low to high degree in x
  double mp[4];                        // its derivative
  double x[kMaxNodes], w[kMaxNodes];   // Gauss-Legendre nodes and weights on [0, 1]
  double bg[3];                        // background colour
};

// The degree-4 polynomial closest to exp(-x) in L2 on [0, 5].  In t = x / 5 the shifted
// Legendre polynomials Q_j(t) = P_j(2t - 1) are orthogonal on [0, 1] with <Q_j, Q_j> =
// 1 / (2j + 1), so the projection is sum_j (2j + 1) <exp(-5t), Q_j> Q_j.  The inner products
// come from a 40-point Gauss-Legendre rule (exact to rounding for this entire integrand).
void mexp_fit(double (&m)[5]) {
  std::vector<double> t, w;
  gauss_legendre(40, t, w);
  double Q[5][5] = {};   // Q[j][k]: coefficient of t^k; Q_{j+1} = ((2j+1)(2t-1) Q_j - j Q_{j-1}) / (j+1)
  Q[0][0] = 1.0;
  Q[1][0] = -1.0;
  Q[1][1] = 2.0;
  for (int j = 1; j < 4; ++j)
    for (int k = 0; k < 5; ++k)
      Q[j + 1][k] = ((2.0 * j + 1.0) * ((k ? 2.0 * Q[j][k - 1] : 0.0) - Q[j][k]) - j * Q[j - 1][k]) / (j + 1.0);
  double c[5] = {};
  for (int j = 0; j < 5; ++j) {
    double a = 0.0;
    for (size_t i = 0; i < t.size(); ++i) {
      const double tt = 0.5 * (1.0 + t[i]);
      double q = 0.0;
      for (int k = 4; k >= 0; --k) q = q * tt + Q[j][k];
      a += 0.5 * w[i] * exp(-kMexpRange * tt) * q;
    }
    a *= 2.0 * j + 1.0;
    for (int k = 0; k < 5; ++k) c[k] += a * Q[j][k];
  }
  for (int k = 0; k < 5; ++k) m[k] = c[k] / pow(kMexpRange, k);
}

VolumeConsts volume_consts(int K, const double* bg) {
  VolumeConsts vc = {};
  mexp_fit(vc.m);
  for (int k = 0; k < 4; ++k) vc.mp[k] = (k + 1) * vc.m[k + 1];
  std::vector<double> t, w;
  gauss_legendre(3 * K + 3, t, w);
  for (int i = 0; i < 3 * K + 3; ++i) {
    vc.x[i] = 0.5 * (1.0 + t[i]);
    vc.w[i] = 0.5 * w[i];
  }
  for (int k = 0; k < 3; ++k) vc.bg[k] = bg ? bg[k] : 0.0;
  return vc;
}

// Horner evaluation of the first N coefficients of c.
template <int N, int CAP>
__device__ __forceinline__ double poly_at(const double (&c)[CAP], double x) {
  static_assert(N <= CAP, "coefficients");
  double v = c[N - 1];
#pragma unroll
  for (int m = N - 2; m >= 0; --m) v = v * x + c[m];
  return v;
}

__device__ __forceinline__ double mexp_at(const VolumeConsts& vc, double s) {
  return (((vc.m[4] * s + vc.m[3]) * s + vc.m[2]) * s + vc.m[1]) * s + vc.m[0];
}
__device__ __forceinline__ double mexp_d(const VolumeConsts& vc, double s) {
  return ((vc.mp[3] * s + vc.mp[2]) * s + vc.mp[1]) * s + vc.mp[0];
}

// Entry offset of the segment from the cell centre and the direction, both in cell units.
__device__ __forceinline__ void seg_local(const double (&o)[3], const double (&r)[3], double ta, const int (&cc)[3],
                                          double lo, double h, double (&d)[3], double (&q)[3]) {
  const double ih = 1.0 / h;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    d[j] = (o[j] + ta * r[j] - (lo + (cc[j] + 0.5) * h)) * ih;
    q[j] = r[j] * ih;
  }
}

// Optical depth on the segment in x: S(x) = D + s int_0^x sigma, from sigma's coefficients.
template <int K>
__device__ __forceinline__ void depth_poly(const double (&bs)[6], double D, double s, double (&sx)[K + 2]) {
  sx[0] = D;
#pragma unroll
  for (int m = 0; m <= K; ++m) sx[m + 1] = s * bs[m] / (m + 1);
}

// ---------------------------------------------------------------------------------------
// Lanes per ray.  kRayLanes neighbouring lanes walk the sub-ranges of one ray.  The optical
// depth at a lane's start and the stop decision need the cells before it, so every lane first
// walks its sub-range for the density alone: the depth it adds (dsum) and the largest depth,
// relative to its start, at which one of its pieces leaves a cell (dmax; a piece that ends at a
// cut inside a cell is not a cell exit, the ray's last piece is).  A scan over the lanes then
// gives each lane its start depth and the largest exit depth of every cell before it; a lane
// after a cell whose exit depth exceeds the threshold adds nothing, and the lane holding that
// cell stops after it, as a walk of the whole ray would.
__device__ __forceinline__ void depth_scan(double s, double m, int l, double& ex_s, double& ex_m, double& tot_s,
                                           double& tot_m) {
  // (sum, max) pairs combine as (a.s + b.s, max(a.m, a.s + b.m)), earlier lane first
  double is = s, im = m;
#pragma unroll
  for (int off = 1; off < kRayLanes; off <<= 1) {
    const double ps = __shfl_up(is, off, kRayLanes), pm = __shfl_up(im, off, kRayLanes);
    if (l >= off) {
      im = fmax(pm, ps + im);
      is = ps + is;
    }
  }
  tot_s = __shfl(is, kRayLanes - 1, kRayLanes);
  tot_m = __shfl(im, kRayLanes - 1, kRayLanes);
  ex_s = __shfl_up(is, 1, kRayLanes);
  ex_m = __shfl_up(im, 1, kRayLanes);
  if (l == 0) {
    ex_s = 0.0;
    ex_m = -INFINITY;
  }
}

// The density pass of one lane over [a, b] (see above).  With `cache`, piece j's density
// polynomial is also left in the first three double2 of its record slot (ray_slot(ray, l, j)),
// where the records pass reads it back instead of evaluating the density row again.
template <class S, typename T>
__device__ void density_pass(const T* __restrict__ L, const double (&o)[3], const double (&r)[3], double a, double b,
                             bool last_lane, double lo, double hi, double h, int n, double& dsum, double& dmax,
                             double2* __restrict__ cache = nullptr, int64_t ray = 0, int l = 0, int perlane = 0) {
  constexpr int K = S::K, Ppad = S::Ppad;
  Dda dda;
  dda.init(o, r, a, b, lo, hi, h, n);
  dsum = 0.0;
  dmax = -INFINITY;
  int64_t cell;
  int cc[3];
  double ta, tb;
  int j = 0;
  while (dda.next(cell, cc, ta, tb)) {
    const double sl = tb - ta;
    double d[3], q[3];
    seg_local(o, r, ta, cc, lo, h, d, q);
    double bs[6];
    segment_poly<S>(L + cell * Ppad, d, q, sl, bs);
    if (cache && j < perlane) {
      double2* cb = cache + ray_slot(ray, l, j, perlane) * (K + 2);
      cb[0] = make_double2(bs[0], bs[1]);
      cb[1] = make_double2(bs[2], bs[3]);
      cb[2] = make_double2(bs[4], bs[5]);
    }
    ++j;
    double sx[K + 2];
    depth_poly<K>(bs, dsum, sl, sx);
    dsum = poly_at<K + 2>(sx, 1.0);
    if (dda.at_plane || last_lane) dmax = fmax(dmax, dsum);
  }
}

// ---------------------------------------------------------------------------------------
// Forward: kRayLanes lanes per ray (density pass, scan, then the lane's share of the colour
// integral from its start depth); the lanes' colour sums are added by a butterfly.
template <class S, typename T>
__global__ void __launch_bounds__(64) volume_kernel(const T* __restrict__ L, const T* __restrict__ O,
                                                    const T* __restrict__ Rd, int64_t R, double t0, double t1,
                                                    double lo, double hi, double h, int n, int64_t G,
                                                    VolumeConsts vc, T* __restrict__ y, T* __restrict__ trans) {
  constexpr int K = S::K, Ppad = S::Ppad, NQ = 3 * K + 3;
  static_assert(NQ <= kMaxNodes, "quadrature nodes");
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ray = gid / kRayLanes;
  const int l = (int)(gid % kRayLanes);
  const bool last_lane = l == kRayLanes - 1;
  double o[3], r[3], ta_r = 0.0, tb_r = 0.0;
  bool hit = false;
  if (ray < R) {
    load3(O, ray, o);
    load3(Rd, ray, r);
    hit = ray_range(o, r, t0, t1, lo, hi, ta_r, tb_r);
  }
  const double a = lane_cut(ta_r, tb_r, l), b = lane_cut(ta_r, tb_r, l + 1);
  double dsum = 0.0, dmax = -INFINITY;
  if (hit) density_pass<S>(L, o, r, a, b, last_lane, lo, hi, h, n, dsum, dmax);
  double D, before_max, D_end, max_exit;
  depth_scan(dsum, dmax, l, D, before_max, D_end, max_exit);
  const int64_t cs = G * Ppad;   // channel stride
  double y0 = 0.0, y1 = 0.0, y2 = 0.0;
  if (hit && !(before_max > kStopDepth)) {
    Dda dda;
    dda.init(o, r, a, b, lo, hi, h, n);
    int64_t cell;
    int cc[3];
    double ta, tb;
    while (dda.next(cell, cc, ta, tb)) {
      const double sl = tb - ta;
      double d[3], q[3];
      seg_local(o, r, ta, cc, lo, h, d, q);
      const T* row = L + cell * Ppad;
      double bs[6], b0[6], b1[6], b2[6];
      segment_poly<S>(row, d, q, sl, bs);
      segment_poly<S>(row + cs, d, q, sl, b0);
      segment_poly<S>(row + 2 * cs, d, q, sl, b1);
      segment_poly<S>(row + 3 * cs, d, q, sl, b2);
      double sx[K + 2];
      depth_poly<K>(bs, D, sl, sx);
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const double x = vc.x[i];
        const double w = sl * vc.w[i] * poly_at<K + 1>(bs, x) * mexp_at(vc, poly_at<K + 2>(sx, x));
        y0 += w * poly_at<K + 1>(b0, x);
        y1 += w * poly_at<K + 1>(b1, x);
        y2 += w * poly_at<K + 1>(b2, x);
      }
      D = poly_at<K + 2>(sx, 1.0);
      if ((dda.at_plane || last_lane) && D > kStopDepth) break;
    }
  }
#pragma unroll
  for (int off = kRayLanes / 2; off >= 1; off >>= 1) {
    y0 += __shfl_xor(y0, off, kRayLanes);
    y1 += __shfl_xor(y1, off, kRayLanes);
    y2 += __shfl_xor(y2, off, kRayLanes);
  }
  if (ray < R && l == 0) {
    const double Tend = max_exit > kStopDepth ? 0.0 : mexp_at(vc, D_end);
    y[3 * ray] = (T)(y0 + vc.bg[0] * Tend);
    y[3 * ray + 1] = (T)(y1 + vc.bg[1] * Tend);
    y[3 * ray + 2] = (T)(y2 + vc.bg[2] * Tend);
    if (trans) trans[ray] = (T)Tend;
  }
}

// ---------------------------------------------------------------------------------------
// Backward, per segment.  Every channel's cotangent row gets sum over the segment of
// a(x) mono(u(x)) dx for a weight function a; mono(u(x)) is a polynomial of degree <= K in x,
// so the segment's whole contribution is fixed by K + 1 numbers: the weights alpha_m at the
// K + 1 Chebyshev-Lobatto points z_m of the segment, alpha_m = s int_0^1 a(x) l_m(x) dx with
// l_m the Lagrange basis on the z_m; then the row gets sum_m alpha_m mono(u(z_m)).  With
// Lam[m][i] = l_m(x_i) at the Gauss-Legendre nodes, Gam[m][i] = int_{x_i}^1 l_m and
// beta_m = int_0^1 l_m (host constants):
//   colour k:  alpha_m = y_bar_k s sum_i w_i (sigma T)(x_i) Lam[m][i];
//   density:   alpha_m = s sum_i w_i (c_y T)(x_i) Lam[m][i] - s^2 sum_i w_i g(x_i) Gam[m][i]
//                        + s (E - Gb) beta_m,        g = c_y sigma mexp'(S),
// where the middle term is the running integral of g with the order of integration swapped
// (int_0^1 l_m(x) int_0^x g = int_0^1 g(y) int_y^1 l_m); every integrand has degree <= 6K + 4,
// so each sum is exact.  The records pass computes the alphas (the E term, which needs the
// ray's total, is added in the reduction, which runs after the whole walk).
struct VolumeProj {
  double lam[6][kMaxNodes];   // l_m(x_i)
  double gam[6][kMaxNodes];   // int_{x_i}^1 l_m
  double beta[6];             // int_0^1 l_m
};

VolumeProj volume_proj(int K, const VolumeConsts& vc) {
  VolumeProj vp = {};
  double z[6];
  for (int m = 0; m <= K; ++m) z[m] = lobatto_node(K, m);
  auto ell = [&](int m, double x) {
    double v = 1.0;
    for (int j = 0; j <= K; ++j)
      if (j != m) v *= (x - z[j]) / (z[m] - z[j]);
    return v;
  };
  std::vector<double> t, w;
  gauss_legendre(8, t, w);   // exact for the degree-K basis
  auto integral = [&](int m, double a, double b) {
    double acc = 0.0;
    for (size_t k = 0; k < t.size(); ++k) acc += w[k] * ell(m, a + 0.5 * (b - a) * (1.0 + t[k]));
    return 0.5 * (b - a) * acc;
  };
  for (int m = 0; m <= K; ++m) {
    for (int i = 0; i < 3 * K + 3; ++i) {
      vp.lam[m][i] = ell(m, vc.x[i]);
      vp.gam[m][i] = integral(m, vc.x[i], 1.0);
    }
    vp.beta[m] = integral(m, 0.0, 1.0);
  }
  return vp;
}

// Records: the forward's walk again (density pass and scan first), with the colour cotangents
// folded into c_y.  Lane l of ray i writes its pieces to its own slots (ray_slot): key = the
// cell; rec[(K + 2) slot] = (ta, tb), then (alpha_m of the density without the E term, with Gb
// counted from the lane's start; alpha_m of sigma T without y_bar_k) for m = 0..K; unused
// slots get the key G (sorted after every cell).  Ex[i kRayLanes + l]
// receives E - Gb0, with E the ray's total of int c_y sigma mexp'(S) (plus (y_bar . bg)
// mexp'(D_end) when the ray did not stop) and Gb0 the same integral over the lanes before l, so
// that the reduction's term s Ex beta_m completes each record of the lane.
template <class S, typename T>
__global__ void __launch_bounds__(64) volume_records_kernel(const T* __restrict__ L, const T* __restrict__ O,
                                                            const T* __restrict__ Rd, int64_t R, double t0,
                                                            double t1, double lo, double hi, double h, int n,
                                                            int64_t G, VolumeConsts vc, VolumeProj vp,
                                                            const T* __restrict__ gy, int perlane,
                                                            uint32_t* __restrict__ keys, double2* __restrict__ rec,
                                                            double* __restrict__ Ex) {
  constexpr int K = S::K, Ppad = S::Ppad, NQ = 3 * K + 3;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ray = gid / kRayLanes;
  const int l = (int)(gid % kRayLanes);
  const bool last_lane = l == kRayLanes - 1;
  double o[3], r[3], ta_r = 0.0, tb_r = 0.0;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  bool hit = false;
  if (ray < R) {
    load3(O, ray, o);
    load3(Rd, ray, r);
    g0 = (double)gy[3 * ray];
    g1 = (double)gy[3 * ray + 1];
    g2 = (double)gy[3 * ray + 2];
    hit = ray_range(o, r, t0, t1, lo, hi, ta_r, tb_r);
  }
  const double a = lane_cut(ta_r, tb_r, l), b = lane_cut(ta_r, tb_r, l + 1);
  double dsum = 0.0, dmax = -INFINITY;
  if (hit) density_pass<S>(L, o, r, a, b, last_lane, lo, hi, h, n, dsum, dmax, rec, ray, l, perlane);
  double D, before_max, D_end, max_exit;
  depth_scan(dsum, dmax, l, D, before_max, D_end, max_exit);
  const int64_t cs = G * Ppad;
  double Gb = 0.0;
  int j = 0;
  if (hit && !(before_max > kStopDepth)) {
    Dda dda;
    dda.init(o, r, a, b, lo, hi, h, n);
    int64_t cell;
    int cc[3];
    double ta, tb;
    while (j < perlane && dda.next(cell, cc, ta, tb)) {
      const double sl = tb - ta;
      double d[3], q[3];
      seg_local(o, r, ta, cc, lo, h, d, q);
      const int64_t slot = ray_slot(ray, l, j, perlane);
      double2* rr = rec + slot * (K + 2);
      const T* row = L + cell * Ppad;
      double bs[6], b0[6], b1[6], b2[6];
      {
        const double2 c0 = rr[0], c1 = rr[1], c2 = rr[2];   // the density pass's polynomial
        bs[0] = c0.x; bs[1] = c0.y; bs[2] = c1.x; bs[3] = c1.y; bs[4] = c2.x; bs[5] = c2.y;
      }
      segment_poly<S>(row + cs, d, q, sl, b0);
      segment_poly<S>(row + 2 * cs, d, q, sl, b1);
      segment_poly<S>(row + 3 * cs, d, q, sl, b2);
      double cy[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) cy[m] = g0 * b0[m] + g1 * b1[m] + g2 * b2[m];
      double sx[K + 2];
      depth_poly<K>(bs, D, sl, sx);
      double ad[K + 1], as[K + 1];
#pragma unroll
      for (int m = 0; m <= K; ++m) ad[m] = as[m] = 0.0;
      double gseg = 0.0;
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const double x = vc.x[i];
        const double sg = poly_at<K + 1>(bs, x), cv = poly_at<K + 1>(cy, x), Sv = poly_at<K + 2>(sx, x);
        const double Tv = mexp_at(vc, Sv), gi = cv * sg * mexp_d(vc, Sv);
        gseg += vc.w[i] * gi;
        const double hA = vc.w[i] * sl * cv * Tv, hB = vc.w[i] * sl * sl * gi, hS = vc.w[i] * sl * sg * Tv;
#pragma unroll
        for (int m = 0; m <= K; ++m) {
          ad[m] += hA * vp.lam[m][i] - hB * vp.gam[m][i];
          as[m] += hS * vp.lam[m][i];
        }
      }
      keys[slot] = (uint32_t)cell;
      rr[0] = make_double2(ta, tb);
#pragma unroll
      for (int m = 0; m <= K; ++m) rr[1 + m] = make_double2(ad[m] - sl * Gb * vp.beta[m], as[m]);
      ++j;
      Gb += sl * gseg;
      D = poly_at<K + 2>(sx, 1.0);
      if ((dda.at_plane || last_lane) && D > kStopDepth) break;
    }
  }
  if (ray < R)
    for (; j < perlane; ++j) keys[ray_slot(ray, l, j, perlane)] = (uint32_t)G;
  // the running integral at each lane's start, and the ray's total
  double is = Gb;
#pragma unroll
  for (int off = 1; off < kRayLanes; off <<= 1) {
    const double ps = __shfl_up(is, off, kRayLanes);
    if (l >= off) is += ps;
  }
  const double gb_tot = __shfl(is, kRayLanes - 1, kRayLanes);
  const double gb0 = is - Gb;
  if (ray < R) {
    const double gbg = g0 * vc.bg[0] + g1 * vc.bg[1] + g2 * vc.bg[2];
    const double E = gb_tot + (max_exit > kStopDepth ? 0.0 : gbg * mexp_d(vc, D_end));
    Ex[gid] = E - gb0;
  }
}

// Per-cell reduction of the records into the four channel rows: density row += sum_m
// (alpha_m + s E beta_m) mono(u_m); colour row k += y_bar_k sum_m alpha'_m mono(u_m).  A group
// of GROUP lanes owns a cell; inside it, four neighbouring lanes share a record and take one row
// each (so a lane holds P sums, not four rows), and the GROUP / 4 record lanes walk the cell's
// records in a strided order, all of a record's gathers in flight together.  The record lanes'
// partial rows are added by a butterfly, and the rows are written into out.
struct VolumeBeta {
  double beta[6];
};

template <class S, typename T, int GROUP>
__global__ void __launch_bounds__(256) volume_reduce_kernel(const uint32_t* __restrict__ starts,
                                                            const uint32_t* __restrict__ perm, int64_t G, int n,
                                                            double lo, double h, const T* __restrict__ O,
                                                            const T* __restrict__ Rd, const double2* __restrict__ rec,
                                                            const double* __restrict__ Ex, const T* __restrict__ gy,
                                                            int perlane, VolumeBeta vb, T* __restrict__ out) {
  constexpr int K = S::K, P = S::P, Ppad = S::Ppad;
  constexpr int RL = GROUP / 4;   // record lanes per cell
  static_assert(RL >= 1, "four lanes per record");
  constexpr int CPW = kWave / GROUP;
  constexpr Lobatto<K> LB{};
  const int lane = threadIdx.x & (kWave - 1);
  const int lane_g = lane & (GROUP - 1);
  const int ch = lane_g & 3, rl = lane_g >> 2;   // this lane's row and record lane
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t wave_id = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t cs = G * Ppad;
  for (int64_t c0 = wave_id * CPW; c0 < G; c0 += waves * CPW) {
    const int64_t cell = c0 + lane / GROUP;
    const bool valid = cell < G;
    const uint32_t rb = valid ? starts[cell] : 0u, re = valid ? starts[cell + 1] : 0u;
    T acc[P];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] = T(0);
    int cc[3];
    decode_cell<3, T>(valid ? cell : 0, n, cc);
    for (uint32_t ri = rb + rl; ri < re; ri += RL) {
      const uint32_t slot = perm[ri];
      const int64_t ray = slot / ((int64_t)perlane * kRayLanes), lane_id = ray * kRayLanes + slot % kRayLanes;
      double o[3], r[3];
      load3(O, ray, o);
      load3(Rd, ray, r);
      const double2* rr = rec + (int64_t)slot * (K + 2);
      const double2 tt = rr[0];
      double2 al[K + 1];
#pragma unroll
      for (int m = 0; m <= K; ++m) al[m] = rr[1 + m];
      const double e_ray = Ex[lane_id];
      const T g = ch > 0 ? gy[3 * ray + ch - 1] : T(0);
      const double sl = tt.y - tt.x;
      double d[3], q[3];
      seg_local(o, r, tt.x, cc, lo, h, d, q);
      const double es = sl * e_ray;
#pragma unroll
      for (int m = 0; m <= K; ++m) {
        const T w = ch == 0 ? (T)(al[m].x + es * vb.beta[m]) : g * (T)al[m].y;
        const double xs = sl * LB.x[m];
        T u[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) u[j] = (T)(d[j] + q[j] * xs);
        T mono[P];
        monomials<S>(u, mono);
#pragma unroll
        for (int k = 0; k < P; ++k) acc[k] += w * mono[k];
      }
    }
#pragma unroll
    for (int off = GROUP / 2; off >= 4; off >>= 1)
#pragma unroll
      for (int k = 0; k < P; ++k) acc[k] += __shfl_xor(acc[k], off, GROUP);
    if (valid && re > rb) {
#pragma unroll
      for (int k = 0; k < P; ++k)
        if (k % RL == rl) out[ch * cs + cell * Ppad + k] += acc[k];
    }
  }
}

template <class S, typename T, int GROUP>
fc2t2_status launch_volume_reduce(const fc2t2_plan_s* pl, const uint32_t* starts, const uint32_t* perm, const T* o,
                                  const T* r, const double2* rec, const double* Ex, const T* gy, int perlane,
                                  const VolumeBeta& vb, T* gL, hipStream_t s) {
  const int threads = 256;
  const int64_t need = ceil_div(pl->G * GROUP, threads);
  const int64_t blocks = need < 16384 ? need : 16384;
  hipLaunchKernelGGL((volume_reduce_kernel<S, T, GROUP>), dim3((unsigned)blocks), dim3(threads), 0, s, starts, perm,
                     pl->G, pl->n, pl->lo, pl->h0, o, r, rec, Ex, gy, perlane, vb, gL);
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

bool volume_ok(const fc2t2_plan_s* pl) { return pl->dim == 3 && pl->C == 4; }

}  // namespace

namespace fc2t2 {

size_t ray_volume_bwd_ws(const fc2t2_plan_s* pl, int64_t R) {
  Carve c(nullptr);
  carve_records(c, pl, R * maxseg_for(pl), pl->K + 2);
  c.take<double>(R * kRayLanes);
  return c.off;
}

}  // namespace fc2t2

namespace {

fc2t2_status launch_volume(const fc2t2_plan_s* pl, const void* L, const void* o, const void* r, double t0, double t1,
                           int64_t R, const double* bg, void* y, void* trans, hipStream_t s) {
  if (R == 0) return FC2T2_OK;
  const VolumeConsts vc = volume_consts(pl->K, bg);
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  const dim3 grid((unsigned)ceil_div(R * kRayLanes, 64));
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    if constexpr (S::D == 3) {
      if (pl->io == FC2T2_IO_F64)
        hipLaunchKernelGGL((volume_kernel<S, double>), grid, dim3(64), 0, s, (const double*)L, (const double*)o,
                           (const double*)r, R, t0, t1, pl->lo, pl->hi, pl->h0, pl->n, pl->G, vc, (double*)y,
                           (double*)trans);
      else
        hipLaunchKernelGGL((volume_kernel<S, float>), grid, dim3(64), 0, s, (const float*)L, (const float*)o,
                           (const float*)r, R, t0, t1, pl->lo, pl->hi, pl->h0, pl->n, pl->G, vc, (float*)y,
                           (float*)trans);
      st = FC2T2_OK;
    }
  });
  if (st) return st;
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

template <typename T>
fc2t2_status volume_backward_t(const fc2t2_plan_s* pl, const T* L, const T* o, const T* r, double t0, double t1,
                               int64_t R, const double* bg, const T* gy, T* gL, void* ws, hipStream_t s) {
  const int maxseg = maxseg_for(pl);
  const int64_t slots = R * maxseg;
  Carve c(ws);
  RecordBufs b = carve_records(c, pl, slots, pl->K + 2);
  double* Ex = c.take<double>(R * kRayLanes);
  const VolumeConsts vc = volume_consts(pl->K, bg);
  const VolumeProj vp = volume_proj(pl->K, vc);
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    if constexpr (S::D == 3) {
      hipLaunchKernelGGL((volume_records_kernel<S, T>), dim3((unsigned)ceil_div(R * kRayLanes, 64)), dim3(64), 0, s, L,
                         o, r, R, t0, t1, pl->lo, pl->hi, pl->h0, pl->n, pl->G, vc, vp, gy, perlane_for(pl), b.keys,
                         b.rec, Ex);
      st = FC2T2_OK;
    }
  });
  if (st) return st;
  FC2T2_LAUNCH_CHECK();
  st = radix_sort_pairs(b.keys, b.keys_sorted, b.perm, slots, key_bits_for(pl->G + 1), b.scratch, s,
                                          (uint32_t)pl->G);
  if (st) return st;
  st = launch_cell_starts(b.keys_sorted, slots, pl->G, b.starts, s, sort_err_word(b.scratch, slots), pl->sort_fail);
  if (st) return st;
  st = FC2T2_EUNSUPPORTED;
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    if constexpr (S::D == 3) {
      VolumeBeta vb;
      for (int m = 0; m < 6; ++m) vb.beta[m] = vp.beta[m];
      // record lanes per cell from the mean records per cell (a ray crosses about 2.3 n cells),
      // four lanes per record
      switch (reduce_group_for(R * 2 * pl->n, pl->G)) {
        case 4: st = launch_volume_reduce<S, T, 16>(pl, b.starts, b.perm, o, r, b.rec, Ex, gy, perlane_for(pl), vb, gL, s); break;
        default: st = launch_volume_reduce<S, T, 64>(pl, b.starts, b.perm, o, r, b.rec, Ex, gy, perlane_for(pl), vb, gL, s); break;
      }
    }
  });
  return st;
}

bool bad_rays(int64_t R) { return R < 0 || R > 0x7FFFFFFFll; }

}  // namespace

extern "C" {

fc2t2_status fc2t2_ray_volume(fc2t2_plan plan, const void* L, const void* o, const void* r, double t0, double t1,
                              int64_t R, const double* bg, void* y, void* trans, hipStream_t stream) {
  if (!plan || !L || bad_rays(R) || !isfinite(t0) || !isfinite(t1)) return FC2T2_EINVAL;
  if (R > 0 && (!o || !r || !y)) return FC2T2_EINVAL;
  if (bg && !(isfinite(bg[0]) && isfinite(bg[1]) && isfinite(bg[2]))) return FC2T2_EINVAL;
  if (!volume_ok(plan) || plan->K > 5) return FC2T2_EUNSUPPORTED;
  StageScope tm(plan, FC2T2_STAGE_RAY, stream);
  return launch_volume(plan, L, o, r, t0, t1, R, bg, y, trans, stream);
}

fc2t2_status fc2t2_ray_volume_backward(fc2t2_plan plan, const void* L, const void* o, const void* r, double t0,
                                       double t1, int64_t R, const double* bg, const void* gy, void* gL, void* ws,
                                       size_t ws_bytes, hipStream_t stream) {
  if (!plan || !L || !gL || bad_rays(R) || !isfinite(t0) || !isfinite(t1)) return FC2T2_EINVAL;
  if (R > 0 && (!o || !r || !gy)) return FC2T2_EINVAL;
  if (bg && !(isfinite(bg[0]) && isfinite(bg[1]) && isfinite(bg[2]))) return FC2T2_EINVAL;
  if (!volume_ok(plan) || plan->K > 5) return FC2T2_EUNSUPPORTED;
  if (R * (int64_t)maxseg_for(plan) > 0xFFFFFFFFll) return FC2T2_EUNSUPPORTED;
  if (R == 0) return FC2T2_OK;
  if (!ws || ws_bytes < ray_volume_bwd_ws(plan, R)) return FC2T2_EWORKSPACE;
  StageScope tm(plan, FC2T2_STAGE_RAY_T, stream);
  return plan->io == FC2T2_IO_F64
             ? volume_backward_t<double>(plan, (const double*)L, (const double*)o, (const double*)r, t0, t1, R, bg,
                                         (const double*)gy, (double*)gL, ws, stream)
             : volume_backward_t<float>(plan, (const float*)L, (const float*)o, (const float*)r, t0, t1, R, bg,
                                        (const float*)gy, (float*)gL, ws, stream);
}

}  // extern "C"

// Ray traversal pieces shared by the ray layers (rays.hip) and the volumetric layer
// (volume.hip): the cell-by-cell walk, the segment polynomial and the record workspace.
#pragma once

#include "plan.h"

namespace fc2t2 {

// ---------------------------------------------------------------------------------------
// Per-axis state is kept in scalars (no runtime-indexed arrays, which would live in
// scratch memory); the axis of the next crossing is chosen with selects.
struct Dda {
  double ox, oy, oz, rx, ry, rz;
  double lo, h;
  int n;
  double t, t_end;
  int cx, cy, cz, sx, sy, sz;
  double mx, my, mz;   // parameter of the next plane crossing per axis
  bool live;
  bool at_plane;       // the last piece ended at a cell face (see next())

  __device__ static double plane_t(double lo, double h, int c, int st, double o, double r) {
    if (st == 0) return INFINITY;
    const int k = st > 0 ? c + 1 : c;
    return (lo + (double)k * h - o) / r;
  }

  __device__ static void start_axis(double lo, double hi, double h, int n, double o, double r, double& ta,
                                    double& tb, bool& live) {
    if (r == 0.0) {
      if (o < lo || o > hi) live = false;
    } else {
      const double a = (lo - o) / r, b = (hi - o) / r;
      ta = fmax(ta, fmin(a, b));
      tb = fmin(tb, fmax(a, b));
    }
  }

  __device__ static void first_cell(double lo, double h, int n, double o, double r, double ta, int& c, int& st,
                                    double& m) {
    st = r > 0.0 ? 1 : (r < 0.0 ? -1 : 0);
    const int cj = (int)floor((o + ta * r - lo) / h);
    c = cj < 0 ? 0 : (cj > n - 1 ? n - 1 : cj);
    m = plane_t(lo, h, c, st, o, r);
    // the entry point can sit on a plane: move past planes that lie at or behind ta
    for (int guard = 0; guard < 2 && st != 0 && m <= ta; ++guard) {
      const int nc = c + st;
      if (nc < 0 || nc > n - 1) break;
      c = nc;
      m = plane_t(lo, h, c, st, o, r);
    }
  }

  __device__ void init(const double (&o_)[3], const double (&r_)[3], double t0, double t1, double lo_,
                       double hi_, double h_, int n_) {
    lo = lo_;
    h = h_;
    n = n_;
    ox = o_[0]; oy = o_[1]; oz = o_[2];
    rx = r_[0]; ry = r_[1]; rz = r_[2];
    double ta = t0, tb = t1;
    live = true;
    start_axis(lo_, hi_, h_, n_, ox, rx, ta, tb, live);
    start_axis(lo_, hi_, h_, n_, oy, ry, ta, tb, live);
    start_axis(lo_, hi_, h_, n_, oz, rz, ta, tb, live);
    if (!(tb > ta)) live = false;
    t = ta;
    t_end = tb;
    at_plane = false;
    first_cell(lo, h, n, ox, rx, ta, cx, sx, mx);
    first_cell(lo, h, n, oy, ry, ta, cy, sy, my);
    first_cell(lo, h, n, oz, rz, ta, cz, sz, mz);
  }

  // Next segment of positive length: cell index (row-major) and [ta, tb].  at_plane is set when
  // the segment ends at a cell face, including a face that lies within rounding past t_end (a
  // cut between two lanes' sub-ranges can land a few ulps before a face; the segment then
  // still ends its cell, and the next lane starts in the next cell).
  __device__ bool next(int64_t& cell, int (&cc)[3], double& ta, double& tb) {
    while (live && t < t_end) {
      const int j = (my < mx) ? ((mz < my) ? 2 : 1) : ((mz < mx) ? 2 : 0);
      const double tm = j == 0 ? mx : (j == 1 ? my : mz);
      const double tn = fmin(tm, t_end);
      const double t_prev = t;
      at_plane = tm <= t_end + 1e-12 * fabs(t_end);
      cc[0] = cx; cc[1] = cy; cc[2] = cz;
      t = tn;
      if (tn < t_end) {
        if (j == 0) {
          cx += sx;
          if (cx < 0 || cx > n - 1) live = false; else mx = plane_t(lo, h, cx, sx, ox, rx);
        } else if (j == 1) {
          cy += sy;
          if (cy < 0 || cy > n - 1) live = false; else my = plane_t(lo, h, cy, sy, oy, ry);
        } else {
          cz += sz;
          if (cz < 0 || cz > n - 1) live = false; else mz = plane_t(lo, h, cz, sz, oz, rz);
        }
      } else {
        live = false;
      }
      if (tn > t_prev) {
        cell = ((int64_t)cc[0] * n + cc[1]) * n + cc[2];
        ta = t_prev;
        tb = tn;
        return true;
      }
    }
    return false;
  }
};

template <typename T>
__device__ __forceinline__ void load3(const T* p, int64_t i, double (&v)[3]) {
  v[0] = (double)p[3 * i];
  v[1] = (double)p[3 * i + 1];
  v[2] = (double)p[3 * i + 2];
}

// Segment polynomial (line to polynomial, section 5.1.1).  The restriction of a cell's
// expansion to a segment is a polynomial of degree <= K; it is recovered exactly (up to
// rounding) from its values at the K + 1 Chebyshev-Lobatto points of the segment, through
// Newton divided differences, as b(x) = sum_m b_m x^m in the normalised parameter
// x = (t - t_a) / s in [0, 1].  Each value is a nested Horner evaluation of the cell
// polynomial from the FP32 row with FP64 accumulation.
__host__ __device__ constexpr double lobatto_node(int K, int i) {
  // (1 - cos(i pi / K)) / 2 for K <= 5, from the exact cosines
  constexpr double c5a = 0.80901699437494742410, c5b = 0.30901699437494742410;   // cos(pi/5), cos(2pi/5)
  constexpr double s2 = 0.70710678118654752440;                                  // cos(pi/4)
  if (i == 0) return 0.0;
  if (i == K) return 1.0;
  switch (K) {
    case 2: return 0.5;
    case 3: return i == 1 ? 0.25 : 0.75;
    case 4: return i == 1 ? 0.5 * (1.0 - s2) : (i == 2 ? 0.5 : 0.5 * (1.0 + s2));
    case 5: return i == 1 ? 0.5 * (1.0 - c5a) : (i == 2 ? 0.5 * (1.0 - c5b) : (i == 3 ? 0.5 * (1.0 + c5b) : 0.5 * (1.0 + c5a)));
  }
  return 0.0;
}

template <int K>
struct Lobatto {
  double x[K + 1];
  double inv[K + 1][K + 1];   // inv[j][i] = 1 / (x_i - x_{i-j})
  constexpr Lobatto() : x{}, inv{} {
    for (int i = 0; i <= K; ++i) x[i] = lobatto_node(K, i);
    for (int j = 1; j <= K; ++j)
      for (int i = j; i <= K; ++i) inv[j][i] = 1.0 / (x[i] - x[i - j]);
  }
};

template <class S, typename R>
__device__ __forceinline__ double cell_eval(const R* row, const double (&u)[3]) {
  constexpr int K = S::K;
  double acc_a = 0.0;
#pragma unroll
  for (int a = K; a >= 0; --a) {
    double acc_b = 0.0;
#pragma unroll
    for (int b = K - a; b >= 0; --b) {
      double acc_c = (double)row[mi_pos3(a, b, K - a - b)];
#pragma unroll
      for (int c = K - a - b - 1; c >= 0; --c) acc_c = (double)row[mi_pos3(a, b, c)] + acc_c * u[2] * (1.0 / (c + 1));
      acc_b = acc_c + acc_b * u[1] * (1.0 / (b + 1));
    }
    acc_a = acc_b + acc_a * u[0] * (1.0 / (a + 1));
  }
  return acc_a;
}

template <class S, typename R>
__device__ void segment_poly(const R* row, const double (&d)[3], const double (&q)[3], double s, double (&b)[6]) {
  constexpr int K = S::K;
  constexpr Lobatto<K> LB{};
  double c[K + 1];
#pragma unroll
  for (int i = 0; i <= K; ++i) {
    const double v = s * LB.x[i];
    const double u[3] = {d[0] + q[0] * v, d[1] + q[1] * v, d[2] + q[2] * v};
    c[i] = cell_eval<S>(row, u);
  }
  // divided differences
#pragma unroll
  for (int j = 1; j <= K; ++j)
#pragma unroll
    for (int i = K; i >= j; --i) c[i] = (c[i] - c[i - 1]) * LB.inv[j][i];
  // Newton form -> monomial coefficients: b = c_K; b = b (x - x_i) + c_i for i = K-1 .. 0
#pragma unroll
  for (int m = 0; m < 6; ++m) b[m] = 0.0;
  b[0] = c[K];
#pragma unroll
  for (int i = K - 1; i >= 0; --i) {
#pragma unroll
    for (int m = K; m >= 1; --m) b[m] = b[m - 1] - LB.x[i] * b[m];
    b[0] = c[i] - LB.x[i] * b[0];
  }
}

// ---------------------------------------------------------------------------------------
// Lanes per ray in the walking kernels: the clipped parameter range [ta, tb] of a ray is cut
// into kRayLanes equal sub-ranges, walked by neighbouring lanes of one wave.  A cell crossed by
// a cut is split into two pieces; each piece is integrated exactly, so the sum over a ray is
// unchanged up to rounding.
constexpr int kRayLanes = 8;

// Clipped parameter range of a ray in the domain box; false if it misses the box.
__device__ inline bool ray_range(const double (&o)[3], const double (&r)[3], double t0, double t1, double lo,
                                 double hi, double& ta, double& tb) {
  bool live = true;
  ta = t0;
  tb = t1;
  Dda::start_axis(lo, hi, 0.0, 0, o[0], r[0], ta, tb, live);
  Dda::start_axis(lo, hi, 0.0, 0, o[1], r[1], ta, tb, live);
  Dda::start_axis(lo, hi, 0.0, 0, o[2], r[2], ta, tb, live);
  return live && tb > ta;
}

// Cut c (0..kRayLanes) of [ta, tb]: lane l walks [cut(l), cut(l + 1)]; neighbours compute the
// shared cut with the same expression, so the sub-ranges tile [ta, tb] exactly.
__device__ __forceinline__ double lane_cut(double ta, double tb, int c) {
  return c == 0 ? ta : (c == kRayLanes ? tb : ta + (tb - ta) * ((double)c / kRayLanes));
}

// Record slots per lane.  Along axis j a sub-range of length (tb - ta) / kRayLanes crosses at
// most |r_j| (tb - ta) / (kRayLanes h) + 1 faces, and |r_j| (tb - ta) <= n h inside the box, so
// a lane has at most 3 n / kRayLanes + 4 pieces; two more absorb rounding.  Piece j of lane l of
// ray i is slot (i perlane + j) kRayLanes + l: a ray owns maxseg = kRayLanes perlane consecutive
// slots (its ray is slot / maxseg, its lane slot % kRayLanes), and the lanes' j-th records are
// neighbours, so a wave's record writes fill whole lines.
inline int perlane_for(const fc2t2_plan_s* pl) { return 3 * pl->n / kRayLanes + 6; }
inline int maxseg_for(const fc2t2_plan_s* pl) { return kRayLanes * perlane_for(pl); }
__host__ __device__ inline int64_t ray_slot(int64_t ray, int lane, int j, int perlane) {
  return ((ray * perlane + j) * kRayLanes) + lane;
}

struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <typename X>
  X* take(size_t count) {
    X* p = base ? (X*)(base + off) : nullptr;
    off += align256(count * sizeof(X));
    return p;
  }
};

struct RecordBufs {
  uint32_t *keys, *keys_sorted, *perm, *starts;
  double2* rec;
  void* scratch;
};

// Keys, sorted keys, permutation, cell starts, rec_per_slot double2 payload words per slot
// and the sort's scratch, carved from one workspace.
inline RecordBufs carve_records(Carve& c, const fc2t2_plan_s* pl, int64_t slots, int rec_per_slot) {
  RecordBufs b;
  b.keys = c.take<uint32_t>(slots);
  b.keys_sorted = c.take<uint32_t>(slots);
  b.perm = c.take<uint32_t>(slots);
  b.starts = c.take<uint32_t>(pl->G + 1);
  b.rec = rec_per_slot ? c.take<double2>(slots * rec_per_slot) : nullptr;
  b.scratch = c.take<char>(radix_sort_scratch_bytes(slots));
  return b;
}

inline bool rays_ok(const fc2t2_plan_s* pl) { return pl->dim == 3; }

}  // namespace fc2t2

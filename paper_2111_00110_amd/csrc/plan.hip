// Plan creation: geometry, the M2L derivative tensors (FP64 on the GPU) and the M2M/L2L
// shift tables.  Section 3 of the paper (multilevel expansion, K^{M2M}, K^{L2L}, K^{M2L}).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <utility>
#include <vector>

#include "plan.h"

using namespace fc2t2;

namespace {

// ---------------------------------------------------------------------------------------
// Partial derivatives of a kernel psi at the cell-centre offsets.
//
// Radial kernels psi(x) = phi(|x|^2): with delta(y) = |x0 + y|^2 - |x0|^2 = sum_i y_i (2 x0_i + y_i),
//   psi(x0 + y) = sum_m phi^(m)(|x0|^2) delta^m / m!,
// and the coefficient of y^g in delta^m / m! is
//   sum over j with |j| = m, ceil(g_i/2) <= j_i <= g_i of prod_i C(j_i, g_i - j_i) (2 x0_i)^(2 j_i - g_i) / j_i!
// so d^g psi(x0) = g! sum_j phi^(|j|)(|x0|^2) prod_i C(j_i, g_i - j_i) (2 x0_i)^(2 j_i - g_i) / j_i!.
//   Gaussian: phi(u) = exp(-u / (2 s^2)),  phi^(m) = (-1/(2 s^2))^m phi.
//   IMQ:      phi(u) = (u + e^2)^(-1/2),   phi^(m) = (-1)^m (2m-1)!! / 2^m (u + e^2)^(-1/2 - m).
// Polynomial kernels: d^g sum_a c_a x^a = sum_{a >= g} c_a a!/(a-g)! x^(a-g).
// ---------------------------------------------------------------------------------------

__device__ double dfact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

__device__ double dbinom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

__device__ double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

// phi^(m)(u) for the radial kernels.
__device__ double radial_deriv(int kind, double param, double u, int m) {
  if (kind == FC2T2_GAUSSIAN) {
    const double a = -1.0 / (2.0 * param * param);
    return ipow(a, m) * exp(a * u);
  }
  // IMQ
  const double base = u + param * param;
  double c = 1.0;
  for (int i = 0; i < m; ++i) c *= -(2.0 * i + 1.0) * 0.5;
  return c * pow(base, -0.5 - m);
}

// d^g psi(x) for the plan's kernel.
__device__ double psi_deriv(int kind, double param, const double* __restrict__ coef,
                            const int* __restrict__ coef_exps, int n_coef, const int (&g)[3], const double (&x)[3]) {
  double val = 0.0;
  if (kind == FC2T2_POLY) {
    for (int a = 0; a < n_coef; ++a) {
      const int e0 = coef_exps[3 * a], e1 = coef_exps[3 * a + 1], e2 = coef_exps[3 * a + 2];
      if (e0 < g[0] || e1 < g[1] || e2 < g[2]) continue;
      double term = coef[a];
      term *= dfact(e0) / dfact(e0 - g[0]) * ipow(x[0], e0 - g[0]);
      term *= dfact(e1) / dfact(e1 - g[1]) * ipow(x[1], e1 - g[1]);
      term *= dfact(e2) / dfact(e2 - g[2]) * ipow(x[2], e2 - g[2]);
      val += term;
    }
    return val;
  }
  const double u = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  // j_i ranges over [ceil(g_i/2), g_i]
  const int lo0 = (g[0] + 1) / 2, lo1 = (g[1] + 1) / 2, lo2 = (g[2] + 1) / 2;
  for (int j0 = lo0; j0 <= g[0]; ++j0) {
    const double f0 = dbinom(j0, g[0] - j0) * ipow(2.0 * x[0], 2 * j0 - g[0]) / dfact(j0);
    for (int j1 = lo1; j1 <= g[1]; ++j1) {
      const double f1 = dbinom(j1, g[1] - j1) * ipow(2.0 * x[1], 2 * j1 - g[1]) / dfact(j1);
      for (int j2 = lo2; j2 <= g[2]; ++j2) {
        const double f2 = dbinom(j2, g[2] - j2) * ipow(2.0 * x[2], 2 * j2 - g[2]) / dfact(j2);
        val += radial_deriv(kind, param, u, j0 + j1 + j2) * f0 * f1 * f2;
      }
    }
  }
  return val * dfact(g[0]) * dfact(g[1]) * dfact(g[2]);
}

__device__ __forceinline__ void offset_of(int dim, int oi, int (&o)[3]) {
  o[0] = o[1] = o[2] = 0;
  int r = oi;
  for (int j = dim - 1; j >= 0; --j) { o[j] = r % 7 - 3; r /= 7; }
}

// One thread per (level, offset, derivative multi-index g): D[lvl][o][g] = d^g psi(-o h_lvl).
__global__ void derivs_kernel(int dim, int kind, double param, const double* __restrict__ coef,
                              const int* __restrict__ coef_exps, int n_coef,
                              const int* __restrict__ g_exps, int n_g, int levels,
                              const double* __restrict__ hl, int n_off, double* __restrict__ D) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)levels * n_off * n_g;
  if (tid >= total) return;
  const int gi = (int)(tid % n_g);
  const int oi = (int)((tid / n_g) % n_off);
  const int lvl = (int)(tid / ((int64_t)n_g * n_off));
  int o[3];
  offset_of(dim, oi, o);
  const double h = hl[lvl];
  double x[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < dim; ++j) x[j] = -o[j] * h;
  const int g[3] = {g_exps[3 * gi], g_exps[3 * gi + 1], g_exps[3 * gi + 2]};
  D[tid] = psi_deriv(kind, param, coef, coef_exps, n_coef, g, x);
}

// ---------------------------------------------------------------------------------------
// Least-squares M2L tensors (section 3.1).  In cell-scaled units the row k of the tensor is the
// coefficient vector c of the polynomial sum_{|n| <= K} c_n u^n / n! closest in L2 over the
// source cell u in [-1/2, 1/2]^d to h^|k| d^k psi(-o h - u h); the integral is tensor
// Gauss-Legendre quadrature (K + 2 nodes per dimension), so c = Pi f with the P x J matrix Pi
// built on the host from the nodes and weights.

// F[o][j][k] = h^|k| d^k psi(-o h - u_j h) for one level; u [J][3].
__global__ void lsq_values_kernel(int dim, int kind, double param, const double* __restrict__ coef,
                                  const int* __restrict__ coef_exps, int n_coef,
                                  const int* __restrict__ k_exps, int P, const double* __restrict__ u, int J,
                                  double h, int n_off, double* __restrict__ F) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)n_off * J * P) return;
  const int k = (int)(tid % P);
  const int j = (int)((tid / P) % J);
  const int oi = (int)(tid / ((int64_t)P * J));
  int o[3];
  offset_of(dim, oi, o);
  double x[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < dim; ++d) x[d] = (-o[d] - u[3 * j + d]) * h;
  const int g[3] = {k_exps[3 * k], k_exps[3 * k + 1], k_exps[3 * k + 2]};
  F[tid] = ipow(h, g[0] + g[1] + g[2]) * psi_deriv(kind, param, coef, coef_exps, n_coef, g, x);
}

// T[lvl][o][n][k] = sum_j Pi[n][j] F[o][j][k] for one level (zero for k >= P).
template <typename T>
__global__ void lsq_project_kernel(int P, int Ppad, int J, int n_off, const double* __restrict__ Pi,
                                   const double* __restrict__ F, T* __restrict__ out) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)n_off * P * Ppad) return;
  const int k = (int)(tid % Ppad);
  const int n = (int)((tid / Ppad) % P);
  const int oi = (int)(tid / ((int64_t)Ppad * P));
  if (k >= P) { out[tid] = T(0); return; }
  const double* f = F + (int64_t)oi * J * P + k;
  const double* pr = Pi + (int64_t)n * J;
  double acc = 0.0;
  for (int j = 0; j < J; ++j) acc += pr[j] * f[(int64_t)j * P];
  out[tid] = (T)acc;
}

// T[lvl][o][n][k] = h^(|k|+|n|) (-1)^|n| D[lvl][o][pos(k+n)], zero for k >= P.
template <typename T>
__global__ void pack_m2l_kernel(int dim, int K, int P, int Ppad, int levels, int n_off, int n_g,
                                const double* __restrict__ hl, const int* __restrict__ exps,
                                const double* __restrict__ D, T* __restrict__ out) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)levels * n_off * P * Ppad;
  if (tid >= total) return;
  const int k = (int)(tid % Ppad);
  const int n = (int)((tid / Ppad) % P);
  const int oi = (int)((tid / ((int64_t)Ppad * P)) % n_off);
  const int lvl = (int)(tid / ((int64_t)Ppad * P * n_off));
  if (k >= P) { out[tid] = T(0); return; }
  const int a0 = exps[3 * k] + exps[3 * n], a1 = exps[3 * k + 1] + exps[3 * n + 1],
            a2 = exps[3 * k + 2] + exps[3 * n + 2];
  const int pos = dim == 2 ? mi_pos2(a0, a1) : mi_pos3(a0, a1, a2);
  const int dk = exps[3 * k] + exps[3 * k + 1] + exps[3 * k + 2];
  const int dn = exps[3 * n] + exps[3 * n + 1] + exps[3 * n + 2];
  double v = D[((int64_t)lvl * n_off + oi) * n_g + pos];
  v *= ipow(hl[lvl], dk + dn);
  if (dn & 1) v = -v;
  out[tid] = (T)v;
}

}  // namespace

namespace fc2t2 {

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on P_Q from the usual cosine
// guesses, P_Q by the three-term recurrence.
void gauss_legendre(int Q, std::vector<double>& t, std::vector<double>& w) {
  t.assign(Q, 0.0);
  w.assign(Q, 0.0);
  for (int i = 0; i < Q; ++i) {
    double x = cos(M_PI * (i + 0.75) / (Q + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= Q; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = Q * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) <= 1e-16) {
        // derivative at the converged node for the weight
        p0 = 1.0;
        p1 = x;
        for (int k = 2; k <= Q; ++k) {
          const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = Q * (x * p1 - p0) / (x * x - 1.0);
        break;
      }
    }
    t[i] = x;
    w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

}  // namespace fc2t2

namespace {

// Weighted least-squares projection for the fitted tensors: nodes u [J][3] (cell units, tensor
// Gauss-Legendre with K + 2 nodes per dimension on [-1/2, 1/2]) and Pi [P][J] with
// c = Pi f the coefficients of sum_n c_n u^n / n! fitting values f at the nodes.  The fit is
// solved in t = 2u with the basis t^n (Householder QR of sqrt(w) t^n), then rescaled:
// c_n = 2^|n| n! c_t[n].
bool lsq_projection(int dim, int K, const std::vector<int>& k_exps, std::vector<double>& u, std::vector<double>& Pi,
                    int& J) {
  const int Q = K + 2, P = nterms(dim, K);
  std::vector<double> t1, w1;
  gauss_legendre(Q, t1, w1);
  J = 1;
  for (int d = 0; d < dim; ++d) J *= Q;
  u.assign((size_t)J * 3, 0.0);
  std::vector<double> sw(J), A((size_t)J * P);   // A column-major: A[c * J + j]
  for (int j = 0; j < J; ++j) {
    int r = j;
    double wt = 1.0, tj[3] = {0.0, 0.0, 0.0};
    for (int d = dim - 1; d >= 0; --d) {
      const int q = r % Q;
      r /= Q;
      tj[d] = t1[q];
      wt *= w1[q];
    }
    for (int d = 0; d < dim; ++d) u[3 * j + d] = 0.5 * tj[d];
    sw[j] = sqrt(wt);
    for (int c = 0; c < P; ++c) {
      double m = sw[j];
      for (int d = 0; d < dim; ++d)
        for (int e = 0; e < k_exps[3 * c + d]; ++e) m *= tj[d];
      A[(size_t)c * J + j] = m;
    }
  }
  // Householder QR: reflectors v_c (stored below the diagonal of A with beta), R on and above it
  std::vector<double> beta(P), diag(P);
  for (int c = 0; c < P; ++c) {
    double* a = &A[(size_t)c * J];
    double norm = 0.0;
    for (int j = c; j < J; ++j) norm += a[j] * a[j];
    norm = sqrt(norm);
    if (!(norm > 0.0)) return false;
    const double alpha = a[c] > 0.0 ? -norm : norm;
    a[c] -= alpha;                     // v = a - alpha e_c, stored in place
    double vv = 0.0;
    for (int j = c; j < J; ++j) vv += a[j] * a[j];
    beta[c] = vv > 0.0 ? 2.0 / vv : 0.0;
    diag[c] = alpha;
    for (int c2 = c + 1; c2 < P; ++c2) {
      double* b = &A[(size_t)c2 * J];
      double dot = 0.0;
      for (int j = c; j < J; ++j) dot += a[j] * b[j];
      dot *= beta[c];
      for (int j = c; j < J; ++j) b[j] -= dot * a[j];
    }
  }
  // column j of Pi_t = R^-1 (Q^T sqrt(w_j) e_j)_{0..P-1}
  Pi.assign((size_t)P * J, 0.0);
  std::vector<double> y(J);
  for (int j = 0; j < J; ++j) {
    std::fill(y.begin(), y.end(), 0.0);
    y[j] = sw[j];
    for (int c = 0; c < P; ++c) {
      const double* a = &A[(size_t)c * J];
      double dot = 0.0;
      for (int i = c; i < J; ++i) dot += a[i] * y[i];
      dot *= beta[c];
      for (int i = c; i < J; ++i) y[i] -= dot * a[i];
    }
    for (int c = P - 1; c >= 0; --c) {
      double v = y[c];
      for (int c2 = c + 1; c2 < P; ++c2) v -= A[(size_t)c2 * J + c] * Pi[(size_t)c2 * J + j];
      Pi[(size_t)c * J + j] = v / diag[c];
    }
  }
  for (int c = 0; c < P; ++c) {
    double sc = 1.0;
    for (int d = 0; d < dim; ++d)
      for (int e = 1; e <= k_exps[3 * c + d]; ++e) sc *= 2.0 * e;
    for (int j = 0; j < J; ++j) Pi[(size_t)c * J + j] *= sc;
  }
  return true;
}

__global__ void zero_counter_kernel(unsigned long long* c) { *c = 0ull; }

struct DevFree {
  std::vector<void*> ptrs;
  ~DevFree() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

}  // namespace

namespace fc2t2 {

// Events of the timed stages: per stage a pool of (before, after) pairs reused between reads.
struct StageTimer {
  static constexpr int kMaxCalls = 4096;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool[FC2T2_STAGE_COUNT];
  int used[FC2T2_STAGE_COUNT] = {};
  bool open[FC2T2_STAGE_COUNT] = {};
};

void stage_begin(const fc2t2_plan_s* pl, int stage, hipStream_t s) {
  StageTimer* t = pl->timer;
  if (!t || stage < 0 || stage >= FC2T2_STAGE_COUNT || t->used[stage] >= StageTimer::kMaxCalls) return;
  auto& pool = t->pool[stage];
  if ((int)pool.size() <= t->used[stage]) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return;
    }
    pool.emplace_back(a, b);
  }
  if (hipEventRecord(pool[t->used[stage]].first, s) == hipSuccess) t->open[stage] = true;
}

void stage_end(const fc2t2_plan_s* pl, int stage, hipStream_t s) {
  StageTimer* t = pl->timer;
  if (!t || stage < 0 || stage >= FC2T2_STAGE_COUNT || !t->open[stage]) return;
  t->open[stage] = false;
  if (hipEventRecord(t->pool[stage][t->used[stage]].second, s) == hipSuccess) ++t->used[stage];
}

void stage_timer_destroy(fc2t2_plan_s* pl) {
  if (!pl->timer) return;
  for (auto& pool : pl->timer->pool)
    for (auto& e : pool) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  delete pl->timer;
  pl->timer = nullptr;
}

}  // namespace fc2t2

extern "C" {

const char* fc2t2_status_string(int status) {
  switch (status) {
    case FC2T2_OK: return "ok";
    case FC2T2_EINVAL: return "invalid argument";
    case FC2T2_EUNSUPPORTED: return "unsupported combination";
    case FC2T2_EHIP: return "HIP runtime error";
    case FC2T2_ENOMEM: return "out of device memory";
    case FC2T2_EWORKSPACE: return "workspace too small";
    case FC2T2_ESCRATCH: return "call needs more scratch than the fixed array of the no-allocation entry point";
  }
  return "unknown status";
}

int fc2t2_multi_indices(int dim, int K, int* out) {
  if ((dim != 2 && dim != 3) || K < 0) return -1;
  const int P = nterms(dim, K);
  if (out) {
    std::vector<int> e((size_t)P * 3);
    mi_fill(dim, K, reinterpret_cast<int(*)[3]>(e.data()));
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < dim; ++j) out[i * dim + j] = e[3 * i + j];
  }
  return P;
}

int fc2t2_supported(int dim, int K) {
  return (dim == 2 && K >= 1 && K <= 6) || (dim == 3 && K >= 1 && K <= 5);
}

fc2t2_status fc2t2_plan_create(const fc2t2_grid* grid, const fc2t2_kernel* kernel, int K,
                               int m2l_prec, int io, int channels, hipStream_t stream,
                               fc2t2_plan* out) {
  if (!grid || !kernel || !out) return FC2T2_EINVAL;
  const int dim = grid->dim, n = grid->n;
  if (dim != 2 && dim != 3) return FC2T2_EINVAL;
  if (n < 4 || (n & (n - 1)) || n > (1 << (kMaxLevels + 1))) return FC2T2_EINVAL;
  if (!(grid->hi > grid->lo) || !isfinite(grid->lo) || !isfinite(grid->hi)) return FC2T2_EINVAL;
  if (K < 1 || channels < 1) return FC2T2_EINVAL;
  if (!fc2t2_supported(dim, K)) return FC2T2_EUNSUPPORTED;
  if (io != FC2T2_IO_F32 && io != FC2T2_IO_F64) return FC2T2_EINVAL;
  const bool fit_lsq = (m2l_prec & FC2T2_M2L_FIT_LSQ) != 0;
  m2l_prec &= ~FC2T2_M2L_FIT_LSQ;
  if (fit_lsq && m2l_prec == FC2T2_M2L_SEPARABLE) return FC2T2_EUNSUPPORTED;   // the fit is not a product
  if (m2l_prec < FC2T2_M2L_F64 || m2l_prec > FC2T2_M2L_F32_MFMA) return FC2T2_EINVAL;
  if (m2l_prec != FC2T2_M2L_SEPARABLE && (io == FC2T2_IO_F64) != (m2l_prec == FC2T2_M2L_F64))
    return FC2T2_EUNSUPPORTED;
  if (m2l_prec == FC2T2_M2L_SEPARABLE && kernel->kind != FC2T2_GAUSSIAN) return FC2T2_EUNSUPPORTED;
  if (kernel->kind == FC2T2_GAUSSIAN || kernel->kind == FC2T2_IMQ) {
    if (!(kernel->param > 0.0) || !isfinite(kernel->param)) return FC2T2_EINVAL;
  } else if (kernel->kind == FC2T2_POLY) {
    if (kernel->n_coef < 1 || !kernel->coef) return FC2T2_EINVAL;
    // n_coef must be C(deg + dim, dim) for some deg
    int deg = -1;
    for (int d = 0; d <= 64; ++d)
      if (nterms(dim, d) == kernel->n_coef) { deg = d; break; }
    if (deg < 0) return FC2T2_EINVAL;
  } else {
    return FC2T2_EINVAL;
  }
  const int64_t G = dim == 2 ? (int64_t)n * n : (int64_t)n * n * n;
  if (G > (int64_t(1) << 31)) return FC2T2_EUNSUPPORTED;

  fc2t2_plan_s* pl = new (std::nothrow) fc2t2_plan_s();
  if (!pl) return FC2T2_ENOMEM;
  pl->dim = dim;
  pl->n = n;
  pl->K = K;
  pl->P = nterms(dim, K);
  pl->Ppad = pad4(pl->P);
  pl->C = channels;
  pl->io = io;
  pl->prec = m2l_prec;
  pl->fit_lsq = fit_lsq;
  pl->kind = kernel->kind;
  pl->lo = grid->lo;
  pl->hi = grid->hi;
  pl->param = kernel->param;
  pl->h0 = (grid->hi - grid->lo) / n;
  pl->G = G;
  int levels = 0;
  while ((2 << levels) < n) ++levels;   // n = 2^(levels + 1)
  pl->levels = levels;
  for (int l = 0; l < levels; ++l) {
    pl->nl[l] = n >> l;
    pl->Gl[l] = dim == 2 ? (int64_t)pl->nl[l] * pl->nl[l] : (int64_t)pl->nl[l] * pl->nl[l] * pl->nl[l];
  }
  pl->n_off = dim == 2 ? 49 : 343;
  if (hipGetDevice(&pl->device) != hipSuccess) { delete pl; return FC2T2_EHIP; }

  auto fail = [&](fc2t2_status st) {
    if (pl->ood) (void)hipFree(pl->ood);
    if (pl->m2l_T) (void)hipFree(pl->m2l_T);
    if (pl->m2l_bf16) (void)hipFree(pl->m2l_bf16);
    if (pl->shift) (void)hipFree(pl->shift);
    if (pl->cell_bounds) (void)hipFree(pl->cell_bounds);
    sep_destroy(pl);
    delete pl;
    return st;
  };

  // ---- device counters: out-of-domain points, grazing ray roots
  if (hipMalloc((void**)&pl->ood, 3 * sizeof(unsigned long long)) != hipSuccess) {
    pl->ood = nullptr;
    return fail(FC2T2_ENOMEM);
  }
  pl->grazing = pl->ood + 1;
  pl->sort_fail = pl->ood + 2;
  if (hipMemsetAsync(pl->ood, 0, 3 * sizeof(unsigned long long), stream) != hipSuccess) return fail(FC2T2_EHIP);

  // ---- host tables
  const int P = pl->P, Ppad = pl->Ppad;
  const int n_g = nterms(dim, 2 * K);
  std::vector<int> g_exps((size_t)n_g * 3), k_exps((size_t)P * 3);
  mi_fill(dim, 2 * K, reinterpret_cast<int(*)[3]>(g_exps.data()));
  mi_fill(dim, K, reinterpret_cast<int(*)[3]>(k_exps.data()));
  std::vector<double> hl(levels);
  for (int l = 0; l < levels; ++l) hl[l] = pl->h0 * (double)(1 << l);
  int n_coef = 0, deg = 0;
  std::vector<int> c_exps(3, 0);
  if (kernel->kind == FC2T2_POLY) {
    n_coef = kernel->n_coef;
    while (nterms(dim, deg) != n_coef) ++deg;
    c_exps.assign((size_t)n_coef * 3, 0);
    mi_fill(dim, deg, reinterpret_cast<int(*)[3]>(c_exps.data()));
  }

  // ---- device scratch for the FP64 derivative pass
  DevFree tmp;
  auto dalloc = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) return nullptr;
    tmp.ptrs.push_back(p);
    return p;
  };
  const size_t nD = (size_t)levels * pl->n_off * n_g;
  double* dD = (double*)dalloc(nD * sizeof(double));
  int* dg = (int*)dalloc(g_exps.size() * sizeof(int));
  int* dk = (int*)dalloc(k_exps.size() * sizeof(int));
  double* dh = (double*)dalloc(hl.size() * sizeof(double));
  int* dce = (int*)dalloc(c_exps.size() * sizeof(int));
  double* dcoef = (double*)dalloc((size_t)(n_coef ? n_coef : 1) * sizeof(double));
  if (!dD || !dg || !dk || !dh || !dce || !dcoef) return fail(FC2T2_ENOMEM);
  if (hipMemcpyAsync(dg, g_exps.data(), g_exps.size() * sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(dk, k_exps.data(), k_exps.size() * sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(dh, hl.data(), hl.size() * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(dce, c_exps.data(), c_exps.size() * sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess)
    return fail(FC2T2_EHIP);
  if (n_coef && hipMemcpyAsync(dcoef, kernel->coef, n_coef * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess)
    return fail(FC2T2_EHIP);
  const size_t nT = (size_t)levels * pl->n_off * P * Ppad;
  const size_t tsz = io == FC2T2_IO_F64 ? 8 : 4;
  if (hipMalloc(&pl->m2l_T, nT * tsz) != hipSuccess) { pl->m2l_T = nullptr; return fail(FC2T2_ENOMEM); }
  pl->m2l_T_bytes = nT * tsz;
  if (!fit_lsq) {
    {
      const int threads = 256;
      const int64_t blocks = ceil_div((int64_t)nD, threads);
      hipLaunchKernelGGL(derivs_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, dim,
                         kernel->kind, kernel->param, dcoef, dce, n_coef, dg, n_g, levels, dh,
                         pl->n_off, dD);
      if (hipGetLastError() != hipSuccess) return fail(FC2T2_EHIP);
    }
    // ---- pack the contraction tensor (f64 for F64 plans, f32 otherwise)
    const int threads = 256;
    const int64_t blocks = ceil_div((int64_t)nT, threads);
    if (io == FC2T2_IO_F64)
      hipLaunchKernelGGL(pack_m2l_kernel<double>, dim3((unsigned)blocks), dim3(threads), 0, stream,
                         dim, K, P, Ppad, levels, pl->n_off, n_g, dh, dk, dD, (double*)pl->m2l_T);
    else
      hipLaunchKernelGGL(pack_m2l_kernel<float>, dim3((unsigned)blocks), dim3(threads), 0, stream,
                         dim, K, P, Ppad, levels, pl->n_off, n_g, dh, dk, dD, (float*)pl->m2l_T);
    if (hipGetLastError() != hipSuccess) return fail(FC2T2_EHIP);
  } else {
    // ---- least-squares fitted tensor, one level at a time
    std::vector<double> u, Pi;
    int J = 0;
    if (!lsq_projection(dim, K, k_exps, u, Pi, J)) return fail(FC2T2_EINVAL);
    double* du = (double*)dalloc(u.size() * sizeof(double));
    double* dPi = (double*)dalloc(Pi.size() * sizeof(double));
    double* dF = (double*)dalloc((size_t)pl->n_off * J * P * sizeof(double));
    if (!du || !dPi || !dF) return fail(FC2T2_ENOMEM);
    if (hipMemcpyAsync(du, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(dPi, Pi.data(), Pi.size() * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess)
      return fail(FC2T2_EHIP);
    const int threads = 256;
    const size_t per_level = (size_t)pl->n_off * P * Ppad;
    for (int l = 0; l < levels; ++l) {
      const int64_t nv = (int64_t)pl->n_off * J * P;
      hipLaunchKernelGGL(lsq_values_kernel, dim3((unsigned)ceil_div(nv, threads)), dim3(threads), 0, stream, dim,
                         kernel->kind, kernel->param, dcoef, dce, n_coef, dk, P, du, J, hl[l], pl->n_off, dF);
      const int64_t blocks = ceil_div((int64_t)per_level, threads);
      if (io == FC2T2_IO_F64)
        hipLaunchKernelGGL(lsq_project_kernel<double>, dim3((unsigned)blocks), dim3(threads), 0, stream, P, Ppad, J,
                           pl->n_off, dPi, dF, (double*)pl->m2l_T + l * per_level);
      else
        hipLaunchKernelGGL(lsq_project_kernel<float>, dim3((unsigned)blocks), dim3(threads), 0, stream, P, Ppad, J,
                           pl->n_off, dPi, dF, (float*)pl->m2l_T + l * per_level);
      if (hipGetLastError() != hipSuccess) return fail(FC2T2_EHIP);
    }
  }
  // ---- sparse M2M / L2L shift lists
  {
    const fc2t2_status st = build_shift_tables(pl, stream);
    if (st != FC2T2_OK) return fail(st);
  }
  // ---- MFMA operand tables
  if (m2l_prec == FC2T2_M2L_SEPARABLE) {
    const fc2t2_status st = sep_build(pl, stream);
    if (st != FC2T2_OK) return fail(st);
  }
  if (prec_is_mfma(m2l_prec)) {
    if (!m2l_mfma_supported(pl)) return fail(FC2T2_EUNSUPPORTED);
    const fc2t2_status st = m2l_mfma_build_tables(pl, stream);
    if (st != FC2T2_OK) return fail(st);
  }
  // ---- per-cell polynomial bounds for the ray-root layer (3-D)
  if (dim == 3 && hipMalloc(&pl->cell_bounds, (size_t)pl->G * 8) != hipSuccess) {
    pl->cell_bounds = nullptr;
    return fail(FC2T2_ENOMEM);
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return fail(FC2T2_EHIP);
  noalloc_setup(pl);   // device address of the no-allocation entry point's fixed scratch
  *out = pl;
  return FC2T2_OK;
}

fc2t2_status fc2t2_plan_destroy(fc2t2_plan plan) {
  if (!plan) return FC2T2_EINVAL;
  if (plan->m2l_T) (void)hipFree(plan->m2l_T);
  if (plan->m2l_bf16) (void)hipFree(plan->m2l_bf16);
  if (plan->shift) (void)hipFree(plan->shift);
  if (plan->cell_bounds) (void)hipFree(plan->cell_bounds);
  if (plan->ood) (void)hipFree(plan->ood);
  sep_destroy(plan);
  stage_timer_destroy(plan);
  delete plan;
  return FC2T2_OK;
}

namespace {
fc2t2_status read_counter(unsigned long long* ctr, int64_t* count, int reset, hipStream_t stream) {
  unsigned long long v = 0;
  if (hipMemcpyAsync(&v, ctr, sizeof(v), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return FC2T2_EHIP;
  *count = (int64_t)v;
  if (reset) {
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, stream, ctr);
    if (hipGetLastError() != hipSuccess) return FC2T2_EHIP;
  }
  return FC2T2_OK;
}
}  // namespace

fc2t2_status fc2t2_out_of_domain(fc2t2_plan plan, int64_t* count, int reset, hipStream_t stream) {
  if (!plan || !count) return FC2T2_EINVAL;
  return read_counter(plan->ood, count, reset, stream);
}

fc2t2_status fc2t2_grazing_roots(fc2t2_plan plan, int64_t* count, int reset, hipStream_t stream) {
  if (!plan || !count) return FC2T2_EINVAL;
  return read_counter(plan->grazing, count, reset, stream);
}

fc2t2_status fc2t2_sort_failures(fc2t2_plan plan, int64_t* count, int reset, hipStream_t stream) {
  if (!plan || !count) return FC2T2_EINVAL;
  return read_counter(plan->sort_fail, count, reset, stream);
}

int fc2t2_plan_P(fc2t2_plan plan) { return plan ? plan->P : -1; }
int fc2t2_plan_P_pad(fc2t2_plan plan) { return plan ? plan->Ppad : -1; }
int fc2t2_plan_levels(fc2t2_plan plan) { return plan ? plan->levels : -1; }
size_t fc2t2_local_numel(fc2t2_plan plan) {
  return plan ? (size_t)plan->C * (size_t)plan->G * (size_t)plan->Ppad : 0;
}

fc2t2_status fc2t2_stage_timing(fc2t2_plan plan, uint32_t stage_mask) {
  if (!plan) return FC2T2_EINVAL;
  if (!plan->timer) plan->timer = new StageTimer();
  for (int st = 0; st < FC2T2_STAGE_COUNT; ++st) {
    plan->timer->used[st] = 0;
    plan->timer->open[st] = false;
  }
  plan->timed_mask = stage_mask & ((1u << FC2T2_STAGE_COUNT) - 1u);
  return FC2T2_OK;
}

fc2t2_status fc2t2_stage_time(fc2t2_plan plan, int stage, double* ms, int64_t* calls) {
  if (!plan || !ms || !calls || stage < 0 || stage >= FC2T2_STAGE_COUNT) return FC2T2_EINVAL;
  *ms = 0.0;
  *calls = 0;
  StageTimer* t = plan->timer;
  if (!t) return FC2T2_OK;
  double total = 0.0;
  for (int i = 0; i < t->used[stage]; ++i) {
    const auto& e = t->pool[stage][i];
    float dt = 0.0f;
    if (hipEventSynchronize(e.second) != hipSuccess || hipEventElapsedTime(&dt, e.first, e.second) != hipSuccess)
      return FC2T2_EHIP;
    total += dt;
  }
  *ms = total;
  *calls = t->used[stage];
  t->used[stage] = 0;
  return FC2T2_OK;
}

}  // extern "C"

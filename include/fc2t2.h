/*
 * fc2t2.h -- C-ABI of the MI355X (gfx950) implementation of the FC^2T^2 expansion and the
 * layers built on it (Lange & Kutz, "FC^2T^2: The Fast Continuous Convolutional Taylor
 * Transform", arXiv 2111.00110).
 *
 * The library evaluates f(q) = sum_n psi(q - p_n) w_n (section 3, eq. (1)) for a smooth,
 * translation-invariant kernel psi on a uniform cell grid:
 *   P2M  -> per-cell moments   M[n] = sum w (p - c)^n / n!           (section 3, P2M)
 *   M2M  -> moments of coarser levels (binomial shift)                (section 3, M2M)
 *   M2L  -> locals from the neighbouring moments through the kernel's partial
 *           derivatives, with the parity window and near-field hole  (section 3, K^{M2L})
 *   L2L  -> coarse locals re-expanded at the finer cells              (section 3, L2L)
 *   L2P  -> f and its derivatives at query points                     (section 3, L2P)
 * plus the explicit layer's backward pass (section 4.1), the line integral and its ray
 * insertion (sections 6.1.1 and 6.2.1), and the first level crossing along a ray with its
 * implicit-function-theorem backward pass (sections 5.1-5.2).
 *
 * Conventions shared by every entry point:
 *  - Every array argument is a DEVICE pointer, row-major, owned by the caller.  The
 *    library allocates device memory only inside fc2t2_plan_create (derivative tensors
 *    and shift tables), and frees it in fc2t2_plan_destroy.  Scratch memory is passed in
 *    by the caller as `ws` of `ws_bytes` bytes, sized by fc2t2_workspace_size.
 *  - Floating-point arrays have the plan's IO type: float for FC2T2_IO_F32, double for
 *    FC2T2_IO_F64.  Integer arrays are int32.
 *  - Every call except fc2t2_plan_create is asynchronous on `stream` and does not
 *    synchronise.  Arguments are validated on the host before anything is launched; on
 *    a non-zero status nothing was launched.
 *  - Outputs of *_backward calls ACCUMULATE (+=) into their buffers; the caller zeroes
 *    them first.  Optional outputs may be NULL.
 *  - Reductions over points use a stable sort by cell and a fixed summation order, with
 *    no floating-point atomics, so results are bitwise reproducible run to run.
 *  - Points outside the domain are assigned to the nearest boundary cell (the method
 *    requires points inside the domain, section 3.2).
 *
 * Local expansions are stored in cell-scaled units: the local coefficient of multi-index k
 * in cell c is Lt[k] = h^|k| d^k f(c) with h the finest cell width, so that
 * f(q) = sum_k Lt[k] u^k / k!, u = (q - c) / h.  Layout: [C][n^dim][P_pad], cells
 * row-major with dimension 0 slowest, multi-indices in the order of fc2t2_multi_indices,
 * entries P..P_pad-1 zero.
 */
#ifndef FC2T2_H
#define FC2T2_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FC2T2_OK = 0,
  FC2T2_EINVAL = 1,        /* a NULL pointer, a negative size or an out-of-range argument */
  FC2T2_EUNSUPPORTED = 2,  /* a valid combination the library does not implement */
  FC2T2_EHIP = 3,          /* a HIP runtime call failed (launch or allocation) */
  FC2T2_ENOMEM = 4,        /* device allocation inside plan creation failed */
  FC2T2_EWORKSPACE = 5,    /* ws_bytes smaller than fc2t2_workspace_size asks */
  FC2T2_ESCRATCH = 6       /* a *_noalloc call needs more scratch than its fixed device array */
} fc2t2_status;

typedef enum {
  FC2T2_GAUSSIAN = 0,      /* psi(x) = exp(-|x|^2 / (2 param^2)), param = sigma */
  FC2T2_IMQ = 1,           /* psi(x) = (|x|^2 + param^2)^(-1/2), param = eps     */
  FC2T2_POLY = 2           /* psi(x) = sum_a coef[a] x^a (graded multi-index order) */
} fc2t2_kernel_kind;

typedef enum {
  FC2T2_M2L_F64 = 0,       /* FP64 contraction (requires FC2T2_IO_F64) */
  FC2T2_M2L_F32 = 1,       /* FP32 contraction */
  FC2T2_M2L_BF16 = 2,      /* BF16 MFMA, FP32 accumulation, one pass */
  FC2T2_M2L_BF16X2 = 3,    /* BF16 MFMA, tensor split hi/lo: two passes */
  FC2T2_M2L_BF16X3 = 4,    /* BF16 MFMA, moments and tensor split hi/lo: three passes */
  FC2T2_M2L_SEPARABLE = 5, /* Gaussian kernels only (section 3.4.1): the tensor factors over the
                              dimensions and M2L runs as one 1-D pass per dimension, the admissible
                              offsets split into disjoint per-axis products (two streams per pass),
                              in the IO precision; fc2t2_m2l then uses the plain contraction */
  FC2T2_M2L_F16X3 = 6,     /* FP16 MFMA, FP32 accumulation, moments and tensor split hi/lo (22
                              bits of mantissa per operand): three passes; each level's tensor
                              and each tile's moments scaled by powers of two into FP16's range */
  FC2T2_M2L_F32_MFMA = 7,  /* FP32 contraction on the matrix cores (v_mfma_f32_16x16x4_f32), the
                              same tiling as the 16-bit forms */
  FC2T2_M2L_FIT_LSQ = 0x100  /* flag OR'ed with a precision other than SEPARABLE (section 3.1):
                                each row k of the M2L tensor is the least-squares polynomial
                                fit, over the source cell, of the k-th derivative of the
                                kernel around the target centre instead of its Taylor
                                coefficients; L2 over the cell by tensor Gauss-Legendre
                                quadrature with K + 2 nodes per dimension.  Plan time only:
                                every later call runs the same kernels */
} fc2t2_m2l_prec;

typedef enum { FC2T2_IO_F32 = 0, FC2T2_IO_F64 = 1 } fc2t2_io;

/* Grid: the cube [lo, hi]^dim split into n^dim cells, n a power of two >= 4.  The
 * expansion has log2(n) - 1 levels; the coarsest has 4 cells per dimension
 * (section 3.2: N2 = 2^(levels+1)). */
typedef struct {
  int dim;                 /* 2 or 3 */
  int n;
  double lo, hi;
} fc2t2_grid;

/* Kernel psi.  For FC2T2_POLY, `coef` is a HOST array of n_coef values, one per
 * multi-index of total degree <= deg in the order of fc2t2_multi_indices(dim, deg), with
 * n_coef = C(deg + dim, dim); it is copied at plan creation. */
typedef struct {
  int kind;                /* fc2t2_kernel_kind */
  double param;
  int n_coef;
  const double* coef;
} fc2t2_kernel;

typedef struct fc2t2_plan_s* fc2t2_plan;

/* Operations, for fc2t2_workspace_size. */
typedef enum {
  FC2T2_OP_EXPAND = 0,               /* count = N sources */
  FC2T2_OP_EVAL_BACKWARD = 1,        /* count = M queries */
  FC2T2_OP_EXPAND_BACKWARD = 2,      /* count = N sources */
  FC2T2_OP_RAY_INTEGRAL_BACKWARD = 3,/* count = R rays */
  FC2T2_OP_RAY_ROOT_BACKWARD = 4,    /* count = R rays */
  FC2T2_OP_EVAL_SORTED = 5,          /* count = M queries (fc2t2_eval_sorted's records) */
  FC2T2_OP_RAY_VOLUME_BACKWARD = 6,  /* count = R rays */
  FC2T2_OP_BIN_POINTS = 7            /* count = N points */
} fc2t2_op;

/* Status text (static storage). */
const char* fc2t2_status_string(int status);

/* Multi-indices n with |n| <= K in the library's order (total degree ascending, then
 * the first component descending, then the second): writes P*dim ints to the HOST array
 * `out` (may be NULL to query P) and returns P = C(K + dim, dim), or -1 if dim is not 2 or
 * 3 or K < 0. */
int fc2t2_multi_indices(int dim, int K, int* out);

/* Supported orders: dim 2 -> 1 <= K <= 6, dim 3 -> 1 <= K <= 5. */
int fc2t2_supported(int dim, int K);

/* Build a plan: validates the arguments, generates every level's M2L tensor
 * T[k, n](o) = h^(|k|+|n|) (-1)^|n| d^(k+n) psi(-o h) for o in [-3, 3]^dim in FP64 on the
 * GPU (section 3, K^{M2L}; derivatives in closed form for the radial kernels), or its
 * least-squares fit when m2l_prec carries FC2T2_M2L_FIT_LSQ, rounds it to the contraction
 * precision, and uploads the M2M/L2L shift tables.  m2l_prec is a fc2t2_m2l_prec value,
 * optionally OR'ed with FC2T2_M2L_FIT_LSQ.  `channels` is the number C of weight columns.
 * Synchronises `stream`.  *out is set only on success. */
fc2t2_status fc2t2_plan_create(const fc2t2_grid* grid, const fc2t2_kernel* kernel, int K,
                               int m2l_prec, int io, int channels, hipStream_t stream,
                               fc2t2_plan* out);
fc2t2_status fc2t2_plan_destroy(fc2t2_plan plan);

/* Plan properties. */
int fc2t2_plan_P(fc2t2_plan plan);            /* multi-indices per cell */
int fc2t2_plan_P_pad(fc2t2_plan plan);        /* row stride of a local-expansion cell */
int fc2t2_plan_levels(fc2t2_plan plan);

/* Points outside [lo, hi]^dim (NaN included) that fc2t2_expand (sources) and fc2t2_eval
 * (queries) have met on this plan since its creation or the last reset, counted on the
 * device; each such point was binned into the nearest boundary cell (the method assumes
 * points inside the domain, section 3.2).  Copies the count to *count, synchronising
 * `stream`; reset != 0 then zeroes the counter (ordered on `stream`).  EINVAL for NULLs. */
fc2t2_status fc2t2_out_of_domain(fc2t2_plan plan, int64_t* count, int reset, hipStream_t stream);
size_t fc2t2_local_numel(fc2t2_plan plan);    /* C * n^dim * P_pad elements */

/* Sorts by cell (of sources, queries, ray records) whose decoupled look-back gave up waiting on
 * this plan since its creation or the last reset, counted on the device; same calling rules as
 * fc2t2_out_of_domain.  A failed sort leaves every cell empty for the stages after it (their
 * per-cell outputs are zero, per-point outputs in sorted order are not written), so a non-zero
 * count means the outputs of the calls since the last read are not valid. */
fc2t2_status fc2t2_sort_failures(fc2t2_plan plan, int64_t* count, int reset, hipStream_t stream);

/* Test aid for the failure path above, process-wide: enable != 0 makes tile 1 of every one-sweep
 * pass withhold its published counts and shortens the look-back's bounded wait to a few polls, so
 * the tiles after it give up (every kernel still ends normally); enable = 0 restores normal
 * sorting.  Calls made while it is enabled do not produce valid results. */
void fc2t2_debug_sort_fault(int enable);

/* Ray roots that fc2t2_ray_root classified as grazing (FC2T2_ROOT_GRAZING) on this plan since
 * its creation or the last reset, counted on the device; same calling rules as
 * fc2t2_out_of_domain. */
fc2t2_status fc2t2_grazing_roots(fc2t2_plan plan, int64_t* count, int reset, hipStream_t stream);

/* Scratch bytes `op` needs for `count` points or rays (0 for an invalid op). */
size_t fc2t2_workspace_size(fc2t2_plan plan, int op, int64_t count);

/* Expansion (section 3): L = locals of f(.) = sum_n psi(. - p_n) w_n at the finest level.
 *   p [N][dim], w [N][C] in; L [C][n^dim][P_pad] out (overwritten).  N may be 0. */
fc2t2_status fc2t2_expand(fc2t2_plan plan, const void* p, const void* w, int64_t N, void* L,
                          void* ws, size_t ws_bytes, hipStream_t stream);

/* L2P (section 3) with the derivatives of section 3.2's accessor:
 *   q [M][dim] in; y [M][C] out; grad [M][C][dim] out or NULL; hess [M][C][dim(dim+1)/2]
 *   out or NULL, upper triangle row by row (xx, xy, (xz,) yy, (yz, zz)). */
fc2t2_status fc2t2_eval(fc2t2_plan plan, const void* L, const void* q, int64_t M, void* y,
                        void* grad, void* hess, hipStream_t stream);

/* L2P (section 3) with the queries taken in cell order: bins and sorts q [M][dim] by cell into
 * the workspace (the sorted coordinates, input indices and cell starts stay there), then
 * evaluates y [M] (input order) from the sorted records, each cell's row read once from
 * memory.  The records serve fc2t2_eval_backward_sorted for the same plan, q and M (a training
 * step sorts its queries once).  FP32 IO and one channel only (EUNSUPPORTED otherwise);
 * ws_bytes >= fc2t2_workspace_size(plan, FC2T2_OP_EVAL_SORTED, M); out-of-domain queries are
 * counted as by fc2t2_eval. */
fc2t2_status fc2t2_eval_sorted(fc2t2_plan plan, const void* L, const void* q, int64_t M, void* y,
                               void* ws, size_t ws_bytes, hipStream_t stream);

/* The two halves of fc2t2_eval_sorted (section 3.3 binning, then L2P of section 3), so that a
 * caller can sort a step's queries on one stream while another builds the expansion:
 * fc2t2_sort_queries bins and sorts q [M][dim] by cell into `ws` (the records described above;
 * q is not read again), and fc2t2_eval_presorted evaluates y [M] (input order) from those
 * records and L.  The second call must be ordered after the first (same stream, or an event);
 * same plan, M and ws, ws not written in between.  Same support, workspace size and
 * out-of-domain counting as fc2t2_eval_sorted; the records then serve
 * fc2t2_eval_backward_sorted as well. */
fc2t2_status fc2t2_sort_queries(fc2t2_plan plan, const void* q, int64_t M, void* ws, size_t ws_bytes,
                                hipStream_t stream);
fc2t2_status fc2t2_eval_presorted(fc2t2_plan plan, const void* L, int64_t M, void* y, const void* ws,
                                  size_t ws_bytes, hipStream_t stream);

/* fc2t2_eval_backward from the records an fc2t2_eval_sorted call left in `ws` (same plan, same
 * queries and M, ws not written in between; q is not read again): one pass over the sorted
 * queries gives gL (the transpose of L2P, per-cell sums) and gq [M][dim] = gy . grad f(q) (NULL
 * to skip; L is then not read), both written at the queries' input positions.  accumulate != 0
 * adds into gL and gq, 0 overwrites them. */
fc2t2_status fc2t2_eval_backward_sorted(fc2t2_plan plan, const void* L, int64_t M, const void* gy,
                                        void* gL, void* gq, const void* ws, size_t ws_bytes,
                                        int accumulate, hipStream_t stream);

/* Backward of fc2t2_eval's value output (section 4.1): with gy [M][C],
 *   gL [C][n^dim][P_pad] += d(sum gy*y)/dL  (the transpose of L2P),
 *   gq [M][dim] += gy . grad f(q)  (NULL to skip). */
fc2t2_status fc2t2_eval_backward(fc2t2_plan plan, const void* L, const void* q, int64_t M,
                                 const void* gy, void* gL, void* gq, void* ws,
                                 size_t ws_bytes, hipStream_t stream);

/* Backward of fc2t2_expand (section 4.1: the second expansion, with the roles of sources
 * and targets swapped, computed as the exact transpose L2L^T -> M2L^T -> M2M^T -> P2M^T):
 * with gL the cotangent of L,
 *   gp [N][dim] += d/dp, gw [N][C] += d/dw  (either may be NULL). */
fc2t2_status fc2t2_expand_backward(fc2t2_plan plan, const void* gL, const void* p,
                                   const void* w, int64_t N, void* gp, void* gw, void* ws,
                                   size_t ws_bytes, hipStream_t stream);

/* fc2t2_eval_backward and fc2t2_expand_backward with a choice: accumulate != 0 adds into
 * gL, gq (respectively gp, gw) as the calls above do; accumulate == 0 overwrites them with
 * the gradient (gL is zeroed when M == 0), so a caller with fresh gradient buffers needs no
 * fill first.  Same kernels, same arguments, same workspace. */
fc2t2_status fc2t2_eval_backward_ex(fc2t2_plan plan, const void* L, const void* q, int64_t M,
                                    const void* gy, void* gL, void* gq, void* ws,
                                    size_t ws_bytes, int accumulate, hipStream_t stream);
fc2t2_status fc2t2_expand_backward_ex(fc2t2_plan plan, const void* gL, const void* p,
                                      const void* w, int64_t N, void* gp, void* gw, void* ws,
                                      size_t ws_bytes, int accumulate, hipStream_t stream);

/* Line integral (section 6.1.1): y[r][c] = integral over t in [t0, t1] of f(o_r + t r_r),
 * f taken as zero outside the domain, computed exactly cell by cell from L (dim 3 only).
 *   o [R][3], r [R][3] (need not be unit) in; y [R][C] out. */
fc2t2_status fc2t2_ray_integral(fc2t2_plan plan, const void* L, const void* o, const void* r,
                                double t0, double t1, int64_t R, void* y,
                                hipStream_t stream);

/* Backward of fc2t2_ray_integral (section 6.2.1, ray insertion): gL += the segment
 * integrals of each cell's monomials weighted by gy [R][C]. */
fc2t2_status fc2t2_ray_integral_backward(fc2t2_plan plan, const void* o, const void* r,
                                         double t0, double t1, int64_t R, const void* gy,
                                         void* gL, void* ws, size_t ws_bytes,
                                         hipStream_t stream);

/* Ray root (section 5.1, C == 1, dim 3): tau_r = level_frac * max of f along the clipped
 * ray, then the first t where f - tau_r goes from negative to non-negative (a root on a
 * cell face belongs to the earlier cell).  Outputs: t [R] (NaN if none), normal [R][3] =
 * grad f at the root (zero if none), hit [R] int32 (1 hit, 0 dead ray: no crossing, or
 * f >= tau at entry), saved [R][FC2T2_ROOT_SAVED] (state for the backward, IO type: root
 * point [0..2], the root's finest cell index as the bits of an unsigned integer of the
 * slot's width [3], r . grad f [4], H r [5..7], tau [8], t [9], the kind of the hit [10]:
 * FC2T2_ROOT_SMOOTH, FC2T2_ROOT_FACE (the level is crossed by the jump of the piecewise
 * expansion across a cell face) or FC2T2_ROOT_GRAZING (|r . grad f| <= FC2T2_GRAZE_COS
 * |r| |grad f|: the ray is tangent to the level set to within that cosine; counted on the
 * device, read with fc2t2_grazing_roots)).  The root is polished by one FP64 Newton step.
 * The call first writes per-cell bounds of L into a buffer the plan owns, so ray-root calls
 * on one plan must not overlap in time (issue them on one stream).  EUNSUPPORTED for grids
 * of more than 2^32 cells. */
#define FC2T2_ROOT_SAVED 12
#define FC2T2_ROOT_SMOOTH 0
#define FC2T2_ROOT_FACE 1
#define FC2T2_ROOT_GRAZING 2
#define FC2T2_GRAZE_COS 1e-4
fc2t2_status fc2t2_ray_root(fc2t2_plan plan, const void* L, const void* o, const void* r,
                            double t0, double t1, int64_t R, double level_frac, void* t,
                            void* normal, int32_t* hit, void* saved, hipStream_t stream);

/* fc2t2_ray_root with given levels: the first t where f - tau[r] goes from negative to
 * non-negative, for a per-ray level tau [R] (IO type) instead of level_frac * max f, e.g. the
 * zero level of an implicit surface with a constant bias (section 5.1).  Same outputs, kinds
 * and backward (saved[8] holds the given level); the maximum along the ray is not computed. */
fc2t2_status fc2t2_ray_root_at(fc2t2_plan plan, const void* L, const void* o, const void* r,
                               double t0, double t1, int64_t R, const void* tau, void* t,
                               void* normal, int32_t* hit, void* saved, hipStream_t stream);

/* Test aid: root finding of fc2t2_ray_root / fc2t2_ray_root_at solves every polynomial of degree
 * <= 4 by closed forms by default (section 5.1: Ferrari's method for the quartic, Cardano's for
 * the cubic, the quadratic formula, each root polished by Newton steps): for K <= 4 the segment
 * polynomial's roots and critical points, for K = 5 its critical points (the root on each monotone
 * piece then comes from the safeguarded iteration).  enable != 0 switches every later call in the
 * process to the derivative cascade throughout (critical points by recursion on the derivatives,
 * safeguarded Newton on monotone pieces), enable == 0 back.  Both give the same roots to
 * rounding; the switch lets a test compare them on the same rays. */
void fc2t2_debug_root_cascade(int enable);

/* Backward of fc2t2_ray_root (section 5.2, implicit function theorem), tau held fixed:
 * gL += a (q* - c)^k / k! + sum_j gn_j d/dq_j (q* - c)^k / k!, with
 * a = -(gt + gn . H r) / (r . grad f), for every ray with hit = 1.  The theorem needs
 * r . grad f != 0: a FC2T2_ROOT_FACE hit has a root that does not move with L (it stays on the face) and a
 * FC2T2_ROOT_GRAZING hit one of unbounded sensitivity, so both insert the dipole term only (a = 0).
 * gt [R] and gn [R][3] may each be NULL (zero). */
fc2t2_status fc2t2_ray_root_backward(fc2t2_plan plan, const void* saved, const int32_t* hit,
                                     int64_t R, const void* gt, const void* gn, void* gL,
                                     void* ws, size_t ws_bytes, hipStream_t stream);

/* Binning (section 3.3: a point's finest box is the integer part of its scaled coordinates,
 * clamped to the grid), as the expansion and the sorted evaluation do it: points x [N][dim]
 * (IO type) sorted stably by the row-major index of their finest cell.  Outputs (caller-owned,
 * uint32): keys_sorted [N] the cell indices in sorted order, perm [N] the input index of each
 * sorted position (equal cells keep input order), starts [G + 1] the first sorted position of
 * each cell (starts[G] = N), G = n^dim.  With pay_out (FP32 IO, one channel): the coordinates
 * travel with the sort, pay_out [N][dim] in sorted order, or [N][dim + 1] with extra [N] (one
 * value per point, e.g. a weight) appended.  Points outside the domain are counted
 * (fc2t2_out_of_domain).  A failed look-back in the sort empties every cell and is counted
 * (fc2t2_sort_failures).  Workspace FC2T2_OP_BIN_POINTS. */
fc2t2_status fc2t2_bin_points(fc2t2_plan plan, const void* x, int64_t N, const void* extra,
                              uint32_t* keys_sorted, uint32_t* perm, uint32_t* starts,
                              void* pay_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* Volumetric rendering (section 6.1.2; dim 3, C == 4: channel 0 the density sigma, channels
 * 1..3 the colour c = (R, G, B); K <= 5).  Per ray, with S the optical depth from the entry
 * point of the clipped ray and mexp the degree-4 polynomial closest to exp(-x) in L2 on
 * [0, 5] standing in for the transmittance exp(-S):
 *   y[r][k] = int T sigma c_k dt + bg[k] T_end,    T = mexp(S),
 * computed exactly cell by cell (every factor is a polynomial of t inside a cell).  The walk
 * ends after the first cell whose exit depth exceeds FC2T2_VOLUME_STOP_DEPTH (the fit is used
 * below 5 only); T_end = 0 then, else mexp(total depth).  o, r [R][3] (r need not be unit);
 * bg: host array of 3 doubles, the background colour (section 6.2.2), or NULL for black.
 * Outputs y [R][3] and, when trans is not NULL, trans [R] = T_end (IO type).  The density is
 * used as the expansion gives it (a caller keeps it non-negative, e.g. through non-negative
 * density weights). */
#define FC2T2_VOLUME_STOP_DEPTH 4.5
fc2t2_status fc2t2_ray_volume(fc2t2_plan plan, const void* L, const void* o, const void* r,
                              double t0, double t1, int64_t R, const double* bg, void* y,
                              void* trans, hipStream_t stream);

/* Backward of fc2t2_ray_volume (section 6.2.2) as the exact derivative of its forward, the
 * stop decision held fixed: with gy [R][3] the colour cotangents, gL += for colour channel k
 * the integrals of gy_k sigma T mono, and for the density channel the integrals of H mono with
 *   H(t) = c_y T + int_t^end c_y sigma mexp'(S) + [walk did not stop] (gy . bg) mexp'(S_end),
 * c_y = sum_k gy_k c_k (a change of density at t changes the depth at every later point);
 * mono = (q - centre)^k / k! in cell units.  L is the forward's expansion (the derivative
 * depends on it); workspace FC2T2_OP_RAY_VOLUME_BACKWARD.  EUNSUPPORTED when
 * R (3 n + 4) > 2^32. */
fc2t2_status fc2t2_ray_volume_backward(fc2t2_plan plan, const void* L, const void* o,
                                       const void* r, double t0, double t1, int64_t R,
                                       const double* bg, const void* gy, void* gL, void* ws,
                                       size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): fc2t2_ray_root_backward with its scratch in a
 * fixed device array of FC2T2_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU
 * it runs on until the process ends, instead of a caller workspace.  Same arguments
 * otherwise, same kernels and same results; it allocates nothing and frees nothing.
 * FC2T2_ESCRATCH when the call needs more scratch than the array holds, i.e. when
 * fc2t2_workspace_size(plan, FC2T2_OP_RAY_ROOT_BACKWARD, R) > FC2T2_NOALLOC_SCRATCH_BYTES
 * (131072 rays on a 128^3 grid fit); FC2T2_EHIP if the array's address could not be resolved
 * when the plan was created.  All calls on one GPU share its array and every call rewrites
 * what it reads, so calls that overlap in time on one GPU (other streams, other threads)
 * race; issue them on one stream. */
#define FC2T2_NOALLOC_SCRATCH_BYTES (16u << 20)
fc2t2_status fc2t2_ray_root_backward_noalloc(fc2t2_plan plan, const void* saved, const int32_t* hit,
                                             int64_t R, const void* gt, const void* gn, void* gL,
                                             hipStream_t stream);

/* Stage entry point: one M2L launch at one level (section 3, K^{M2L}) between caller-owned
 * grids of that level, [C][n_level^dim][P_pad] in that level's cell-scaled units
 * (moments M[n] / h_level^|n|, locals h_level^|k| d^k f).  transpose = 0 computes
 * out (+)= M2L(in); transpose = 1 computes the transpose out (+)= M2L^T(in).  accumulate
 * selects += over overwrite.  For per-stage timing and custom level pipelines. */
fc2t2_status fc2t2_m2l(fc2t2_plan plan, int level, int transpose, const void* in, void* out,
                       int accumulate, hipStream_t stream);

/* Elements of one level's grid: C * n_level^dim * P_pad (0 for an invalid level). */
size_t fc2t2_level_numel(fc2t2_plan plan, int level);

/* ---- Stage timing (a measurement aid, not part of the method) ----
 * Stages of the pipeline, each one kernel launch per call unless noted. */
typedef enum {
  FC2T2_STAGE_SORT = 0,   /* binning: cell keys, radix passes, cell starts (several launches) */
  FC2T2_STAGE_P2M,        /* per-cell moment reduction over the sorted sources */
  FC2T2_STAGE_SHIFT_UP,   /* M2M up the pyramid, or L2L^T (a few multi-level launches) */
  FC2T2_STAGE_M2L,        /* M2L at every level (one launch on the MFMA path) */
  FC2T2_STAGE_SHIFT_DOWN, /* L2L down the pyramid, or M2M^T (a few multi-level launches) */
  FC2T2_STAGE_L2P,        /* evaluation at the queries */
  FC2T2_STAGE_L2P_T,      /* per-cell reduction of query cotangents (with q_bar when fused) */
  FC2T2_STAGE_M2L_T,      /* transposed M2L at every level */
  FC2T2_STAGE_P2M_T,      /* per-source gradients w_bar, p_bar */
  FC2T2_STAGE_RAY,        /* ray integral or ray root kernel (forward) */
  FC2T2_STAGE_RAY_T,      /* ray cotangent records and their per-cell reduction (backward) */
  FC2T2_STAGE_QGRAD,      /* q_bar = gy . grad f(q) as its own pass over the queries */
  FC2T2_STAGE_COUNT
} fc2t2_stage;

/* Selects the stages to time: bit s of stage_mask times stage s.  From then on the library
 * records a HIP event on the launch stream before and after every timed stage's launches.
 * Clears what was recorded.  FC2T2_EINVAL for a null plan. */
fc2t2_status fc2t2_stage_timing(fc2t2_plan plan, uint32_t stage_mask);

/* Waits for the events recorded for `stage` since the last call for it (or since
 * fc2t2_stage_timing), writes their summed duration in milliseconds to *ms and the number of
 * timed calls to *calls, and clears them.  At most 4096 calls per stage are kept between reads;
 * later ones are not timed.  FC2T2_EINVAL for a bad stage or null outputs, FC2T2_EHIP if an
 * event query fails.  One thread per plan. */
fc2t2_status fc2t2_stage_time(fc2t2_plan plan, int stage, double* ms, int64_t* calls);

#ifdef __cplusplus
}
#endif

#endif /* FC2T2_H */

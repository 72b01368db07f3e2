// Internal plan state and the launchers each translation unit provides.
#pragma once

#include <vector>

#include "common.h"

namespace fc2t2 {
struct StageTimer;
}
struct SepTables;

struct fc2t2_plan_s {
  int dim, n, K, P, Ppad, C, levels, io, prec, kind;
  bool fit_lsq = false;            // M2L tensors fitted by least squares (section 3.1)
  unsigned long long* ood = nullptr;   // device counter: points outside the domain (expand, eval)
  unsigned long long* grazing = nullptr;   // device counter: grazing ray roots (ray root); the
                                           //   second word of the ood allocation
  unsigned long long* sort_fail = nullptr; // device counter: sorts whose look-back gave up; third word
  double lo, hi, param;
  double h0;                      // finest cell width
  int64_t G;                      // finest cells
  int nl[fc2t2::kMaxLevels];      // cells per dimension at each level
  int64_t Gl[fc2t2::kMaxLevels];  // cells at each level
  int n_off;                      // 7^dim source offsets o in [-3, 3]^dim
  // Device tables (owned by the plan).
  void* m2l_T = nullptr;          // [levels][n_off][P][Ppad], contraction type (f32/f64):
                                  //   T[lvl][o][n][k] = h^(|k|+|n|) (-1)^|n| d^(k+n) psi(-o h)
  size_t m2l_T_bytes = 0;
  void* m2l_bf16 = nullptr;       // MFMA operand tables (layout owned by m2l_mfma.hip)
  size_t m2l_bf16_bytes = 0;
  float t_scale[2][fc2t2::kMaxLevels] = {};   // FP16 operands: power of two applied to each
                                               //   [direction][level] tensor
  void* shift = nullptr;          // sparse M2M/L2L shift lists (layout owned by tree.hip)
  size_t shift_beg_off = 0;
  int shift_n_up = 0, shift_n_down = 0;
  SepTables* sep = nullptr;       // separable M2L tables (layout owned by separable.hip)
  void* cell_bounds = nullptr;    // 3-D: [G] float2 (lower, upper) bound of each finest cell's
                                  //   polynomial over the cell, rebuilt by every ray-root call
  int device = 0;
  void* noalloc_scratch = nullptr;   // this device's fixed scratch array (rays.hip), or null
  // Stage timing (measurement aid): bit s of timed_mask brackets stage s with events.
  uint32_t timed_mask = 0;
  fc2t2::StageTimer* timer = nullptr;
  // Occupancy stamp of the current call (1..255): a cell is occupied iff its byte equals it.
  // Every map is written in full each call; a stale byte that matched would only disable a
  // skip, never cause a wrong one.
  mutable uint8_t occ_gen = 0;
};

namespace fc2t2 {

inline size_t io_size(const fc2t2_plan_s* pl) { return pl->io == FC2T2_IO_F64 ? 8 : 4; }
inline size_t grid_elems(const fc2t2_plan_s* pl, int lvl) {
  return (size_t)pl->C * (size_t)pl->Gl[lvl] * (size_t)pl->Ppad;
}
// Elements of a level pyramid holding levels [first, levels).
inline size_t pyramid_elems(const fc2t2_plan_s* pl, int first) {
  size_t s = 0;
  for (int l = first; l < pl->levels; ++l) s += grid_elems(pl, l);
  return s;
}

// ---- plan.hip
// Gauss-Legendre nodes t and weights w of the Q-point rule on [-1, 1].
void gauss_legendre(int Q, std::vector<double>& t, std::vector<double>& w);
// stage timing
void stage_begin(const fc2t2_plan_s* pl, int stage, hipStream_t s);
void stage_end(const fc2t2_plan_s* pl, int stage, hipStream_t s);
void stage_timer_destroy(fc2t2_plan_s* pl);
// Brackets a stage's launches with events when the plan times that stage.
struct StageScope {
  const fc2t2_plan_s* pl;
  int stage;
  hipStream_t s;
  bool on;
  StageScope(const fc2t2_plan_s* p, int st, hipStream_t str)
      : pl(p), stage(st), s(str), on(((p->timed_mask >> st) & 1u) != 0) {
    if (on) stage_begin(pl, stage, s);
  }
  ~StageScope() {
    if (on) stage_end(pl, stage, s);
  }
  StageScope(const StageScope&) = delete;
  StageScope& operator=(const StageScope&) = delete;
};

// ---- sort.hip
// Stable LSD radix sort of (key, index) pairs by the low `key_bits` bits.  keys_in is
// read only; keys_out/vals_out receive the sorted keys and the original indices.  `frequent`
// names a key expected many times (the records' unused-slot key), counted without contention.
size_t radix_sort_scratch_bytes(int64_t N);
fc2t2_status radix_sort_pairs(const uint32_t* keys_in, uint32_t* keys_out, uint32_t* vals_out,
                              int64_t N, int key_bits, void* scratch, hipStream_t s,
                              uint32_t frequent = 0xFFFFFFFFu);
// starts[c] = first sorted position with key >= c, for c in [0, G]; starts[G] = N.
// The same for points: keys (written to `keys`) are the linear finest-cell indices of x.
// With pay_out, each point's coordinates and its extra_words (1..4) values in `extra`
// ([N][extra_words]) travel with it: pay_out [N][dim + extra_words] receives them in sorted order
// (FP32: sort_payload_ok); with pay_out and no `extra`, the coordinates alone: pay_out [N][dim].
// With ood, the points outside the domain are added to *ood.
fc2t2_status sort_points_by_cell(const fc2t2_plan_s* pl, const void* x, int64_t N, uint32_t* keys,
                                 uint32_t* keys_out, uint32_t* vals_out, void* scratch, hipStream_t s,
                                 const void* extra = nullptr, void* pay_out = nullptr,
                                 unsigned long long* ood = nullptr, int extra_words = 1);
// FP32 points whose sorts can carry their coordinates and up to four values each.
bool sort_payload_ok(const fc2t2_plan_s* pl);
// err: the sort's failure word (sort_err_word); when set, every cell comes out empty and
// *fail_ctr is incremented.
fc2t2_status launch_cell_starts(const uint32_t* keys_sorted, int64_t N, int64_t G,
                                uint32_t* starts, hipStream_t s, const uint32_t* err,
                                unsigned long long* fail_ctr);
// The failure word of the sort whose scratch (for N records) is `scratch`: non-zero after a
// pass whose look-back gave up; the sorted arrays are then not valid.
const uint32_t* sort_err_word(const void* scratch, int64_t N);
int key_bits_for(int64_t G);

// ---- p2m_l2p.hip
// P2M: M0 = moments of the sorted sources (overwrite).
fc2t2_status launch_p2m(const fc2t2_plan_s* pl, const void* p, const void* w, int64_t N,
                        const uint32_t* starts, const uint32_t* perm, void* M0, hipStream_t s,
                        uint8_t* occ = nullptr, uint8_t gen = 1);
// Transpose of L2P: gL += (or =) sum over the sorted queries of gy (q - c)^k / k!.
fc2t2_status launch_l2p_T(const fc2t2_plan_s* pl, const void* q, const void* gy, int64_t M,
                          const uint32_t* starts, const uint32_t* perm, void* gL, hipStream_t s,
                          bool accumulate = true);
// P2M, or the transpose of L2P, from records sorted with their data (pay [count][dim + C]:
// coordinates and the C weights or cotangents; FP32, C <= 4).
fc2t2_status launch_reduce_sorted(const fc2t2_plan_s* pl, const void* pay, int64_t count, const uint32_t* starts,
                                  void* out, bool accumulate, hipStream_t s, uint8_t* occ = nullptr,
                                  uint8_t gen = 1);
// Finest-level occupancy from points: occ cleared, then occ[cell] = gen at every cell holding
// a point.
fc2t2_status launch_mark_cells(const fc2t2_plan_s* pl, const void* x, int64_t N, uint8_t* occ, uint8_t gen,
                               hipStream_t s);
// Transpose of L2P fused with gq += gy grad f(q) (one channel only); accumulate applies to gL,
// gq is always accumulated into.
fc2t2_status launch_l2p_T_qgrad(const fc2t2_plan_s* pl, const void* L, const void* q, const void* gy, int64_t M,
                                const uint32_t* starts, const uint32_t* perm, void* gL, void* gq, hipStream_t s,
                                bool accumulate = true);
// L2P: y (overwrite), grad/hess (overwrite, optional).
fc2t2_status launch_l2p(const fc2t2_plan_s* pl, const void* L, const void* q, int64_t M, void* y,
                        void* grad, void* hess, hipStream_t s);
// gq += (or =) sum_c gy[c] grad_c f(q).
fc2t2_status launch_l2p_qgrad(const fc2t2_plan_s* pl, const void* L, const void* q, int64_t M,
                              const void* gy, void* gq, hipStream_t s, bool accumulate = true);
// Transpose of P2M: gw += <GM0, mono>, gp += w <GM0, grad mono> / h (or = for both).
fc2t2_status launch_p2m_T(const fc2t2_plan_s* pl, const void* GM0, const void* p, const void* w,
                          int64_t N, void* gp, void* gw, hipStream_t s, bool accumulate = true);
// q_bar from queries sorted with their data (FP32, one channel): pay [M][dim + 1], keys the
// sorted cells, perm the input indices; gq[perm[r]] += (or =) gy grad f(q) / h.
fc2t2_status launch_qgrad_sorted(const fc2t2_plan_s* pl, const void* L, const void* pay, const uint32_t* keys,
                                 const uint32_t* perm, int64_t M, void* gq, hipStream_t s, bool accumulate,
                                 const uint32_t* err);
// L2P over queries sorted with their coordinates (FP32, one channel): pay [M][dim], keys the
// sorted cells, perm the input indices; y[perm[r]] = f(q_r).
fc2t2_status launch_l2p_sorted(const fc2t2_plan_s* pl, const void* L, const void* pay, const uint32_t* keys,
                               const uint32_t* perm, int64_t M, void* y, hipStream_t s, const uint32_t* err);
// Transpose of L2P fused with q_bar over the same sorted queries: gL (+)= per-cell sums of
// gy[perm[r]] (q_r - c)^k / k!, and gq[perm[r]] (+)= gy grad f(q_r) (one pass, one channel).
fc2t2_status launch_l2p_T_qgrad_sorted(const fc2t2_plan_s* pl, const void* L, const void* pay, const uint32_t* starts,
                                       const uint32_t* perm, const void* gy, int64_t M, void* gL, void* gq,
                                       hipStream_t s, bool accumulate);
// p[0 .. elems) = 0 in the plan's IO type (a fill kernel, safe under graph capture).
fc2t2_status launch_zero(const fc2t2_plan_s* pl, void* p, int64_t elems, hipStream_t s);

// ---- tree.hip
// Sparse shift lists of the plan's (dim, K), uploaded to pl->shift.
fc2t2_status build_shift_tables(fc2t2_plan_s* pl, hipStream_t s);
// Whole pyramid passes: grids[l+1] = up-shift(grids[l]) for every level (M2M, and the
// transpose of L2L), and grids[l] += down-shift(grids[l+1]) from the coarsest to the finest
// (L2L, and the transpose of M2M); several levels per launch.
// With occ (per-level byte maps, occ[0] filled), the up pass also sets occ[l+1][I] = gen when
// any child's occ[l] == gen, else 0.
fc2t2_status upshift_pyramid(const fc2t2_plan_s* pl, void* const* grids, hipStream_t s,
                             uint8_t* const* occ = nullptr, uint8_t gen = 1);
fc2t2_status downshift_pyramid(const fc2t2_plan_s* pl, void* const* grids, hipStream_t s);
// M2L at one level: L (+)= sum_o T(o) M[i + o] over the admissible offsets.
fc2t2_status launch_m2l(const fc2t2_plan_s* pl, int lvl, const void* M, void* L, bool accumulate,
                        hipStream_t s);
// Transpose: GM (+)= sum_o T(o)^T GL[j - o].
fc2t2_status launch_m2l_T(const fc2t2_plan_s* pl, int lvl, const void* GL, void* GM,
                          bool accumulate, hipStream_t s);
// M2L (or its transpose) at every level, outputs overwritten; ins/outs indexed by level.
// Optional occupancy maps (occ[l] per level, == gen: the cell or its subtree holds a source):
// the forward skips (writes zeros for) target tiles whose whole source window is empty; the
// transpose does so for tiles none of whose outputs is occupied.  Results at every cell the
// method reads are unchanged.
fc2t2_status launch_m2l_all(const fc2t2_plan_s* pl, const void* const* ins, void* const* outs,
                            bool transpose, hipStream_t s, const uint8_t* const* occ = nullptr,
                            uint8_t gen = 1, void* sep_ws = nullptr);

// ---- separable.hip (Gaussian kernels)
bool sep_supported(const fc2t2_plan_s* pl);
fc2t2_status sep_build(fc2t2_plan_s* pl, hipStream_t s);
void sep_destroy(fc2t2_plan_s* pl);
size_t sep_ws_bytes(const fc2t2_plan_s* pl);
// M2L (or its transpose) at every level by one-dimensional passes; ws of sep_ws_bytes bytes.
fc2t2_status launch_m2l_separable(const fc2t2_plan_s* pl, const void* const* ins, void* const* outs, bool transpose,
                                  void* ws, hipStream_t s);
inline bool prec_is_mfma(int prec) {
  return (prec >= FC2T2_M2L_BF16 && prec <= FC2T2_M2L_BF16X3) || prec == FC2T2_M2L_F16X3 ||
         prec == FC2T2_M2L_F32_MFMA;
}
inline bool m2l_is_mfma(const fc2t2_plan_s* pl) { return prec_is_mfma(pl->prec); }

// ---- m2l_mfma.hip
bool m2l_mfma_supported(const fc2t2_plan_s* pl);
size_t m2l_mfma_table_bytes(const fc2t2_plan_s* pl);
size_t m2l_mfma_table_bytes_only(const fc2t2_plan_s* pl);   // operand tables without the scales
fc2t2_status m2l_mfma_build_tables(fc2t2_plan_s* pl, hipStream_t s);
// Levels [lvl0, lvl1) in one launch; ins/outs are indexed by level.
fc2t2_status launch_m2l_mfma(const fc2t2_plan_s* pl, int lvl0, int lvl1, const void* const* ins,
                             void* const* outs, bool accumulate, bool transpose, hipStream_t s,
                             const uint8_t* const* occ = nullptr, uint8_t gen = 1);

// ---- rays.hip
size_t ray_integral_bwd_ws(const fc2t2_plan_s* pl, int64_t R);
fc2t2_status launch_ray_integral(const fc2t2_plan_s* pl, const void* L, const void* o,
                                 const void* r, double t0, double t1, int64_t R, void* y,
                                 hipStream_t s);
fc2t2_status ray_integral_backward(const fc2t2_plan_s* pl, const void* o, const void* r, double t0,
                                   double t1, int64_t R, const void* gy, void* gL, void* ws,
                                   hipStream_t s);
fc2t2_status launch_ray_root(const fc2t2_plan_s* pl, const void* L, const void* o, const void* r,
                             double t0, double t1, int64_t R, double frac, void* t, void* normal,
                             int32_t* hit, void* saved, hipStream_t s, const void* tau_in = nullptr);
size_t ray_root_bwd_ws(const fc2t2_plan_s* pl, int64_t R);
// Resolves the device address of the fixed scratch array of the no-allocation entry point on
// the current device (once per device) into pl->noalloc_scratch; leaves it null on failure.
void noalloc_setup(fc2t2_plan_s* pl);
fc2t2_status ray_root_backward(const fc2t2_plan_s* pl, const void* saved, const int32_t* hit,
                               int64_t R, const void* gt, const void* gn, void* gL, void* ws,
                               hipStream_t s);


// ---- volume.hip
size_t ray_volume_bwd_ws(const fc2t2_plan_s* pl, int64_t R);

}  // namespace fc2t2

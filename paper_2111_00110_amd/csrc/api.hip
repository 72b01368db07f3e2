// The explicit layer's entry points (sections 3 and 4.1): expansion, evaluation and their
// backward passes, with argument validation and workspace carving.
#include "plan.h"

using namespace fc2t2;

namespace {

// Bump allocator over the caller's workspace (256-byte aligned pieces).
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

struct SortBufs {
  uint32_t *keys, *keys_sorted, *perm, *starts;
  void* pay;      // [count][dim + 1] sorted point data (when the sort carries it)
  void* scratch;
};

SortBufs carve_sort(Carve& c, const fc2t2_plan_s* pl, int64_t count) {
  SortBufs b;
  b.keys = c.take<uint32_t>(count);
  b.keys_sorted = c.take<uint32_t>(count);
  b.perm = c.take<uint32_t>(count);
  b.starts = c.take<uint32_t>(pl->G + 1);
  b.pay = sort_payload_ok(pl) ? (void*)c.take<float>((size_t)count * (pl->dim + pl->C)) : nullptr;
  b.scratch = c.take<char>(radix_sort_scratch_bytes(count));
  return b;
}

// Sorts points by cell; with `extra` (`words` values per point) and a carved payload buffer, the
// coordinates and those values are sorted along into b.pay.
fc2t2_status bin_and_sort(const fc2t2_plan_s* pl, const void* x, int64_t count, const SortBufs& b,
                          hipStream_t s, const void* extra = nullptr, unsigned long long* ood = nullptr,
                          int words = 1) {
  fc2t2_status st = sort_points_by_cell(pl, x, count, b.keys, b.keys_sorted, b.perm, b.scratch, s, extra,
                                        extra ? b.pay : nullptr, ood, words);
  if (st) return st;
  return launch_cell_starts(b.keys_sorted, count, pl->G, b.starts, s, sort_err_word(b.scratch, count), pl->sort_fail);
}

// The next occupancy stamp of a plan (1..255).
uint8_t next_gen(const fc2t2_plan_s* pl) {
  pl->occ_gen = (uint8_t)(pl->occ_gen % 255 + 1);
  return pl->occ_gen;
}

// Occupancy byte maps of every level (== the call's stamp: the cell's subtree holds a source).
void carve_occupancy(Carve& c, const fc2t2_plan_s* pl, uint8_t** occ) {
  for (int l = 0; l < kMaxLevels; ++l) occ[l] = nullptr;
  for (int l = 0; l < pl->levels; ++l) occ[l] = c.take<uint8_t>((size_t)pl->Gl[l]);
}

// Pyramid of grids for levels [first, levels): returns per-level pointers.
void carve_pyramid(Carve& c, const fc2t2_plan_s* pl, int first, void** lv) {
  for (int l = 0; l < kMaxLevels; ++l) lv[l] = nullptr;
  for (int l = first; l < pl->levels; ++l) lv[l] = c.take<char>(grid_elems(pl, l) * io_size(pl));
}

size_t ws_expand(const fc2t2_plan_s* pl, int64_t N) {
  Carve c(nullptr);
  carve_sort(c, pl, N);
  void* lv[kMaxLevels];
  carve_pyramid(c, pl, 0, lv);
  carve_pyramid(c, pl, 1, lv);
  uint8_t* occ[kMaxLevels];
  carve_occupancy(c, pl, occ);
  c.take<char>(sep_ws_bytes(pl));
  return c.off;
}

// Records of queries sorted by cell with their coordinates, kept from fc2t2_eval_sorted for
// fc2t2_eval_backward_sorted.
struct QueryRecords {
  uint32_t *keys, *keys_sorted, *perm, *starts;
  float* pay;     // [M][dim]
  void* scratch;
};

QueryRecords carve_query_records(Carve& c, const fc2t2_plan_s* pl, int64_t M) {
  QueryRecords b;
  b.keys = c.take<uint32_t>(M);
  b.keys_sorted = c.take<uint32_t>(M);
  b.perm = c.take<uint32_t>(M);
  b.starts = c.take<uint32_t>(pl->G + 1);
  b.pay = c.take<float>((size_t)M * pl->dim);
  b.scratch = c.take<char>(radix_sort_scratch_bytes(M));
  return b;
}

size_t ws_eval_sorted(const fc2t2_plan_s* pl, int64_t M) {
  Carve c(nullptr);
  carve_query_records(c, pl, M);
  return c.off;
}

size_t ws_bin_points(int64_t N) {
  Carve c(nullptr);
  c.take<uint32_t>(N);
  c.take<char>(radix_sort_scratch_bytes(N));
  return c.off;
}

size_t ws_eval_backward(const fc2t2_plan_s* pl, int64_t M) {
  Carve c(nullptr);
  carve_sort(c, pl, M);
  return c.off;
}

size_t ws_expand_backward(const fc2t2_plan_s* pl) {
  Carve c(nullptr);
  void* lv[kMaxLevels];
  carve_pyramid(c, pl, 1, lv);
  carve_pyramid(c, pl, 0, lv);
  uint8_t* occ[kMaxLevels];
  carve_occupancy(c, pl, occ);
  c.take<char>(sep_ws_bytes(pl));
  return c.off;
}

bool bad_count(int64_t n) { return n < 0 || n > 0xFFFFFFFFll; }

}  // namespace

namespace fc2t2 {

// Expansion of the finest moments M0 into the finest locals L0: M2M up the pyramid, M2L at
// every level (one launch), then L2L down the pyramid accumulating into each finer level.
// occ: occupancy maps with level 0 stamped with gen (the rest are filled on the way up).
fc2t2_status expand_from_moments(const fc2t2_plan_s* pl, void** Mlv, void** Llv, void* L0, hipStream_t s,
                                 uint8_t** occ, uint8_t gen, void* sep_ws) {
  Llv[0] = L0;
  fc2t2_status st;
  {
    StageScope t(pl, FC2T2_STAGE_SHIFT_UP, s);
    st = upshift_pyramid(pl, Mlv, s, occ, gen);
  }
  if (st) return st;
  {
    StageScope t(pl, FC2T2_STAGE_M2L, s);
    st = launch_m2l_all(pl, (const void* const*)Mlv, Llv, false, s, (const uint8_t* const*)occ, gen, sep_ws);
  }
  if (st) return st;
  StageScope t(pl, FC2T2_STAGE_SHIFT_DOWN, s);
  return downshift_pyramid(pl, Llv, s);
}

// Transpose of expand_from_moments: G_L0 -> G_M0 (L2L^T up, M2L^T at every level, M2M^T down).
fc2t2_status expand_T_to_moments(const fc2t2_plan_s* pl, const void* GL0, void** GLlv, void** GMlv,
                                 hipStream_t s, uint8_t** occ, uint8_t gen, void* sep_ws) {
  GLlv[0] = (void*)GL0;
  fc2t2_status st;
  {
    StageScope t(pl, FC2T2_STAGE_SHIFT_UP, s);
    st = upshift_pyramid(pl, GLlv, s, occ, gen);             // L2L^T
  }
  if (st) return st;
  {
    StageScope t(pl, FC2T2_STAGE_M2L_T, s);
    st = launch_m2l_all(pl, (const void* const*)GLlv, GMlv, true, s, (const uint8_t* const*)occ, gen, sep_ws);
  }
  if (st) return st;
  StageScope t(pl, FC2T2_STAGE_SHIFT_DOWN, s);
  return downshift_pyramid(pl, GMlv, s);                     // M2M^T
}

}  // namespace fc2t2

namespace {

fc2t2_status eval_backward_impl(fc2t2_plan plan, const void* L, const void* q, int64_t M, const void* gy, void* gL,
                                void* gq, void* ws, size_t ws_bytes, hipStream_t stream, bool acc) {
  if (!plan || bad_count(M)) return FC2T2_EINVAL;
  if (M > 0 && (!q || !gy)) return FC2T2_EINVAL;
  if (gq && !L) return FC2T2_EINVAL;
  if (M == 0) {   // nothing to add; overwriting means zero
    return gL && !acc ? launch_zero(plan, gL, (int64_t)grid_elems(plan, 0), stream) : FC2T2_OK;
  }
  if (gL) {
    const size_t need = ws_eval_backward(plan, M);
    if (!ws || ws_bytes < need) return FC2T2_EWORKSPACE;
    Carve c(ws);
    SortBufs sb = carve_sort(c, plan, M);
    fc2t2_status st;
    const bool carry = sb.pay != nullptr && plan->C == 1;   // the sorted q_bar pass is one channel
    {
      StageScope t(plan, FC2T2_STAGE_SORT, stream);
      st = bin_and_sort(plan, q, M, sb, stream, carry ? gy : nullptr);
    }
    if (st) return st;
    if (carry) {   // contiguous sorted queries
      {
        StageScope t(plan, FC2T2_STAGE_L2P_T, stream);
        st = launch_reduce_sorted(plan, sb.pay, M, sb.starts, gL, acc, stream);
      }
      if (st || !gq) return st;
      StageScope t(plan, FC2T2_STAGE_QGRAD, stream);
      // q_bar in cell order (rows from cache, scattered writes of q_bar) in 2-D; in input order
      // (scattered row reads, contiguous writes) in 3-D, where the wider scattered writes
      // measured slower
      if (plan->dim == 2)
        return launch_qgrad_sorted(plan, L, sb.pay, sb.keys_sorted, sb.perm, M, gq, stream, acc,
                                   sort_err_word(sb.scratch, M));
      return launch_l2p_qgrad(plan, L, q, M, gy, gq, stream, acc);
    }
    StageScope t(plan, FC2T2_STAGE_L2P_T, stream);
    if (gq && plan->C == 1) {   // one pass over the sorted queries produces both (q_bar accumulated)
      if (!acc && (st = launch_zero(plan, gq, M * plan->dim, stream))) return st;
      return launch_l2p_T_qgrad(plan, L, q, gy, M, sb.starts, sb.perm, gL, gq, stream, acc);
    }
    st = launch_l2p_T(plan, q, gy, M, sb.starts, sb.perm, gL, stream, acc);
    if (st) return st;
    if (gq) return launch_l2p_qgrad(plan, L, q, M, gy, gq, stream, acc);
    return FC2T2_OK;
  }
  StageScope t(plan, FC2T2_STAGE_QGRAD, stream);
  if (gq) return launch_l2p_qgrad(plan, L, q, M, gy, gq, stream, acc);
  return FC2T2_OK;
}

fc2t2_status expand_backward_impl(fc2t2_plan plan, const void* gL, const void* p, const void* w, int64_t N,
                                  void* gp, void* gw, void* ws, size_t ws_bytes, hipStream_t stream, bool acc) {
  if (!plan || !gL || bad_count(N)) return FC2T2_EINVAL;
  if (N > 0 && (!p || !w)) return FC2T2_EINVAL;
  if (N == 0 || (!gp && !gw)) return FC2T2_OK;
  const size_t need = ws_expand_backward(plan);
  if (!ws || ws_bytes < need) return FC2T2_EWORKSPACE;
  Carve c(ws);
  void* GLlv[kMaxLevels];
  void* GMlv[kMaxLevels];
  carve_pyramid(c, plan, 1, GLlv);
  carve_pyramid(c, plan, 0, GMlv);
  uint8_t* occ[kMaxLevels];
  carve_occupancy(c, plan, occ);
  void* sep_ws = c.take<char>(sep_ws_bytes(plan));
  const uint8_t gen = next_gen(plan);
  fc2t2_status st;
  {
    StageScope t(plan, FC2T2_STAGE_SORT, stream);   // binning of the sources (occupancy only)
    st = launch_mark_cells(plan, p, N, occ[0], gen, stream);
  }
  if (st) return st;
  st = expand_T_to_moments(plan, gL, GLlv, GMlv, stream, occ, gen, sep_ws);
  if (st) return st;
  StageScope t(plan, FC2T2_STAGE_P2M_T, stream);
  return launch_p2m_T(plan, GMlv[0], p, w, N, gp, gw, stream, acc);
}

}  // namespace

extern "C" {

size_t fc2t2_workspace_size(fc2t2_plan plan, int op, int64_t count) {
  if (!plan || count < 0) return 0;
  switch (op) {
    case FC2T2_OP_EXPAND: return ws_expand(plan, count);
    case FC2T2_OP_EVAL_BACKWARD: return ws_eval_backward(plan, count);
    case FC2T2_OP_EXPAND_BACKWARD: return ws_expand_backward(plan);
    case FC2T2_OP_RAY_INTEGRAL_BACKWARD: return ray_integral_bwd_ws(plan, count);
    case FC2T2_OP_RAY_ROOT_BACKWARD: return ray_root_bwd_ws(plan, count);
    case FC2T2_OP_EVAL_SORTED: return ws_eval_sorted(plan, count);
    case FC2T2_OP_RAY_VOLUME_BACKWARD: return ray_volume_bwd_ws(plan, count);
    case FC2T2_OP_BIN_POINTS: return ws_bin_points(count);
  }
  return 0;
}

fc2t2_status fc2t2_expand(fc2t2_plan plan, const void* p, const void* w, int64_t N, void* L,
                          void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!plan || !L || bad_count(N)) return FC2T2_EINVAL;
  if (N > 0 && (!p || !w)) return FC2T2_EINVAL;
  const size_t need = ws_expand(plan, N);
  if (!ws || ws_bytes < need) return FC2T2_EWORKSPACE;
  Carve c(ws);
  SortBufs sb = carve_sort(c, plan, N);
  void* Mlv[kMaxLevels];
  void* Llv[kMaxLevels];
  carve_pyramid(c, plan, 0, Mlv);
  carve_pyramid(c, plan, 1, Llv);
  uint8_t* occ[kMaxLevels];
  carve_occupancy(c, plan, occ);
  void* sep_ws = c.take<char>(sep_ws_bytes(plan));
  const uint8_t gen = next_gen(plan);
  fc2t2_status st;
  const bool carry = sb.pay != nullptr;   // sort the points' data along with the keys
  {
    StageScope t(plan, FC2T2_STAGE_SORT, stream);
    st = bin_and_sort(plan, p, N, sb, stream, carry ? w : nullptr, plan->ood, plan->C);
  }
  if (st) return st;
  {
    StageScope t(plan, FC2T2_STAGE_P2M, stream);
    st = carry ? launch_reduce_sorted(plan, sb.pay, N, sb.starts, Mlv[0], false, stream, occ[0], gen)
               : launch_p2m(plan, p, w, N, sb.starts, sb.perm, Mlv[0], stream, occ[0], gen);
  }
  if (st) return st;
  return expand_from_moments(plan, Mlv, Llv, L, stream, occ, gen, sep_ws);
}

fc2t2_status fc2t2_eval(fc2t2_plan plan, const void* L, const void* q, int64_t M, void* y, void* grad,
                        void* hess, hipStream_t stream) {
  if (!plan || !L || bad_count(M)) return FC2T2_EINVAL;
  if (M > 0 && (!q || !y)) return FC2T2_EINVAL;
  StageScope t(plan, FC2T2_STAGE_L2P, stream);
  return launch_l2p(plan, L, q, M, y, grad, hess, stream);
}

fc2t2_status fc2t2_bin_points(fc2t2_plan plan, const void* x, int64_t N, const void* extra, uint32_t* keys_sorted,
                              uint32_t* perm, uint32_t* starts, void* pay_out, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
  if (!plan || !starts || bad_count(N)) return FC2T2_EINVAL;
  if (N > 0 && (!x || !keys_sorted || !perm)) return FC2T2_EINVAL;
  if (extra && !pay_out) return FC2T2_EINVAL;
  if (pay_out && !sort_payload_ok(plan)) return FC2T2_EUNSUPPORTED;
  if (plan->G > 0xFFFFFFFFll) return FC2T2_EUNSUPPORTED;
  if (!ws || ws_bytes < ws_bin_points(N)) return FC2T2_EWORKSPACE;
  Carve c(ws);
  uint32_t* keys = c.take<uint32_t>(N);
  void* scratch = c.take<char>(radix_sort_scratch_bytes(N));
  StageScope t(plan, FC2T2_STAGE_SORT, stream);
  if (N > 0) {
    const fc2t2_status st = sort_points_by_cell(plan, x, N, keys, keys_sorted, perm, scratch, stream, extra, pay_out,
                                                plan->ood, 1);
    if (st) return st;
  }
  return launch_cell_starts(keys_sorted, N, plan->G, starts, stream, N > 0 ? sort_err_word(scratch, N) : nullptr,
                            plan->sort_fail);
}

fc2t2_status fc2t2_sort_queries(fc2t2_plan plan, const void* q, int64_t M, void* ws, size_t ws_bytes,
                                hipStream_t stream) {
  if (!plan || bad_count(M)) return FC2T2_EINVAL;
  if (M > 0 && !q) return FC2T2_EINVAL;
  if (!sort_payload_ok(plan) || plan->C != 1) return FC2T2_EUNSUPPORTED;
  if (!ws || ws_bytes < ws_eval_sorted(plan, M)) return FC2T2_EWORKSPACE;
  if (M == 0) return FC2T2_OK;
  Carve c(ws);
  const QueryRecords b = carve_query_records(c, plan, M);
  StageScope t(plan, FC2T2_STAGE_SORT, stream);
  fc2t2_status st = sort_points_by_cell(plan, q, M, b.keys, b.keys_sorted, b.perm, b.scratch, stream, nullptr,
                                        b.pay, plan->ood);
  if (st) return st;
  return launch_cell_starts(b.keys_sorted, M, plan->G, b.starts, stream, sort_err_word(b.scratch, M),
                            plan->sort_fail);
}

fc2t2_status fc2t2_eval_presorted(fc2t2_plan plan, const void* L, int64_t M, void* y, const void* ws,
                                  size_t ws_bytes, hipStream_t stream) {
  if (!plan || !L || bad_count(M)) return FC2T2_EINVAL;
  if (M > 0 && !y) return FC2T2_EINVAL;
  if (!sort_payload_ok(plan) || plan->C != 1) return FC2T2_EUNSUPPORTED;
  if (!ws || ws_bytes < ws_eval_sorted(plan, M)) return FC2T2_EWORKSPACE;
  if (M == 0) return FC2T2_OK;
  Carve c((void*)ws);
  const QueryRecords b = carve_query_records(c, plan, M);
  StageScope t(plan, FC2T2_STAGE_L2P, stream);
  return launch_l2p_sorted(plan, L, b.pay, b.keys_sorted, b.perm, M, y, stream, sort_err_word(b.scratch, M));
}

fc2t2_status fc2t2_eval_sorted(fc2t2_plan plan, const void* L, const void* q, int64_t M, void* y, void* ws,
                               size_t ws_bytes, hipStream_t stream) {
  if (!plan || !L || bad_count(M)) return FC2T2_EINVAL;
  if (M > 0 && (!q || !y)) return FC2T2_EINVAL;
  fc2t2_status st = fc2t2_sort_queries(plan, q, M, ws, ws_bytes, stream);
  if (st) return st;
  return fc2t2_eval_presorted(plan, L, M, y, ws, ws_bytes, stream);
}

fc2t2_status fc2t2_eval_backward_sorted(fc2t2_plan plan, const void* L, int64_t M, const void* gy, void* gL,
                                        void* gq, const void* ws, size_t ws_bytes, int accumulate,
                                        hipStream_t stream) {
  if (!plan || !gL || bad_count(M)) return FC2T2_EINVAL;
  if (M > 0 && !gy) return FC2T2_EINVAL;
  if (gq && !L) return FC2T2_EINVAL;
  if (!sort_payload_ok(plan) || plan->C != 1) return FC2T2_EUNSUPPORTED;
  if (!ws || ws_bytes < ws_eval_sorted(plan, M)) return FC2T2_EWORKSPACE;
  if (M == 0) return accumulate ? FC2T2_OK : launch_zero(plan, gL, (int64_t)grid_elems(plan, 0), stream);
  Carve c((void*)ws);
  const QueryRecords b = carve_query_records(c, plan, M);
  StageScope t(plan, FC2T2_STAGE_L2P_T, stream);
  return launch_l2p_T_qgrad_sorted(plan, L, b.pay, b.starts, b.perm, gy, M, gL, gq, stream, accumulate != 0);
}

fc2t2_status fc2t2_eval_backward(fc2t2_plan plan, const void* L, const void* q, int64_t M,
                                 const void* gy, void* gL, void* gq, void* ws, size_t ws_bytes,
                                 hipStream_t stream) {
  return eval_backward_impl(plan, L, q, M, gy, gL, gq, ws, ws_bytes, stream, true);
}

fc2t2_status fc2t2_eval_backward_ex(fc2t2_plan plan, const void* L, const void* q, int64_t M,
                                    const void* gy, void* gL, void* gq, void* ws, size_t ws_bytes,
                                    int accumulate, hipStream_t stream) {
  return eval_backward_impl(plan, L, q, M, gy, gL, gq, ws, ws_bytes, stream, accumulate != 0);
}

fc2t2_status fc2t2_expand_backward(fc2t2_plan plan, const void* gL, const void* p, const void* w,
                                   int64_t N, void* gp, void* gw, void* ws, size_t ws_bytes,
                                   hipStream_t stream) {
  return expand_backward_impl(plan, gL, p, w, N, gp, gw, ws, ws_bytes, stream, true);
}

fc2t2_status fc2t2_expand_backward_ex(fc2t2_plan plan, const void* gL, const void* p, const void* w,
                                      int64_t N, void* gp, void* gw, void* ws, size_t ws_bytes,
                                      int accumulate, hipStream_t stream) {
  return expand_backward_impl(plan, gL, p, w, N, gp, gw, ws, ws_bytes, stream, accumulate != 0);
}

fc2t2_status fc2t2_m2l(fc2t2_plan plan, int level, int transpose, const void* in, void* out,
                       int accumulate, hipStream_t stream) {
  if (!plan || !in || !out || level < 0 || level >= plan->levels) return FC2T2_EINVAL;
  StageScope t(plan, transpose ? FC2T2_STAGE_M2L_T : FC2T2_STAGE_M2L, stream);
  return transpose ? launch_m2l_T(plan, level, in, out, accumulate != 0, stream)
                   : launch_m2l(plan, level, in, out, accumulate != 0, stream);
}

size_t fc2t2_level_numel(fc2t2_plan plan, int level) {
  if (!plan || level < 0 || level >= plan->levels) return 0;
  return grid_elems(plan, level);
}

}  // extern "C"

// M2L on the matrix cores (gfx950 v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// The M2L of one level (section 3, K^{M2L}) is a convolution whose 6^d-wide window depends
// on the parity of the target cell.  Grouping targets by parity makes it an implicit GEMM
// per parity class:
//     L[t, k] = sum_{(o, n)} M[t + o, n] * T_o[n, k]
// rows t = targets of one parity, columns k = local multi-indices, reduction over the 6^d
// admissible offsets o times the source multi-indices n.  The tensor T_o depends only on
// the offset, so one table serves every parity; above the finest level the hole offsets
// (|o| <= 1) hold zero blocks, so every level walks the same 6^d window.
//
// The transpose M2L^T has the same structure: substituting o' = -o, the source-side
// window of a source cell's parity is again [-2, 3] (even) / [-3, 2] (odd), with the
// tensor T'_{o'}[k, n] = T_{-o'}[n, k]; it runs the same kernel with a second table.
//
// Work decomposition: a workgroup owns a TPX x TPY (x TPZ) block of parent cells, i.e. all
// 2^d children parities of it; wave w owns parity class w and RM = (parents / 16) row tiles
// of 16 targets, for NT column tiles of 16.  The reduction runs over slices of 8 source
// multi-indices (n8): for each slice the moments of the tile's source region
// ((2 TP + 4)^d cells) are staged in LDS as BF16 hi and lo planes (16 B per cell each);
// each 32-deep MFMA step takes four consecutive offsets of the parity's window (one per
// 16-lane group).  B fragments stream from the per-level table (L2-resident).
//
// Operand precision variants (template parameter EL):
//  * BF16 (v_mfma_f32_16x16x32_bf16): 1 pass  Mhi*Thi; 2 passes + Mhi*Tlo (the tensor's
//    rounding dominates the one-pass error); 3 passes + Mlo*Thi.  A BF16 hi/lo pair holds 16
//    bits of mantissa, so three passes leave about 2^-17 per operand.
//  * FP16 (v_mfma_f32_16x16x32_f16, same rate): three passes of an FP16 hi/lo split, which holds
//    22 bits of mantissa (about 2^-22 per operand, the FP32 class).  FP16's narrow exponent
//    range is handled with powers of two (exact, and undone exactly on the output):
//      - the input index i (source multi-index n forward, local k transposed) is scaled by
//        s_i = 2^floor(log2(2^|i| i!)): cell-scaled moments and local cotangents are bounded by
//        their cell sum over 2^|i| i!, so the scaled inputs are of one magnitude across i, and
//        the tensor's rows are divided by the same s_i (the products are unchanged);
//      - each level's scaled tensor gets the power of two that brings its largest entry to
//        2^14 (plan time), and each workgroup its scaled source region (a pre-pass over it);
//    the accumulator is multiplied back when written.  Without the per-index scaling the small
//    low-order terms of a level fall below FP16's normal range, where the matrix cores flush
//    them.
//  * FP32 (v_mfma_f32_16x16x4_f32): the plain FP32 contraction on the matrix cores, the same
//    data flow with FP32 operands and eight 4-deep instructions per 32-deep step.
#include <string.h>

#include "plan.h"

using namespace fc2t2;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kElBf16 = 0, kElF16 = 1, kElF32 = 2;
constexpr float kF16Top = 16384.f;   // 2^14: the largest scaled FP16 operand

__device__ __forceinline__ unsigned short bf16_bits_rne(float x) {
  unsigned u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
  return (unsigned short)u;
}
__device__ __forceinline__ float bf16_bits_to_float(unsigned short b) {
  return __uint_as_float(((unsigned)b) << 16);
}
__device__ __forceinline__ unsigned short f16_bits_rne(float x) {
  return __builtin_bit_cast(unsigned short, (_Float16)x);
}
__device__ __forceinline__ float f16_bits_to_float(unsigned short b) {
  return (float)__builtin_bit_cast(_Float16, b);
}
// 2^e with 2^e * amax in (2^13, 2^14]: the power of two that brings the largest magnitude
// to the top of the FP16 range used (1 for an all-zero input; at most 2^100, so that it and
// its inverse stay finite in FP32).
__device__ __host__ inline float f16_scale_for(float amax) {
  if (!(amax > 0.f) || !(amax < INFINITY)) return 1.f;
  int e;
  frexpf(amax, &e);            // amax = m 2^e, m in [0.5, 1)
  return ldexpf(1.f, 14 - (e < -86 ? -86 : e));
}

constexpr int ceil8(int p) { return (p + 7) / 8 * 8; }
constexpr int ntiles(int p) { return (p + 15) / 16; }

// ---------------------------------------------------------------------------------------
// Table: [dir][plane][lvl][o in 7^D (+1 zero block)][n8][NT*16][8] 16-bit operands.
//   dir 0 (forward):   in-channel n, out-channel k, value T[lvl][o][n][k]
//   dir 1 (transpose): in-channel k, out-channel n, value T[lvl][-o][n][k]
// Entries are zero outside [0, P), and for hole offsets (max |o| <= 1) above the finest
// level.  BF16: plane 0 = bf16(v), plane 1 = bf16(v - plane 0).  FP16: the same with
// v = T * scale[lvl].  FP32: the two 16-bit planes of a direction hold one plane of FP32 values
// [lvl][o][n8][NT*16][8].
struct LevelScales {
  float s[2][kMaxLevels];      // [direction][level]
};
__global__ void pack_mfma_table_kernel(const float* __restrict__ T, int D, int P, int Ppad, int P8,
                                       int NTC, int levels, int n_off, unsigned short* __restrict__ out,
                                       int64_t plane_stride, int64_t dir_stride, int el, LevelScales sc,
                                       const float* __restrict__ in_scale) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per_lvl = (int64_t)(n_off + 1) * P8 * NTC;   // (o, in, out) triples
  const int64_t total = 2 * (int64_t)levels * per_lvl;
  if (tid >= total) return;
  // decompose: dir, lvl, o, n8, outc, j  (in = n8*8 + j)
  int64_t r = tid;
  const int j = (int)(r % 8); r /= 8;
  const int outc = (int)(r % NTC); r /= NTC;
  const int n8 = (int)(r % (P8 / 8)); r /= (P8 / 8);
  const int oi = (int)(r % (n_off + 1)); r /= (n_off + 1);
  const int lvl = (int)(r % levels); r /= levels;
  const int dir = (int)r;
  const int inc = n8 * 8 + j;
  float v = 0.0f;
  if (oi < n_off && inc < P && outc < P) {
    int o[3] = {0, 0, 0};
    int rr = oi;
    for (int d = D - 1; d >= 0; --d) { o[d] = rr % 7 - 3; rr /= 7; }
    const int am = max(max(abs(o[0]), abs(o[1])), abs(o[2]));
    if (lvl == 0 || am > 1) {
      if (dir == 0) {
        v = T[(((int64_t)lvl * n_off + oi) * P + inc) * Ppad + outc];
      } else {
        int om = 0;
        for (int d = 0; d < D; ++d) om = om * 7 + (3 - o[d]);
        v = T[(((int64_t)lvl * n_off + om) * P + outc) * Ppad + inc];
      }
    }
  }
  // destination layout index (without dir/plane)
  const int64_t idx = ((((int64_t)lvl * (n_off + 1) + oi) * (P8 / 8) + n8) * NTC + outc) * 8 + j;
  if (el == kElF32) {
    reinterpret_cast<float*>(out + dir * dir_stride)[idx] = v;
    return;
  }
  unsigned short hi, lo;
  if (el == kElF16) {
    const float vs = inc < P ? v / in_scale[inc] * sc.s[dir][lvl] : 0.f;
    hi = f16_bits_rne(vs);
    lo = f16_bits_rne(vs - f16_bits_to_float(hi));
  } else {
    hi = bf16_bits_rne(v);
    lo = bf16_bits_rne(v - bf16_bits_to_float(hi));
  }
  out[dir * dir_stride + idx] = hi;
  out[dir * dir_stride + plane_stride + idx] = lo;
}

// Largest magnitude of each level's tensor with its input index scaled out, per direction
// (forward: input n, |T[n][k]| / s_n; transposed: input k, |T[n][k]| / s_k), as the bits of a
// non-negative float (ordered like unsigned integers, so an integer max is exact and
// order-independent).  Only the offsets a level uses count: the hole (max |o| <= 1) is not
// part of the levels above the finest.  out [2][levels].
__global__ void level_absmax_kernel(const float* __restrict__ T, int D, int P, int Ppad, int64_t per_level,
                                    int levels, const float* __restrict__ in_scale, unsigned* __restrict__ out) {
  const int lvl = blockIdx.y;
  if (lvl >= levels) return;
  float m0 = 0.f, m1 = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_level; i += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(i % Ppad), n = (int)((i / Ppad) % P);
    if (k >= P) continue;
    if (lvl > 0) {
      int rr = (int)(i / ((int64_t)P * Ppad)), am = 0;
      for (int d = 0; d < D; ++d) {
        am = max(am, abs(rr % 7 - 3));
        rr /= 7;
      }
      if (am <= 1) continue;
    }
    const float a = fabsf(T[lvl * per_level + i]);
    m0 = fmaxf(m0, a / in_scale[n]);
    m1 = fmaxf(m1, a / in_scale[k]);
  }
  for (int off = 32; off >= 1; off >>= 1) {
    m0 = fmaxf(m0, __shfl_xor(m0, off));
    m1 = fmaxf(m1, __shfl_xor(m1, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out + lvl, __float_as_uint(m0));
    atomicMax(out + kMaxLevels + lvl, __float_as_uint(m1));
  }
}

// ---------------------------------------------------------------------------------------
template <int D, int P, int TPX, int TPY, int TPZ, int PASSES, int EL>
struct Cfg {
  static constexpr int P8 = ceil8(P);
  static constexpr int NT = ntiles(P);
  static constexpr int NTC = NT * 16;
  static constexpr int NPAR = 1 << D;                 // parity classes = waves
  static constexpr int PARENTS = TPX * TPY * TPZ;
  static constexpr int RM = PARENTS / 16;             // row tiles per wave
  static constexpr int SX = 2 * TPX + 4, SY = 2 * TPY + 4, SZ = D == 3 ? 2 * TPZ + 4 : 1;
  static constexpr int CELLS = SX * SY * SZ;
  static constexpr int WIN = D == 3 ? 216 : 36;       // 6^D admissible offsets per parity
  static constexpr int KSTEPS = WIN / 4;
  static constexpr int THREADS = 64 * NPAR;
  static_assert(PARENTS % 16 == 0, "parent tile must hold a multiple of 16 parents");
  static_assert(D == 3 || TPZ == 1, "2-D tiles have TPZ = 1");
};

// One launch covers every level of the pyramid: the levels' M2L are independent given the
// moments, so the workgroups of the small coarse levels run beside those of the finest.
struct M2LLevel {
  const float* in;
  float* out;
  const uint8_t* occ;      // occupancy of the level's cells, or null (dense)
  const unsigned short* Bhi;
  const unsigned short* Blo;   // FP32 operands: unused (Bhi holds the FP32 plane)
  float unscale;               // 1 / the level's tensor scale (FP16 operands), else 1
  int64_t G_l;
  int n_l, tiles_y, tiles_z, block_begin;
};
struct M2LBatch {
  M2LLevel lv[kMaxLevels];
  const float* in_scale;   // FP16 operands: s_i per input index (P8 entries, zero-padded)
  int nlev, Ppad, accumulate;
  int occ_out;             // 0: skip tiles with an empty source region; 1: with no occupied target
  int gen;                 // occupied <=> byte == gen
};

template <class C>
__global__ void __launch_bounds__(C::THREADS) m2l_mfma_kernel(const M2LBatch batch) {
  constexpr int D = C::D_, P = C::P_;
  constexpr int P8 = C::P8, NT = C::NT, NTC = C::NTC, RM = C::RM;
  constexpr int SX = C::SX, SY = C::SY, SZ = C::SZ, CELLS = C::CELLS;
  constexpr int PASSES = C::PASSES_;
  constexpr int EL = C::EL_;
  constexpr int KSTEPS = C::KSTEPS;
  // staged moments: 16-bit hi (and lo) planes, or one FP32 plane in the space of both
  __shared__ __attribute__((aligned(16))) unsigned short lds_hi[EL == kElF32 ? CELLS * 16 : CELLS * 8];
  __shared__ __attribute__((aligned(16))) unsigned short lds_lo[PASSES >= 3 ? CELLS * 8 : 8];
  float* const lds_f = reinterpret_cast<float*>(lds_hi);

  const int ch = blockIdx.y;
  // XCD-aware order: consecutive logical tiles share an XCD (dispatch is round-robin over 8)
  const int nblk = gridDim.x;
  int bid = blockIdx.x;
  if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);
  int lvl = batch.nlev - 1;
  while (lvl > 0 && bid < batch.lv[lvl].block_begin) --lvl;
  const M2LLevel& LV = batch.lv[lvl];
  const float* __restrict__ Min = LV.in;
  float* __restrict__ Lout = LV.out;
  const unsigned short* __restrict__ Bhi = LV.Bhi;
  const unsigned short* __restrict__ Blo = LV.Blo;
  const int n_l = LV.n_l, Ppad = batch.Ppad, accumulate = batch.accumulate;
  const int64_t G_l = LV.G_l;
  const int tiles_y = LV.tiles_y, tiles_z = LV.tiles_z;
  bid -= LV.block_begin;
  const int tz = bid % tiles_z;
  const int ty = (bid / tiles_z) % tiles_y;
  const int tx = bid / (tiles_z * tiles_y);
  // region origin (cell coords at this level) = 2 * parent origin - 2
  const int rx0 = 2 * tx * C::TPX_ - 2, ry0 = 2 * ty * C::TPY_ - 2, rz0 = D == 3 ? 2 * tz * C::TPZ_ - 2 : 0;

  const int tid = threadIdx.x;
  if (LV.occ) {
    // sparse sources: a tile whose source region (forward) or whose targets (transpose) hold
    // no occupied cell contributes nothing the method reads; it writes zeros and stops
    int any = 0;
    if (!batch.occ_out) {
      for (int c = tid; c < CELLS; c += C::THREADS) {
        const int cz = c % SZ, cy = (c / SZ) % SY, cx = c / (SZ * SY);
        const int gx = rx0 + cx, gy = ry0 + cy, gz = rz0 + cz;
        if (gx >= 0 && gx < n_l && gy >= 0 && gy < n_l && (D == 2 || (gz >= 0 && gz < n_l))) {
          const int64_t cell = D == 3 ? ((int64_t)gx * n_l + gy) * n_l + gz : (int64_t)gx * n_l + gy;
          any |= LV.occ[cell] == batch.gen;
        }
      }
    } else {
      constexpr int TX = 2 * C::TPX_, TY = 2 * C::TPY_, TZ = D == 3 ? 2 * C::TPZ_ : 1;
      for (int c = tid; c < TX * TY * TZ; c += C::THREADS) {
        const int cz = c % TZ, cy = (c / TZ) % TY, cx = c / (TZ * TY);
        const int gx = rx0 + 2 + cx, gy = ry0 + 2 + cy, gz = D == 3 ? rz0 + 2 + cz : 0;
        if (gx < n_l && gy < n_l && (D == 2 || gz < n_l)) {
          const int64_t cell = D == 3 ? ((int64_t)gx * n_l + gy) * n_l + gz : (int64_t)gx * n_l + gy;
          any |= LV.occ[cell] == batch.gen;
        }
      }
    }
    if (!__syncthreads_or(any)) {
      if (!accumulate) {
        constexpr int TX = 2 * C::TPX_, TY = 2 * C::TPY_, TZ = D == 3 ? 2 * C::TPZ_ : 1;
        float* __restrict__ Lz = Lout + (int64_t)ch * G_l * Ppad;
        for (int i = tid; i < TX * TY * TZ * Ppad; i += C::THREADS) {
          const int c = i / Ppad, k = i - c * Ppad;
          const int cz = c % TZ, cy = (c / TZ) % TY, cx = c / (TZ * TY);
          const int gx = rx0 + 2 + cx, gy = ry0 + 2 + cy, gz = D == 3 ? rz0 + 2 + cz : 0;
          if (gx < n_l && gy < n_l && (D == 2 || gz < n_l)) {
            const int64_t cell = D == 3 ? ((int64_t)gx * n_l + gy) * n_l + gz : (int64_t)gx * n_l + gy;
            Lz[cell * Ppad + k] = 0.f;
          }
        }
      }
      return;
    }
  }
  const int wave = tid >> 6, lane = tid & 63;
  const int px_bit = D == 3 ? (wave >> 2) & 1 : (wave >> 1) & 1;
  const int py_bit = D == 3 ? (wave >> 1) & 1 : wave & 1;
  const int pz_bit = D == 3 ? wave & 1 : 0;
  const int row = lane & 15, grp = lane >> 4;

  // LDS cell index of this lane's target for each row tile (A operand rows)
  int tcell[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const int p = m * 16 + row;
    const int pz = p % C::TPZ_, py = (p / C::TPZ_) % C::TPY_, px = p / (C::TPZ_ * C::TPY_);
    const int cx = 2 * px + px_bit + 2, cy = 2 * py + py_bit + 2, cz = D == 3 ? 2 * pz + pz_bit + 2 : 0;
    tcell[m] = (cx * SY + cy) * SZ + cz;
  }
  const int wlo_x = px_bit ? -3 : -2, wlo_y = py_bit ? -3 : -2, wlo_z = pz_bit ? -3 : -2;

  floatx4 acc[RM][NT];
#pragma unroll
  for (int m = 0; m < RM; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = floatx4{0.f, 0.f, 0.f, 0.f};

  const float* __restrict__ Mch = Min + (int64_t)ch * G_l * Ppad;
  // window entry e = 4 s + grp as digits (ex, ey, ez) in base 6; advanced by 4 per step
  const int e0 = grp;

  // FP16 operands: the power of two that brings the region's largest moment to 2^14
  float mscale = 1.f;
  __shared__ float s_in[EL == kElF16 ? P8 : 1];
  if constexpr (EL == kElF16) {
    __shared__ float red[C::THREADS / 64];
    if (tid < P8) s_in[tid] = batch.in_scale[tid];
    __syncthreads();
    float m = 0.f;
    for (int c = tid; c < CELLS; c += C::THREADS) {
      const int cz = c % SZ, cy = (c / SZ) % SY, cx = c / (SZ * SY);
      const int gx = rx0 + cx, gy = ry0 + cy, gz = rz0 + cz;
      if (gx >= 0 && gx < n_l && gy >= 0 && gy < n_l && (D == 2 || (gz >= 0 && gz < n_l))) {
        const int64_t cell = D == 3 ? ((int64_t)gx * n_l + gy) * n_l + gz : (int64_t)gx * n_l + gy;
        const float4* src = reinterpret_cast<const float4*>(Mch + cell * Ppad);
        for (int k = 0; k < Ppad / 4; ++k) {
          const float4 a = src[k];
          m = fmaxf(m, fmaxf(fmaxf(fabsf(a.x) * s_in[4 * k], fabsf(a.y) * s_in[4 * k + 1]),
                             fmaxf(fabsf(a.z) * s_in[4 * k + 2], fabsf(a.w) * s_in[4 * k + 3])));
        }
      }
    }
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (lane == 0) red[wave] = m;
    __syncthreads();
    m = red[0];
#pragma unroll
    for (int w = 1; w < C::THREADS / 64; ++w) m = fmaxf(m, red[w]);
    mscale = f16_scale_for(m);
  }

  for (int n8 = 0; n8 < P8 / 8; ++n8) {
    // ---- stage the source region's slice [n8*8, n8*8+8) as bf16 hi / lo
    for (int c = tid; c < CELLS; c += C::THREADS) {
      const int cz = c % SZ, cy = (c / SZ) % SY, cx = c / (SZ * SY);
      const int gx = rx0 + cx, gy = ry0 + cy, gz = rz0 + cz;
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = 0.f;
      const bool inside = gx >= 0 && gx < n_l && gy >= 0 && gy < n_l && (D == 2 || (gz >= 0 && gz < n_l));
      if (inside) {
        const int64_t cell = D == 3 ? ((int64_t)gx * n_l + gy) * n_l + gz : (int64_t)gx * n_l + gy;
        const float* src = Mch + cell * Ppad + n8 * 8;
        if (n8 * 8 + 4 <= Ppad) {
          const float4 a = *reinterpret_cast<const float4*>(src);
          v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        }
        if (n8 * 8 + 8 <= Ppad) {
          const float4 b = *reinterpret_cast<const float4*>(src + 4);
          v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        }
      }
      if constexpr (EL == kElF32) {
        *reinterpret_cast<float4*>(&lds_f[c * 8]) = make_float4(v[0], v[1], v[2], v[3]);
        *reinterpret_cast<float4*>(&lds_f[c * 8 + 4]) = make_float4(v[4], v[5], v[6], v[7]);
        continue;
      }
      unsigned short hi[8], lo[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if constexpr (EL == kElF16) {
          const float vs = v[j] * s_in[n8 * 8 + j] * mscale;
          hi[j] = f16_bits_rne(vs);
          lo[j] = f16_bits_rne(vs - f16_bits_to_float(hi[j]));
        } else {
          hi[j] = bf16_bits_rne(v[j]);
          lo[j] = bf16_bits_rne(v[j] - bf16_bits_to_float(hi[j]));
        }
      }
      uint4 h4, l4;
      h4.x = hi[0] | ((unsigned)hi[1] << 16); h4.y = hi[2] | ((unsigned)hi[3] << 16);
      h4.z = hi[4] | ((unsigned)hi[5] << 16); h4.w = hi[6] | ((unsigned)hi[7] << 16);
      l4.x = lo[0] | ((unsigned)lo[1] << 16); l4.y = lo[2] | ((unsigned)lo[3] << 16);
      l4.z = lo[4] | ((unsigned)lo[5] << 16); l4.w = lo[6] | ((unsigned)lo[7] << 16);
      *reinterpret_cast<uint4*>(&lds_hi[c * 8]) = h4;
      if constexpr (PASSES >= 3) *reinterpret_cast<uint4*>(&lds_lo[c * 8]) = l4;
    }
    __syncthreads();

    // ---- 32-deep MFMA steps: group g of the wave takes window entry 4 * s + g
    int ex, ey, ez;
    if constexpr (D == 3) { ez = e0 % 6; ey = (e0 / 6) % 6; ex = e0 / 36; }
    else { ez = 0; ey = e0 % 6; ex = e0 / 6; }
    auto b_base = [&](int qx, int qy, int qz) -> int64_t {
      const int ox = wlo_x + qx, oy = wlo_y + qy, oz = D == 3 ? wlo_z + qz : 0;
      const int ob = D == 3 ? ((ox + 3) * 7 + (oy + 3)) * 7 + (oz + 3) : (ox + 3) * 7 + (oy + 3);
      return (((int64_t)ob * (P8 / 8) + n8) * NTC + row) * 8;
    };
    // B fragments: 8 consecutive 16-bit values per lane per column tile (hi, and lo), or for FP32
    // operands 8 FP32 values (the two uint4 of a tile hold its first and last four)
    auto fetch_b = [&](int64_t bb, uint4 (&fh)[NT], uint4 (&fl)[NT]) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if constexpr (EL == kElF32) {
          const float* bf = reinterpret_cast<const float*>(Bhi) + bb + (int64_t)t * 16 * 8;
          fh[t] = *reinterpret_cast<const uint4*>(bf);
          fl[t] = *reinterpret_cast<const uint4*>(bf + 4);
        } else {
          fh[t] = *reinterpret_cast<const uint4*>(Bhi + bb + (int64_t)t * 16 * 8);
          if constexpr (PASSES >= 2) fl[t] = *reinterpret_cast<const uint4*>(Blo + bb + (int64_t)t * 16 * 8);
        }
      }
    };
    auto advance = [&](int& qx, int& qy, int& qz) {
      if constexpr (D == 3) {
        qz += 4;
        if (qz >= 6) { qz -= 6; ++qy; if (qy >= 6) { qy -= 6; ++qx; } }
      } else {
        qy += 4;
        if (qy >= 6) { qy -= 6; ++qx; }
      }
    };
    uint4 nbh[NT], nbl[NT];
    fetch_b(b_base(ex, ey, ez), nbh, nbl);
    for (int s = 0; s < KSTEPS; ++s) {
      uint4 bh[NT], bl[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        bh[t] = nbh[t];
        if constexpr (PASSES >= 2 || EL == kElF32) bl[t] = nbl[t];
      }
      const int ox = wlo_x + ex, oy = wlo_y + ey, oz = D == 3 ? wlo_z + ez : 0;
      const int delta = (ox * SY + oy) * SZ + oz;
      // prefetch the next step's B fragments
      if (s + 1 < KSTEPS) {
        advance(ex, ey, ez);
        fetch_b(b_base(ex, ey, ez), nbh, nbl);
      }
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const int cidx = tcell[m] + delta;
        if constexpr (EL == kElF32) {
          // eight 4-deep FP32 steps: step j takes source multi-index n8 * 8 + j of the lane's
          // window offset (k index = lane group), as the 32-deep 16-bit step does in one
          const float4 a0 = *reinterpret_cast<const float4*>(&lds_f[cidx * 8]);
          const float4 a1 = *reinterpret_cast<const float4*>(&lds_f[cidx * 8 + 4]);
          const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const float bv[8] = {__uint_as_float(bh[t].x), __uint_as_float(bh[t].y), __uint_as_float(bh[t].z),
                                 __uint_as_float(bh[t].w), __uint_as_float(bl[t].x), __uint_as_float(bl[t].y),
                                 __uint_as_float(bl[t].z), __uint_as_float(bl[t].w)};
#pragma unroll
            for (int j = 0; j < 8; ++j)
              acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j], bv[j], acc[m][t], 0, 0, 0);
          }
        } else if constexpr (EL == kElF16) {
          const halfx8 ah = __builtin_bit_cast(halfx8, *reinterpret_cast<const uint4*>(&lds_hi[cidx * 8]));
          const halfx8 al = __builtin_bit_cast(halfx8, *reinterpret_cast<const uint4*>(&lds_lo[cidx * 8]));
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const halfx8 bhv = __builtin_bit_cast(halfx8, bh[t]), blv = __builtin_bit_cast(halfx8, bl[t]);
            acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bhv, acc[m][t], 0, 0, 0);
            acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, blv, acc[m][t], 0, 0, 0);
            acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bhv, acc[m][t], 0, 0, 0);
          }
        } else {
          const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&lds_hi[cidx * 8]));
          bf16x8 al;
          if constexpr (PASSES >= 3) al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&lds_lo[cidx * 8]));
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const bf16x8 bhv = __builtin_bit_cast(bf16x8, bh[t]);
            acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bhv, acc[m][t], 0, 0, 0);
            if constexpr (PASSES >= 2)
              acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, __builtin_bit_cast(bf16x8, bl[t]), acc[m][t], 0, 0, 0);
            if constexpr (PASSES >= 3) acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bhv, acc[m][t], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- write: lane holds D[4*grp + i][row] of each (m, t) tile (scaled back for FP16 operands:
  // a product of powers of two, exact)
  float* __restrict__ Lch = Lout + (int64_t)ch * G_l * Ppad;
  const float unscale = EL == kElF16 ? LV.unscale / mscale : 1.f;
#pragma unroll
  for (int m = 0; m < RM; ++m) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = m * 16 + 4 * grp + i;
      const int pz = p % C::TPZ_, py = (p / C::TPZ_) % C::TPY_, px = p / (C::TPZ_ * C::TPY_);
      const int gx = rx0 + 2 + 2 * px + px_bit, gy = ry0 + 2 + 2 * py + py_bit;
      const int gz = D == 3 ? rz0 + 2 + 2 * pz + pz_bit : 0;
      if (gx >= n_l || gy >= n_l || (D == 3 && gz >= n_l)) continue;
      const int64_t cell = D == 3 ? ((int64_t)gx * n_l + gy) * n_l + gz : (int64_t)gx * n_l + gy;
      float* dst = Lch + cell * Ppad;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int k = t * 16 + row;
        if (k < P) {
          const float v = acc[m][t][i] * unscale;
          if (accumulate) dst[k] += v; else dst[k] = v;
        } else if (k < Ppad && !accumulate) {
          dst[k] = 0.f;
        }
      }
    }
  }
}

// Expose the template parameters under names usable inside the kernel.
template <int D, int P, int TPX, int TPY, int TPZ, int PASSES, int EL>
struct CfgX : Cfg<D, P, TPX, TPY, TPZ, PASSES, EL> {
  static constexpr int D_ = D, P_ = P, TPX_ = TPX, TPY_ = TPY, TPZ_ = TPZ, PASSES_ = PASSES, EL_ = EL;
};

template <int D, int P, int PASSES, int EL>
struct Tile;
// 2-D: 8 x 4 parents (128 targets, 4 waves, two 16-row tiles each)
template <int P, int PASSES, int EL>
struct Tile<2, P, PASSES, EL> { using type = CfgX<2, P, 8, 4, 1, PASSES, EL>; };
// 3-D: 8 x 4 x 4 parents for P > 35 (1024 targets, 8 waves, eight 16-row tiles each: the tensor
// fragment a wave loads feeds 8 row tiles), 8 x 4 x 2 for P <= 35 (half the LDS, two workgroups
// per compute unit, and finer blocks when tiles are skipped)
template <int P, int PASSES, int EL>
struct Tile<3, P, PASSES, EL> { using type = CfgX<3, P, 8, 4, (P <= 35 ? 2 : 4), PASSES, EL>; };

template <class C>
fc2t2_status launch_cfg(const fc2t2_plan_s* pl, int lvl0, int lvl1, const void* const* ins, void* const* outs,
                        bool accumulate, const unsigned short* base, int64_t plane, int64_t per_lvl,
                        hipStream_t s, const uint8_t* const* occ, uint8_t gen, bool transpose) {
  M2LBatch b;
  b.nlev = 0;
  b.Ppad = pl->Ppad;
  b.accumulate = accumulate ? 1 : 0;
  b.occ_out = transpose ? 1 : 0;
  b.gen = gen;
  int blocks = 0;
  for (int lvl = lvl0; lvl < lvl1; ++lvl) {
    const int n_l = pl->nl[lvl];
    const int npar = n_l / 2;
    const int tx = (npar + C::TPX_ - 1) / C::TPX_, ty = (npar + C::TPY_ - 1) / C::TPY_;
    const int tz = C::D_ == 3 ? (npar + C::TPZ_ - 1) / C::TPZ_ : 1;
    M2LLevel& L = b.lv[b.nlev++];
    L.in = (const float*)ins[lvl];
    L.out = (float*)outs[lvl];
    L.occ = occ ? occ[lvl] : nullptr;
    if (C::EL_ == kElF32) {   // one FP32 plane [lvl][...] in the direction's space
      L.Bhi = base + 2 * lvl * per_lvl;
      L.Blo = nullptr;
    } else {
      L.Bhi = base + lvl * per_lvl;
      L.Blo = base + plane + lvl * per_lvl;
    }
    L.unscale = C::EL_ == kElF16 ? 1.f / pl->t_scale[transpose ? 1 : 0][lvl] : 1.f;
    L.G_l = pl->Gl[lvl];
    L.n_l = n_l;
    L.tiles_y = ty;
    L.tiles_z = tz;
    L.block_begin = blocks;
    blocks += tx * ty * tz;
  }
  b.in_scale = (const float*)((const char*)pl->m2l_bf16 + m2l_mfma_table_bytes_only(pl));
  const dim3 grid((unsigned)blocks, pl->C);
  hipLaunchKernelGGL((m2l_mfma_kernel<C>), grid, dim3(C::THREADS), 0, s, b);
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

struct TableGeom {
  int P8, NTC;
  int64_t per_lvl, plane, dir;
};

TableGeom table_geom(const fc2t2_plan_s* pl) {
  TableGeom g;
  g.P8 = ceil8(pl->P);
  g.NTC = ntiles(pl->P) * 16;
  g.per_lvl = (int64_t)(pl->n_off + 1) * g.P8 * g.NTC;
  g.plane = g.per_lvl * pl->levels;
  g.dir = 2 * g.plane;
  return g;
}

}  // namespace

namespace fc2t2 {

size_t m2l_mfma_table_bytes_only(const fc2t2_plan_s* pl) {
  const TableGeom g = table_geom(pl);
  return align256((size_t)g.dir * 2 * sizeof(unsigned short));
}

bool m2l_mfma_supported(const fc2t2_plan_s* pl) {
  return pl->io == FC2T2_IO_F32 && fc2t2_supported(pl->dim, pl->K);
}

size_t m2l_mfma_table_bytes(const fc2t2_plan_s* pl) {
  // the operand tables, then the FP16 input scales (64 floats) and the scratch of the
  // per-level maxima (2 x kMaxLevels words)
  return m2l_mfma_table_bytes_only(pl) + 64 * sizeof(float) + 2 * kMaxLevels * sizeof(unsigned);
}

int operand_el(const fc2t2_plan_s* pl) {
  return pl->prec == FC2T2_M2L_F16X3 ? kElF16 : (pl->prec == FC2T2_M2L_F32_MFMA ? kElF32 : kElBf16);
}

fc2t2_status m2l_mfma_build_tables(fc2t2_plan_s* pl, hipStream_t s) {
  const size_t bytes = m2l_mfma_table_bytes(pl);
  if (hipMalloc(&pl->m2l_bf16, bytes) != hipSuccess) { pl->m2l_bf16 = nullptr; return FC2T2_ENOMEM; }
  pl->m2l_bf16_bytes = bytes;
  const TableGeom g = table_geom(pl);
  const int el = operand_el(pl);
  LevelScales sc;
  for (int d = 0; d < 2; ++d)
    for (int l = 0; l < kMaxLevels; ++l) sc.s[d][l] = 1.f;
  // input-index scales s_i = 2^floor(log2(2^|i| i!)) (FP16 operands; ones otherwise), zero-padded
  float host_in[64] = {};
  {
    int mi[64 * 3];
    fc2t2_multi_indices(pl->dim, pl->K, mi);
    for (int i = 0; i < pl->P; ++i) {
      double v = 1.0;
      for (int j = 0; j < pl->dim; ++j)
        for (int a = 2; a <= mi[i * pl->dim + j]; ++a) v *= a;
      for (int j = 0; j < pl->dim; ++j) v *= (double)(1 << mi[i * pl->dim + j]);
      int e;
      frexp(v, &e);
      host_in[i] = el == kElF16 ? (float)ldexp(1.0, e - 1) : 1.f;
    }
  }
  float* in_scale = (float*)((char*)pl->m2l_bf16 + m2l_mfma_table_bytes_only(pl));
  unsigned* amax = (unsigned*)(in_scale + 64);
  if (hipMemcpyAsync(in_scale, host_in, sizeof(host_in), hipMemcpyHostToDevice, s) != hipSuccess) return FC2T2_EHIP;
  if (el == kElF16) {
    // per (direction, level) power of two bringing the largest scaled tensor entry to 2^14
    const int64_t per_level = (int64_t)pl->n_off * pl->P * pl->Ppad;
    if (hipMemsetAsync(amax, 0, 2 * kMaxLevels * sizeof(unsigned), s) != hipSuccess) return FC2T2_EHIP;
    hipLaunchKernelGGL(level_absmax_kernel, dim3(64, pl->levels), dim3(256), 0, s, (const float*)pl->m2l_T, pl->dim,
                       pl->P, pl->Ppad, per_level, pl->levels, (const float*)in_scale, amax);
    FC2T2_LAUNCH_CHECK();
    unsigned host[2 * kMaxLevels] = {};
    if (hipMemcpyAsync(host, amax, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return FC2T2_EHIP;
    for (int d = 0; d < 2; ++d)
      for (int l = 0; l < pl->levels; ++l) {
        float m;
        memcpy(&m, &host[d * kMaxLevels + l], sizeof(m));
        sc.s[d][l] = f16_scale_for(m);
      }
  }
  for (int d = 0; d < 2; ++d)
    for (int l = 0; l < kMaxLevels; ++l) pl->t_scale[d][l] = sc.s[d][l];
  const int64_t total = 2 * (int64_t)pl->levels * g.per_lvl;
  hipLaunchKernelGGL(pack_mfma_table_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s,
                     (const float*)pl->m2l_T, pl->dim, pl->P, pl->Ppad, g.P8, g.NTC, pl->levels, pl->n_off,
                     (unsigned short*)pl->m2l_bf16, g.plane, g.dir, el, sc, (const float*)in_scale);
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

fc2t2_status launch_m2l_mfma(const fc2t2_plan_s* pl, int lvl0, int lvl1, const void* const* ins,
                             void* const* outs, bool accumulate, bool transpose, hipStream_t s,
                             const uint8_t* const* occ, uint8_t gen) {
  if (!pl->m2l_bf16) return FC2T2_EUNSUPPORTED;
  const TableGeom g = table_geom(pl);
  const unsigned short* base = (const unsigned short*)pl->m2l_bf16 + (transpose ? g.dir : 0);
  fc2t2_status st = FC2T2_EUNSUPPORTED;
  dispatch_shape(pl->dim, pl->K, [&](auto shape) {
    using S = decltype(shape);
    switch (pl->prec) {
      case FC2T2_M2L_BF16:
        st = launch_cfg<typename Tile<S::D, S::P, 1, kElBf16>::type>(pl, lvl0, lvl1, ins, outs, accumulate, base, g.plane, g.per_lvl, s, occ, gen, transpose);
        break;
      case FC2T2_M2L_BF16X2:
        st = launch_cfg<typename Tile<S::D, S::P, 2, kElBf16>::type>(pl, lvl0, lvl1, ins, outs, accumulate, base, g.plane, g.per_lvl, s, occ, gen, transpose);
        break;
      case FC2T2_M2L_BF16X3:
        st = launch_cfg<typename Tile<S::D, S::P, 3, kElBf16>::type>(pl, lvl0, lvl1, ins, outs, accumulate, base, g.plane, g.per_lvl, s, occ, gen, transpose);
        break;
      case FC2T2_M2L_F16X3:
        st = launch_cfg<typename Tile<S::D, S::P, 3, kElF16>::type>(pl, lvl0, lvl1, ins, outs, accumulate, base, g.plane, g.per_lvl, s, occ, gen, transpose);
        break;
      case FC2T2_M2L_F32_MFMA:
        st = launch_cfg<typename Tile<S::D, S::P, 1, kElF32>::type>(pl, lvl0, lvl1, ins, outs, accumulate, base, g.plane, g.per_lvl, s, occ, gen, transpose);
        break;
    }
  });
  return st;
}

}  // namespace fc2t2

// Per-cell segmented reduction over records sorted by cell (shared by P2M, the transpose
// of L2P, ray insertion and root insertion).
#pragma once

#include "plan.h"

namespace fc2t2 {

template <int D, typename T>
__device__ __forceinline__ void decode_cell(int64_t cell, int n, int (&ic)[3]) {
  ic[0] = ic[1] = ic[2] = 0;
  if constexpr (D == 2) {
    ic[1] = (int)(cell % n);
    ic[0] = (int)(cell / n);
  } else {
    ic[2] = (int)(cell % n);
    ic[1] = (int)((cell / n) % n);
    ic[0] = (int)(cell / ((int64_t)n * n));
  }
}

// out[ch][cell][:] (+)= sum over the cell's sorted records of fn(record); the record is the
// input index perm[r] of sorted position r, or r itself when perm is null (records whose
// data was sorted along with the keys).  occ (optional) receives gen for cells with records
// and 0 for the others.
// With kWaveCells, a cell holding more than 8 GROUP records is taken by the whole wave
// instead (crowded cells of clustered sources); it costs registers, so it is opt-in.
template <class S, typename T, int GROUP, bool kWaveCells, class F>
__global__ void __launch_bounds__(256) reduce_cells_kernel(const uint32_t* __restrict__ starts,
                                                           const uint32_t* __restrict__ perm,
                                                           int64_t G, int n, T lo, T h,
                                                           T* __restrict__ out, int accumulate, F fn,
                                                           uint8_t* __restrict__ occ, uint8_t gen) {
  constexpr int P = S::P, Ppad = S::Ppad, D = S::D;
  constexpr int CPW = kWave / GROUP;          // cells a wave takes per round
  constexpr uint32_t kBig = 8 * GROUP;        // records above which the whole wave takes the cell
  const int lane = threadIdx.x & (kWave - 1);
  const int lane_g = lane & (GROUP - 1);
  const int ch = blockIdx.y;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t wave_id = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  T* __restrict__ base = out + (int64_t)ch * G * Ppad;

  auto centre_of = [&](int64_t cell, T (&centre)[3]) {
    int ic[3];
    decode_cell<D, T>(cell, n, ic);
#pragma unroll
    for (int j = 0; j < 3; ++j) centre[j] = lo + (T(ic[j]) + T(0.5)) * h;
  };
  auto write_row = [&](int64_t cell, T (&s)[P], int lanes, int my) {
    T* __restrict__ dst = base + cell * Ppad;
#pragma unroll
    for (int k = 0; k < Ppad; ++k) {
      if (k % lanes == my) {
        const T v = k < P ? s[k] : T(0);
        if (accumulate) dst[k] += v; else dst[k] = v;
      }
    }
  };

  for (int64_t c0 = wave_id * CPW; c0 < G; c0 += waves * CPW) {
    const int64_t cell = c0 + lane / GROUP;
    const bool valid = cell < G;
    const uint32_t b = valid ? starts[cell] : 0u, e = valid ? starts[cell + 1] : 0u;
    if (occ && valid && lane_g == 0 && ch == 0) occ[cell] = e > b ? gen : 0;
    const bool big = kWaveCells && valid && (e - b) > kBig;
    // cells with few records: one group of GROUP lanes each
    if (valid && !big) {
      T centre[3];
      centre_of(cell, centre);
      T s[P], c[P];
#pragma unroll
      for (int k = 0; k < P; ++k) { s[k] = T(0); c[k] = T(0); }
      for (uint32_t r = b + lane_g; r < e; r += GROUP) {
        T v[P];
        fn(perm ? perm[r] : r, centre, ch, v, cell);
#pragma unroll
        for (int k = 0; k < P; ++k) acc2(s[k], c[k], v[k]);
      }
#pragma unroll
      for (int k = 0; k < P; ++k) s[k] += c[k];
#pragma unroll
      for (int off = GROUP / 2; off >= 1; off >>= 1) {
#pragma unroll
        for (int k = 0; k < P; ++k) s[k] += __shfl_xor(s[k], off, GROUP);
      }
      write_row(cell, s, GROUP, lane_g);
    }
    // cells with many records: the whole wave, one cell at a time
    if constexpr (!kWaveCells) continue;
    uint64_t bigs = __ballot(big && lane_g == 0);
    while (bigs) {
      const int src = __ffsll((unsigned long long)bigs) - 1;
      bigs &= bigs - 1;
      const int64_t bc = __shfl(cell, src);
      const uint32_t bb = __shfl(b, src), be = __shfl(e, src);
      T centre[3];
      centre_of(bc, centre);
      T s[P], c[P];
#pragma unroll
      for (int k = 0; k < P; ++k) { s[k] = T(0); c[k] = T(0); }
      for (uint32_t r = bb + lane; r < be; r += kWave) {
        T v[P];
        fn(perm ? perm[r] : r, centre, ch, v, bc);
#pragma unroll
        for (int k = 0; k < P; ++k) acc2(s[k], c[k], v[k]);
      }
#pragma unroll
      for (int k = 0; k < P; ++k) s[k] += c[k];
#pragma unroll
      for (int off = kWave / 2; off >= 1; off >>= 1) {
#pragma unroll
        for (int k = 0; k < P; ++k) s[k] += __shfl_xor(s[k], off);
      }
      write_row(bc, s, kWave, lane);
    }
  }
}


// Lanes per cell from the mean number of records per cell.
inline int reduce_group_for(int64_t records, int64_t cells) {
  const double avg = cells > 0 ? (double)records / (double)cells : 0.0;
  return avg < 24.0 ? 4 : (avg < 96.0 ? 16 : 64);
}

template <class S, typename T, int GROUP, bool kWaveCells, class F>
fc2t2_status launch_reduce_cells_g(const fc2t2_plan_s* pl, const uint32_t* starts, const uint32_t* perm,
                                   T* out, bool accumulate, const F& fn, hipStream_t s, uint8_t* occ,
                                   uint8_t gen) {
  const int threads = 256;
  const int64_t need = ceil_div(pl->G * GROUP, threads);   // one round of cells per wave
  const int64_t blocks = need < 16384 ? need : 16384;
  hipLaunchKernelGGL((reduce_cells_kernel<S, T, GROUP, kWaveCells, F>), dim3((unsigned)blocks, pl->C), dim3(threads), 0, s,
                     starts, perm, pl->G, pl->n, (T)pl->lo, (T)pl->h0, out, accumulate ? 1 : 0, fn, occ, gen);
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

template <class S, typename T, class F, bool kWaveCells = false>
fc2t2_status launch_reduce_cells(const fc2t2_plan_s* pl, const uint32_t* starts, const uint32_t* perm,
                                 int64_t records, T* out, bool accumulate, const F& fn, hipStream_t s,
                                 uint8_t* occ = nullptr, uint8_t gen = 1) {
  switch (reduce_group_for(records, pl->G)) {
    case 4: return launch_reduce_cells_g<S, T, 4, kWaveCells>(pl, starts, perm, out, accumulate, fn, s, occ, gen);
    case 16: return launch_reduce_cells_g<S, T, 16, kWaveCells>(pl, starts, perm, out, accumulate, fn, s, occ, gen);
    default: return launch_reduce_cells_g<S, T, 64, false>(pl, starts, perm, out, accumulate, fn, s, occ, gen);
  }
}

}  // namespace fc2t2

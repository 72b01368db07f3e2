// Binning of points to finest-level cells (section 3.3: the box of a point is an integer
// cast of its scaled coordinate) and a stable LSD radix sort of (cell, index) pairs, so
// that the per-cell reductions (P2M, L2P^T, ray insertion) visit every cell's records in
// input order without floating-point atomics.
#include <algorithm>

#include "plan.h"

using namespace fc2t2;

namespace {

constexpr int kThreads = 256;
constexpr int kBins = 256;                 // 8-bit digits
constexpr int kMaxPasses = 4;
// One-sweep passes: a tile is kItems consecutive items per lane, each wave a contiguous run of
// kItems * 64; 16 items per lane without payload, 8 with (LDS holds the staged payload).
constexpr int kWaves = kThreads / kWave;
constexpr int kTileMin = kThreads * 8;
template <int PW>
struct SweepShape {
  static constexpr int kItems = PW > 0 ? 8 : 16;
  static constexpr int kWaveRun = kItems * kWave;
  static constexpr int kTile = kThreads * kItems;
};
constexpr int kHistBlocks = 2048;  // at most this many histogram blocks; each writes its own counts
// Tile status words: value in the low 30 bits, flag in the top two (0 = not yet published,
// 1 = the tile's own counts, 2 = counts of all tiles up to and including this one).
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 2u << 30;
constexpr uint32_t kValMask = kFlagAgg - 1u;
constexpr uint32_t kMaxSpins = 1u << 22;   // bounded wait: a predecessor that never publishes sets err
// Test aid (fc2t2_debug_sort_fault): the spin limit of the look-back and a tile that withholds
// its published counts, so that the bounded wait gives up on purpose and every kernel still
// ends normally.
uint32_t g_max_spins = kMaxSpins;
uint32_t g_withhold_tile = 0xFFFFFFFFu;

// Sums the histogram blocks' counts in kSlices slices per pass: block (pass, slice), thread
// digit, writes sums[slice][pass][digit] (the sweep adds the slices).  Also clears the error word.
constexpr int kSlices = 16;
__global__ void __launch_bounds__(kThreads) sort_hist_sum_kernel(const uint32_t* __restrict__ part, int nblocks,
                                                                 uint32_t* __restrict__ sums,
                                                                 uint32_t* __restrict__ err) {
  const int pass = blockIdx.x, slice = blockIdx.y, d = threadIdx.x;
  uint32_t sum = 0;
#pragma unroll 8
  for (int b = slice; b < nblocks; b += kSlices) sum += part[((size_t)b * kMaxPasses + pass) * kBins + d];
  sums[((size_t)slice * kMaxPasses + pass) * kBins + d] = sum;
  if (pass == 0 && slice == 0 && d == 0) *err = 0u;
}

// Digit counts of every pass in one read of the keys (computed from points when x is given,
// then written to keys), one row of counts per block, and clearing of the passes' tile status
// words.
template <typename T, int D>
__global__ void __launch_bounds__(kThreads) sort_hist_kernel(const T* __restrict__ x, T lo, T scale, int n,
                                                             uint32_t* __restrict__ keys, uint32_t N, int npass,
                                                             uint32_t frequent, uint32_t* __restrict__ ghist,
                                                             uint32_t* __restrict__ status, uint32_t status_words,
                                                             unsigned long long* __restrict__ ood) {
  __shared__ uint32_t h[kMaxPasses][kBins];
  const int tid = threadIdx.x;
#pragma unroll
  for (int ps = 0; ps < kMaxPasses; ++ps) h[ps][tid] = 0u;
  __syncthreads();
  const uint32_t stride = gridDim.x * kThreads;
  constexpr int kBatch = 8;   // points per thread per round, loaded before any is used
  uint32_t nfreq = 0;         // keys equal to `frequent`, counted here and added once
  for (uint32_t i0 = blockIdx.x * kThreads + tid; i0 < N; i0 += kBatch * stride) {
    uint32_t key[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const uint32_t i = i0 + b * stride;
      key[b] = 0;
      if (i >= N) continue;
      if (x) {
        bool out = false;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const T xv = x[(size_t)i * D + j];
          out = out || outside_domain<T>(xv, lo, scale, n);
          key[b] = key[b] * (uint32_t)n + (uint32_t)cell_coord<T>(xv, lo, scale, n);
        }
        keys[i] = key[b];
        if (ood) count_lanes(out, ood);
      } else {
        key[b] = keys[i];
      }
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (i0 + b * stride >= N) continue;
      if (key[b] == frequent) {
        ++nfreq;
        continue;
      }
      for (int ps = 0; ps < npass; ++ps) atomicAdd(&h[ps][(key[b] >> (8 * ps)) & (kBins - 1)], 1u);
    }
  }
  if (nfreq)
    for (int ps = 0; ps < npass; ++ps) atomicAdd(&h[ps][(frequent >> (8 * ps)) & (kBins - 1)], nfreq);
  __syncthreads();
  uint32_t* mine = ghist + (size_t)blockIdx.x * kMaxPasses * kBins;   // this block's counts
  for (int ps = 0; ps < npass; ++ps) mine[ps * kBins + tid] = h[ps][tid];
  for (uint32_t w = blockIdx.x * kThreads + tid; w < status_words; w += stride) status[w] = 0u;
}

// Block-wide exclusive scan of one value per thread (256 threads); returns the total.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t& excl, uint32_t* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    const uint32_t t = tid >= off ? sh[tid - off] : 0u;
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  excl = sh[tid] - v;
  const uint32_t total = sh[kThreads - 1];
  __syncthreads();
  return total;
}

__device__ __forceinline__ uint32_t load_status(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_status(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One stable pass over 8 bits of the key.  Tile t is block t: workgroups are dispatched in
// index order on each XCD, so the lowest unfinished tile is always resident and every wait
// below ends; the wait is bounded besides (err).  Ranks: each wave
// walks its run item by item (input order), ranking a lane among equal digits with ballots
// and a per-wave running count; wave offsets come from the per-wave counts.  The tile then
// publishes its digit counts, looks back over the preceding tiles' status words for its
// global offsets (decoupled look-back), and writes each digit's items as one contiguous run
// through an LDS staging copy in digit order.
// Optional payload: PW 32-bit words per item, written to pay_out [N][PW]; read from pa (na words
// per item) and pb (PW - na words per item), either staged with the key through LDS (GATHER
// false: pa, pb indexed by input position) or fetched at write time by the item's original
// index (GATHER true, the last pass: pa, pb are the unsorted inputs and vals carry the original
// indices), so that earlier passes move only keys and indices.
template <int PW, bool GATHER = false, int NA = PW>
__global__ void __launch_bounds__(kThreads) onesweep_kernel(const uint32_t* __restrict__ keys_in,
                                                            const uint32_t* __restrict__ vals_in, uint32_t N,
                                                            int shift, const uint32_t* __restrict__ ghist,
                                                            uint32_t* __restrict__ status,
                                                            uint32_t* __restrict__ keys_out,
                                                            uint32_t* __restrict__ vals_out, uint32_t* __restrict__ err,
                                                            const uint32_t* __restrict__ pa, int na,
                                                            const uint32_t* __restrict__ pb,
                                                            uint32_t* __restrict__ pay_out, uint32_t max_spins,
                                                            uint32_t withhold_tile) {
  constexpr int PS = GATHER ? 0 : PW;   // payload words staged through LDS
  constexpr int kItems = SweepShape<PS>::kItems, kWaveRun = SweepShape<PS>::kWaveRun;
  constexpr int kTile = SweepShape<PS>::kTile;
  __shared__ uint32_t wcount[kWaves][kBins];
  __shared__ uint32_t s_excl[kBins];
  __shared__ uint32_t s_gbase[kBins];
  __shared__ uint32_t scan_sh[kThreads];
  __shared__ uint32_t s_key[kTile];
  __shared__ uint32_t s_val[kTile];
  __shared__ uint32_t s_pay[PS > 0 ? PS * kTile : 1];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) wcount[w][tid] = 0u;
  __syncthreads();
  const uint32_t tile = blockIdx.x;
  const uint32_t run0 = tile * (uint32_t)kTile + (uint32_t)wave * kWaveRun;
  uint32_t key[kItems], val[kItems], rank[kItems];
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint32_t i = run0 + (uint32_t)j * kWave + lane;
    const bool ok = i < N;
    key[j] = ok ? keys_in[i] : 0u;
    val[j] = ok ? (vals_in ? vals_in[i] : i) : 0u;
  }
  uint32_t pay[kItems][PS > 0 ? PS : 1];
  if constexpr (PS > 0) {
    const int nb = PW - na;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint32_t i = run0 + (uint32_t)j * kWave + lane;
#pragma unroll
      for (int w = 0; w < PW; ++w)
        pay[j][w] = i < N ? (w < na ? pa[(size_t)i * na + w] : pb[(size_t)i * nb + (w - na)]) : 0u;
    }
  }
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t* wc = wcount[wave];
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const bool ok = run0 + (uint32_t)j * kWave + lane < N;
    const uint32_t digit = (key[j] >> shift) & (kBins - 1);
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot(ok && ((digit >> b) & 1u));
      peers &= ((digit >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t before = ok ? wc[digit] : 0u;
    rank[j] = before + below;
    __builtin_amdgcn_wave_barrier();
    if (ok && below == 0u) wc[digit] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per digit (thread tid): offsets of the waves and the tile's count
  uint32_t cnt = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t t = wcount[w][tid];
    wcount[w][tid] = cnt;
    cnt += t;
  }
  uint32_t* my = status + (size_t)tile * kBins + tid;
  const bool publish = tile != withhold_tile;
  if (publish) store_status(my, (tile == 0 ? kFlagInc : kFlagAgg) | cnt);
  uint32_t excl;
  block_exclusive_scan(cnt, excl, scan_sh);
  s_excl[tid] = excl;
  // look back 16 tiles per round: their status words are loaded together and consumed from
  // the nearest; a tile that has not published yet ends the round (polled again after a sleep)
  uint32_t prefix = 0;
  if (tile > 0) {
    constexpr int kLook = 16;
    int t = (int)tile - 1;
    uint32_t spins = 0;
    for (;;) {
      uint32_t v[kLook];
#pragma unroll
      for (int k = 0; k < kLook; ++k) v[k] = (t - k >= 0) ? load_status(status + (size_t)(t - k) * kBins + tid) : kFlagInc;
      bool done = false, stall = false;
      int used = 0;
#pragma unroll
      for (int k = 0; k < kLook; ++k) {
        if (done || stall) continue;
        if ((v[k] & ~kValMask) == 0u) {
          stall = true;
        } else {
          prefix += v[k] & kValMask;
          used = k + 1;
          if (v[k] & kFlagInc) done = true;
        }
      }
      if (done) break;
      t -= used;
      if (stall) {
        if (++spins > max_spins) {
          atomicOr(err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (publish) store_status(my, kFlagInc | (prefix + cnt));
  }
  uint32_t dtot = 0;
#pragma unroll
  for (int cp = 0; cp < kSlices; ++cp) dtot += ghist[(size_t)cp * kMaxPasses * kBins + tid];
  uint32_t dbase;
  block_exclusive_scan(dtot, dbase, scan_sh);
  s_gbase[tid] = dbase + prefix;
  __syncthreads();
  const uint32_t tile0 = tile * (uint32_t)kTile;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    if (run0 + (uint32_t)j * kWave + lane >= N) continue;
    const uint32_t digit = (key[j] >> shift) & (kBins - 1);
    const uint32_t lp = s_excl[digit] + wcount[wave][digit] + rank[j];
    s_key[lp] = key[j];
    s_val[lp] = val[j];
    if constexpr (PS > 0) {
#pragma unroll
      for (int w = 0; w < PW; ++w) s_pay[w * kTile + lp] = pay[j][w];
    }
  }
  __syncthreads();
  const uint32_t count = (N - tile0) < (uint32_t)kTile ? (N - tile0) : (uint32_t)kTile;
  if constexpr (GATHER && PW > 0) {
    // every item's position and original index first, then all of the thread's gathers in
    // flight together, then the writes.  v is an original index (< N) unless an earlier pass
    // failed (err set): the indices are then not a permutation, and the gather must not follow
    // them out of the inputs.
    constexpr int NB = PW - NA;
    uint32_t pos[kItems], v[kItems], kk[kItems], pv[kItems][PW];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint32_t t = (uint32_t)j * kThreads + tid;
      pos[j] = N;
      v[j] = N;
      kk[j] = 0u;
      if (t < count) {
        kk[j] = s_key[t];
        const uint32_t digit = (kk[j] >> shift) & (kBins - 1);
        pos[j] = s_gbase[digit] + (t - s_excl[digit]);
        v[j] = s_val[t];
      }
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const bool in = v[j] < N;
      const size_t vi = in ? v[j] : 0u;
#pragma unroll
      for (int w = 0; w < NA; ++w) pv[j][w] = pa[vi * NA + w];
#pragma unroll
      for (int w = 0; w < NB; ++w) pv[j][NA + w] = pb[vi * NB + w];
      if (!in)
#pragma unroll
        for (int w = 0; w < PW; ++w) pv[j][w] = 0u;
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      if (pos[j] >= N) continue;   // past the tile's end, or after a failed look-back (err set)
      keys_out[pos[j]] = kk[j];
      vals_out[pos[j]] = v[j];
#pragma unroll
      for (int w = 0; w < PW; ++w) pay_out[(size_t)pos[j] * PW + w] = pv[j][w];
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint32_t t = (uint32_t)j * kThreads + tid;
    if (t >= count) continue;
    const uint32_t k = s_key[t];
    const uint32_t digit = (k >> shift) & (kBins - 1);
    const uint32_t pos = s_gbase[digit] + (t - s_excl[digit]);
    if (pos >= N) continue;   // only after a failed look-back (err set)
    keys_out[pos] = k;
    vals_out[pos] = s_val[t];
    if constexpr (PW > 0) {
#pragma unroll
      for (int w = 0; w < PW; ++w) pay_out[(size_t)pos * PW + w] = s_pay[w * kTile + t];
    }
  }
}

// Cell starts of a sorted key array.  After a failed sort (err set) every cell is empty, so no
// later stage reads the unsorted records, and the plan's failure counter is incremented once.
__global__ void __launch_bounds__(256) cell_starts_kernel(const uint32_t* __restrict__ keys, int64_t N,
                                                          int64_t G, uint32_t* __restrict__ starts,
                                                          const uint32_t* __restrict__ err,
                                                          unsigned long long* __restrict__ fail_ctr) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > G) return;
  if (err && *err) {
    starts[c] = 0u;
    if (c == 0 && fail_ctr) atomicAdd(fail_ctr, 1ull);
    return;
  }
  int64_t lo = 0, hi = N;   // first position with key >= c
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] < c) lo = mid + 1; else hi = mid;
  }
  starts[c] = (uint32_t)lo;
}

}  // namespace

namespace fc2t2 {

int key_bits_for(int64_t G) {
  int b = 0;
  while ((int64_t(1) << b) < G) ++b;
  return b < 1 ? 1 : b;
}

}  // namespace fc2t2

namespace {

struct SortScratch {
  uint32_t *ktmp, *vtmp, *part, *ghist, *status, *err;
  uint32_t max_tiles;
};
// Histogram blocks for N keys and `words` status words to clear: about 8 items per thread, so
// that a streaming read of 10^7 keys keeps enough loads in flight on every CU.
int hist_blocks(int64_t N, int64_t words) {
  const int64_t work = N > words ? N : words;
  return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(work, kThreads * 8), 1), kHistBlocks);
}
int64_t max_status_words(int64_t N) { return (int64_t)kMaxPasses * ceil_div(N > 0 ? N : 1, kTileMin) * kBins; }
int64_t part_words(int64_t N) { return (int64_t)hist_blocks(N, max_status_words(N)) * kMaxPasses * kBins; }

SortScratch carve_scratch(void* scratch, int64_t N) {
  SortScratch c;
  c.max_tiles = (uint32_t)ceil_div(N > 0 ? N : 1, kTileMin);
  char* p = (char*)scratch;
  c.ktmp = (uint32_t*)p;
  p += align256((size_t)N * 4);
  c.vtmp = (uint32_t*)p;
  p += align256((size_t)N * 4);
  c.part = (uint32_t*)p;                  // per histogram block: kMaxPasses x kBins counts
  p += align256((size_t)part_words(N) * 4);
  c.ghist = (uint32_t*)p;                 // kSlices x kMaxPasses x kBins partial totals, then err
  c.err = c.ghist + kSlices * kMaxPasses * kBins;
  p += align256((kSlices * kMaxPasses * kBins + 1) * 4);
  c.status = (uint32_t*)p;
  return c;
}

// Passes of 8 bits; with a payload (PW > 0) the passes before the last move keys and indices
// only, and the last gathers each item's payload from the inputs by its original index.
template <int PW, int NA = PW>
fc2t2_status onesweep_passes(const uint32_t* keys_in, uint32_t* keys_out, uint32_t* vals_out, uint32_t N,
                             int npass, const SortScratch& c, const uint32_t* pa, int na, const uint32_t* pb,
                             uint32_t* pay_out, hipStream_t s) {
  const uint32_t* kin = keys_in;
  const uint32_t* vin = nullptr;
  for (int pass = 0; pass < npass; ++pass) {
    const bool to_out = ((npass - 1 - pass) % 2) == 0;
    const bool last = pass == npass - 1;
    uint32_t* kout = to_out ? keys_out : c.ktmp;
    uint32_t* vout = to_out ? vals_out : c.vtmp;
    const uint32_t tiles = (uint32_t)ceil_div(N, SweepShape<0>::kTile);
    if (PW > 0 && last)
      hipLaunchKernelGGL((onesweep_kernel<PW, true, NA>), dim3(tiles), dim3(kThreads), 0, s, kin, vin, N, 8 * pass,
                         c.ghist + pass * kBins, c.status + (size_t)pass * c.max_tiles * kBins, kout, vout, c.err,
                         pa, na, pb, pay_out, g_max_spins, g_withhold_tile);
    else
      hipLaunchKernelGGL((onesweep_kernel<0>), dim3(tiles), dim3(kThreads), 0, s, kin, vin, N, 8 * pass,
                         c.ghist + pass * kBins, c.status + (size_t)pass * c.max_tiles * kBins, kout, vout, c.err,
                         nullptr, 0, nullptr, nullptr, g_max_spins, g_withhold_tile);
    FC2T2_LAUNCH_CHECK();
    kin = kout;
    vin = vout;
  }
  return FC2T2_OK;
}

// Histogram (and keys from points when x is given) for npass passes of 8 bits; `frequent` is a
// key the caller expects many times (counted per thread instead of by shared-memory atomics on
// one address), or kNoKey.
constexpr uint32_t kNoKey = 0xFFFFFFFFu;
template <typename T, int D>
fc2t2_status sort_prologue(const T* x, T lo, T scale, int n, uint32_t* keys, uint32_t N, int npass,
                           unsigned long long* ood,
                           const SortScratch& c, hipStream_t s, uint32_t frequent = kNoKey) {
  const uint32_t status_words = (uint32_t)npass * c.max_tiles * kBins;
  const int blocks = hist_blocks(N, status_words);
  hipLaunchKernelGGL((sort_hist_kernel<T, D>), dim3(blocks), dim3(kThreads), 0, s, x, lo, scale, n, keys, N, npass,
                     frequent, c.part, c.status, status_words, ood);
  FC2T2_LAUNCH_CHECK();
  hipLaunchKernelGGL(sort_hist_sum_kernel, dim3(npass, kSlices), dim3(kThreads), 0, s, c.part, blocks, c.ghist,
                     c.err);
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

}  // namespace

namespace fc2t2 {

size_t radix_sort_scratch_bytes(int64_t N) {
  const int64_t tiles = ceil_div(N > 0 ? N : 1, kTileMin);
  return align256((size_t)N * 4) * 2 + align256((size_t)part_words(N) * 4) +
         align256((kSlices * kMaxPasses * kBins + 1) * 4) +
         align256((size_t)kMaxPasses * tiles * kBins * 4);
}

fc2t2_status radix_sort_pairs(const uint32_t* keys_in, uint32_t* keys_out, uint32_t* vals_out,
                              int64_t N, int key_bits, void* scratch, hipStream_t s, uint32_t frequent) {
  if (N == 0) return FC2T2_OK;
  if (N >= (int64_t)kValMask || key_bits > 8 * kMaxPasses) return FC2T2_EUNSUPPORTED;
  const SortScratch c = carve_scratch(scratch, N);
  const int npass = (key_bits + 7) / 8;
  fc2t2_status st =
      sort_prologue<float, 1>(nullptr, 0.f, 0.f, 0, (uint32_t*)keys_in, (uint32_t)N, npass, nullptr, c, s, frequent);
  if (st) return st;
  return onesweep_passes<0>(keys_in, keys_out, vals_out, (uint32_t)N, npass, c, nullptr, 0, nullptr, nullptr, s);
}

fc2t2_status sort_points_by_cell(const fc2t2_plan_s* pl, const void* x, int64_t N, uint32_t* keys,
                                 uint32_t* keys_out, uint32_t* vals_out, void* scratch, hipStream_t s,
                                 const void* extra, void* pay_out, unsigned long long* ood, int extra_words) {
  if (N == 0) return FC2T2_OK;
  if (N >= (int64_t)kValMask) return FC2T2_EUNSUPPORTED;
  const int key_bits = key_bits_for(pl->G);
  if (key_bits > 8 * kMaxPasses) return FC2T2_EUNSUPPORTED;
  const SortScratch c = carve_scratch(scratch, N);
  const int npass = (key_bits + 7) / 8;
  const double scale = pl->n / (pl->hi - pl->lo);
  fc2t2_status st;
  if (pl->io == FC2T2_IO_F64)
    st = pl->dim == 2 ? sort_prologue<double, 2>((const double*)x, pl->lo, scale, pl->n, keys, (uint32_t)N, npass, ood, c, s)
                      : sort_prologue<double, 3>((const double*)x, pl->lo, scale, pl->n, keys, (uint32_t)N, npass, ood, c, s);
  else
    st = pl->dim == 2 ? sort_prologue<float, 2>((const float*)x, (float)pl->lo, (float)scale, pl->n, keys, (uint32_t)N,
                                                 npass, ood, c, s)
                      : sort_prologue<float, 3>((const float*)x, (float)pl->lo, (float)scale, pl->n, keys, (uint32_t)N,
                                                 npass, ood, c, s);
  if (st) return st;
  if (pay_out) {
    if (!sort_payload_ok(pl)) return FC2T2_EUNSUPPORTED;
    const uint32_t* pa = (const uint32_t*)x;
    const uint32_t* pb = (const uint32_t*)extra;
    if (!extra)   // the coordinates only: pay_out [N][dim]
      return pl->dim == 2 ? onesweep_passes<2>(keys, keys_out, vals_out, (uint32_t)N, npass, c, pa, 2, nullptr,
                                               (uint32_t*)pay_out, s)
                          : onesweep_passes<3>(keys, keys_out, vals_out, (uint32_t)N, npass, c, pa, 3, nullptr,
                                               (uint32_t*)pay_out, s);
    // the coordinates and extra_words values per point: pay_out [N][dim + extra_words]
    const uint32_t n = (uint32_t)N;
    uint32_t* po = (uint32_t*)pay_out;
    if (pl->dim == 2) {
      switch (extra_words) {
        case 1: return onesweep_passes<3, 2>(keys, keys_out, vals_out, n, npass, c, pa, 2, pb, po, s);
        case 2: return onesweep_passes<4, 2>(keys, keys_out, vals_out, n, npass, c, pa, 2, pb, po, s);
        case 3: return onesweep_passes<5, 2>(keys, keys_out, vals_out, n, npass, c, pa, 2, pb, po, s);
        case 4: return onesweep_passes<6, 2>(keys, keys_out, vals_out, n, npass, c, pa, 2, pb, po, s);
      }
    } else {
      switch (extra_words) {
        case 1: return onesweep_passes<4, 3>(keys, keys_out, vals_out, n, npass, c, pa, 3, pb, po, s);
        case 2: return onesweep_passes<5, 3>(keys, keys_out, vals_out, n, npass, c, pa, 3, pb, po, s);
        case 3: return onesweep_passes<6, 3>(keys, keys_out, vals_out, n, npass, c, pa, 3, pb, po, s);
        case 4: return onesweep_passes<7, 3>(keys, keys_out, vals_out, n, npass, c, pa, 3, pb, po, s);
      }
    }
    return FC2T2_EUNSUPPORTED;
  }
  return onesweep_passes<0>(keys, keys_out, vals_out, (uint32_t)N, npass, c, nullptr, 0, nullptr, nullptr, s);
}

bool sort_payload_ok(const fc2t2_plan_s* pl) { return pl->io == FC2T2_IO_F32 && pl->C <= 4; }

const uint32_t* sort_err_word(const void* scratch, int64_t N) {
  return N > 0 ? carve_scratch((void*)scratch, N).err : nullptr;
}

fc2t2_status launch_cell_starts(const uint32_t* keys_sorted, int64_t N, int64_t G, uint32_t* starts,
                                hipStream_t s, const uint32_t* err, unsigned long long* fail_ctr) {
  const int threads = 256;
  hipLaunchKernelGGL(cell_starts_kernel, dim3((unsigned)ceil_div(G + 1, threads)), dim3(threads), 0, s,
                     keys_sorted, N, G, starts, err, fail_ctr);
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

}  // namespace fc2t2

extern "C" void fc2t2_debug_sort_fault(int enable) {
  g_max_spins = enable ? 64u : kMaxSpins;
  g_withhold_tile = enable ? 1u : 0xFFFFFFFFu;
}

// Binning of points to finest-level cells (section 3.3: the box of a point is an integer
// cast of its scaled coordinate) and a stable LSD radix sort of (cell, index) pairs, so
// that the per-cell reductions (P2M, L2P^T, ray insertion) visit every cell's records in
// input order without floating-point atomics.
#include "plan.h"

using namespace fc2t2;

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 4;
constexpr int kTile = kThreads * kItems;   // keys per block
constexpr int kBins = 256;                 // 8-bit digits

template <typename T, int D>
__global__ void __launch_bounds__(256) cell_keys_kernel(const T* __restrict__ x, int64_t N, T lo,
                                                        T scale, int n, uint32_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  uint32_t key = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) key = key * (uint32_t)n + (uint32_t)cell_coord<T>(x[i * D + j], lo, scale, n);
  keys[i] = key;
}

__global__ void __launch_bounds__(kThreads) radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                              int64_t N, int shift,
                                                              uint32_t* __restrict__ hist,
                                                              int nblocks) {
  __shared__ uint32_t cnt[kBins];
  const int tid = threadIdx.x;
  cnt[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = base + (int64_t)j * kThreads + tid;
    if (i < N) atomicAdd(&cnt[(keys[i] >> shift) & (kBins - 1)], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * nblocks + blockIdx.x] = cnt[tid];
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

// One block per digit: total count of the digit over all tiles.
__global__ void __launch_bounds__(kThreads) radix_digit_total_kernel(const uint32_t* __restrict__ hist,
                                                                     int nblocks,
                                                                     uint32_t* __restrict__ totals) {
  __shared__ uint32_t sh[kThreads];
  const int d = blockIdx.x;
  uint32_t s = 0;
  for (int b = threadIdx.x; b < nblocks; b += kThreads) s += hist[(int64_t)d * nblocks + b];
  uint32_t excl;
  const uint32_t tot = block_exclusive_scan(s, excl, sh);
  if (threadIdx.x == 0) totals[d] = tot;
}

// One block per digit: hist row d becomes the exclusive offsets of (d, tile).
__global__ void __launch_bounds__(kThreads) radix_offsets_kernel(uint32_t* __restrict__ hist, int nblocks,
                                                                 const uint32_t* __restrict__ totals) {
  __shared__ uint32_t sh[kThreads];
  const int d = blockIdx.x;
  const int tid = threadIdx.x;
  // base = sum of totals of smaller digits
  uint32_t excl_d;
  block_exclusive_scan(totals[tid], excl_d, sh);
  __shared__ uint32_t base_sh;
  if (tid == d) base_sh = excl_d;
  __syncthreads();
  uint32_t run = base_sh;
  // scan the row in chunks of kThreads
  for (int start = 0; start < nblocks; start += kThreads) {
    const int b = start + tid;
    const uint32_t v = b < nblocks ? hist[(int64_t)d * nblocks + b] : 0u;
    uint32_t excl;
    const uint32_t tot = block_exclusive_scan(v, excl, sh);
    if (b < nblocks) hist[(int64_t)d * nblocks + b] = run + excl;
    run += tot;
  }
}

// Stable scatter: items of a tile are visited in input order (item j of thread t is key
// base + j * 256 + t); ranks among equal digits come from wave ballots, per-wave counts
// and a running per-digit counter.  The tile is then laid out in LDS in digit order so that
// the global writes of one digit form one contiguous run.
__global__ void __launch_bounds__(kThreads) radix_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, int64_t N, int shift,
    const uint32_t* __restrict__ offsets, int nblocks, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t running[kBins];
  __shared__ uint32_t wcnt[kThreads / kWave][kBins];
  __shared__ uint32_t local_off[kBins];
  __shared__ uint32_t scan_sh[kThreads];
  __shared__ uint32_t s_key[kTile];
  __shared__ uint32_t s_val[kTile];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  running[tid] = 0;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t keys[kItems], vals[kItems], lrank[kItems];
  bool valid[kItems];
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
#pragma unroll
    for (int w = 0; w < kThreads / kWave; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t i = base + (int64_t)j * kThreads + tid;
    valid[j] = i < N;
    keys[j] = valid[j] ? keys_in[i] : 0u;
    vals[j] = valid[j] ? (vals_in ? vals_in[i] : (uint32_t)i) : 0u;
    const uint32_t digit = (keys[j] >> shift) & (kBins - 1);
    uint64_t peers = __ballot(valid[j]);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot(valid[j] && ((digit >> b) & 1u));
      peers &= ((digit >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    if (valid[j] && (peers & lt_mask) == 0ull) wcnt[wave][digit] = (uint32_t)__popcll(peers);
    __syncthreads();
    uint32_t pos = running[digit] + rank;
    for (int w = 0; w < wave; ++w) pos += wcnt[w][digit];
    lrank[j] = pos;   // rank among the tile's items with this digit
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kThreads / kWave; ++w) add += wcnt[w][tid];
    running[tid] += add;
    __syncthreads();
  }
  // running[d] is now the tile's count of digit d; local_off its exclusive scan
  uint32_t excl;
  block_exclusive_scan(running[tid], excl, scan_sh);
  local_off[tid] = excl;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    if (!valid[j]) continue;
    const uint32_t digit = (keys[j] >> shift) & (kBins - 1);
    const uint32_t lp = local_off[digit] + lrank[j];
    s_key[lp] = keys[j];
    s_val[lp] = vals[j];
  }
  __syncthreads();
  const int count = (int)((N - base) < kTile ? (N - base) : kTile);
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int t = j * kThreads + tid;
    if (t >= count) continue;
    const uint32_t key = s_key[t];
    const uint32_t digit = (key >> shift) & (kBins - 1);
    const uint32_t pos = offsets[(int64_t)digit * nblocks + blockIdx.x] + (uint32_t)t - local_off[digit];
    keys_out[pos] = key;
    vals_out[pos] = s_val[t];
  }
}

__global__ void __launch_bounds__(256) cell_starts_kernel(const uint32_t* __restrict__ keys, int64_t N,
                                                          int64_t G, uint32_t* __restrict__ starts) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > G) return;
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

fc2t2_status launch_cell_keys(const fc2t2_plan_s* pl, const void* x, int64_t N, uint32_t* keys,
                              hipStream_t s) {
  if (N == 0) return FC2T2_OK;
  const int threads = 256;
  const dim3 grid((unsigned)ceil_div(N, threads));
  const double scale = pl->n / (pl->hi - pl->lo);
  if (pl->io == FC2T2_IO_F64) {
    if (pl->dim == 2)
      hipLaunchKernelGGL((cell_keys_kernel<double, 2>), grid, dim3(threads), 0, s, (const double*)x, N, pl->lo, scale, pl->n, keys);
    else
      hipLaunchKernelGGL((cell_keys_kernel<double, 3>), grid, dim3(threads), 0, s, (const double*)x, N, pl->lo, scale, pl->n, keys);
  } else {
    if (pl->dim == 2)
      hipLaunchKernelGGL((cell_keys_kernel<float, 2>), grid, dim3(threads), 0, s, (const float*)x, N, (float)pl->lo, (float)scale, pl->n, keys);
    else
      hipLaunchKernelGGL((cell_keys_kernel<float, 3>), grid, dim3(threads), 0, s, (const float*)x, N, (float)pl->lo, (float)scale, pl->n, keys);
  }
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

size_t radix_sort_scratch_bytes(int64_t N) {
  const int64_t nblocks = ceil_div(N > 0 ? N : 1, kTile);
  return align256((size_t)N * 4) * 2 + align256((size_t)nblocks * kBins * 4) + align256(kBins * 4);
}

fc2t2_status radix_sort_pairs(const uint32_t* keys_in, uint32_t* keys_out, uint32_t* vals_out,
                              int64_t N, int key_bits, void* scratch, hipStream_t s) {
  if (N == 0) return FC2T2_OK;
  if (N > 0xFFFFFFFFll) return FC2T2_EUNSUPPORTED;
  const int nblocks = (int)ceil_div(N, kTile);
  char* p = (char*)scratch;
  uint32_t* ktmp = (uint32_t*)p;
  p += align256((size_t)N * 4);
  uint32_t* vtmp = (uint32_t*)p;
  p += align256((size_t)N * 4);
  uint32_t* hist = (uint32_t*)p;
  p += align256((size_t)nblocks * kBins * 4);
  uint32_t* totals = (uint32_t*)p;
  const int npass = (key_bits + 7) / 8;
  const uint32_t* kin = keys_in;
  const uint32_t* vin = nullptr;
  for (int pass = 0; pass < npass; ++pass) {
    const bool to_out = ((npass - 1 - pass) % 2) == 0;
    uint32_t* kout = to_out ? keys_out : ktmp;
    uint32_t* vout = to_out ? vals_out : vtmp;
    const int shift = 8 * pass;
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nblocks), dim3(kThreads), 0, s, kin, N, shift, hist, nblocks);
    hipLaunchKernelGGL(radix_digit_total_kernel, dim3(kBins), dim3(kThreads), 0, s, hist, nblocks, totals);
    hipLaunchKernelGGL(radix_offsets_kernel, dim3(kBins), dim3(kThreads), 0, s, hist, nblocks, totals);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblocks), dim3(kThreads), 0, s, kin, vin, N, shift,
                       hist, nblocks, kout, vout);
    FC2T2_LAUNCH_CHECK();
    kin = kout;
    vin = vout;
  }
  return FC2T2_OK;
}

fc2t2_status launch_cell_starts(const uint32_t* keys_sorted, int64_t N, int64_t G, uint32_t* starts,
                                hipStream_t s) {
  const int threads = 256;
  hipLaunchKernelGGL(cell_starts_kernel, dim3((unsigned)ceil_div(G + 1, threads)), dim3(threads), 0, s,
                     keys_sorted, N, G, starts);
  FC2T2_LAUNCH_CHECK();
  return FC2T2_OK;
}

}  // namespace fc2t2

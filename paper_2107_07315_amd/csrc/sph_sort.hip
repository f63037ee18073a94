// Stable LSD radix sort of (32-bit key, 32-bit value) pairs, 8-bit digits, for the cell build.
// Per pass: block histograms -> one exclusive scan over (digit, block) -> stable scatter.  The
// scatter ranks keys inside a 64-lane wave with ballot-based digit matching and orders waves and
// rounds through LDS counters, so equal keys keep their input order.
#include "sph_internal.h"

namespace {

constexpr int kBlock = 256;             // 4 waves of 64
constexpr int kItems = 16;              // keys per thread per tile
constexpr int kTile = kBlock * kItems;  // 4096 keys per block

__global__ __launch_bounds__(kBlock) void k_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                 uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kTile;
  for (int r = 0; r < kItems; ++r) {
    int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of m entries with one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan(uint32_t* __restrict__ a, int64_t m) {
  __shared__ uint32_t part[1024];
  int64_t per = (m + 1023) / 1024;
  int64_t lo = (int64_t)threadIdx.x * per;
  int64_t hi = lo + per < m ? lo + per : m;
  uint32_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += a[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int64_t i = lo; i < hi; ++i) {
    uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter(const uint32_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ vals, int64_t n,
                                                    int shift, const uint32_t* __restrict__ offs,
                                                    int nblocks, uint32_t* __restrict__ keys_out,
                                                    uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wave_cnt[4][256];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  base[threadIdx.x] = offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
  for (int w = 0; w < 4; ++w) wave_cnt[w][threadIdx.x] = 0;
  __syncthreads();
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t tile0 = (int64_t)blockIdx.x * kTile;
  for (int r = 0; r < kItems; ++r) {
    int64_t i = tile0 + (int64_t)r * kBlock + threadIdx.x;
    bool valid = i < n;
    uint32_t k = valid ? keys[i] : 0u;
    uint32_t v = valid ? vals[i] : 0u;
    uint32_t d = (k >> shift) & 255u;
    // lanes holding the same digit
    unsigned long long match = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      unsigned long long bb = __ballot((d >> b) & 1u);
      match &= ((d >> b) & 1u) ? bb : ~bb;
    }
    uint32_t rank = (uint32_t)__popcll(match & lt);
    bool leader = valid && ((match & lt) == 0ull);
    if (leader) wave_cnt[wave][d] = (uint32_t)__popcll(match);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wave_cnt[w][d];
      keys_out[pos] = k;
      vals_out[pos] = v;
    }
    __syncthreads();
    // advance the per-digit base by this round's total and clear the wave counters
    uint32_t tot = 0;
    for (int w = 0; w < 4; ++w) {
      tot += wave_cnt[w][threadIdx.x];
      wave_cnt[w][threadIdx.x] = 0;
    }
    base[threadIdx.x] += tot;
    __syncthreads();
  }
}

}  // namespace

// Sorts keys[0..n) ascending, carrying vals; on return keys/vals hold the sorted pairs.
sph_status sph_sort_pairs(sph_ctx* c, uint32_t* keys, uint32_t* vals, int64_t n) {
  if (n <= 1) return SPH_OK;
  int nblocks = (int)((n + kTile - 1) / kTile);
  if (nblocks > c->sort.max_blocks) return SPH_E_ARG;
  uint32_t *ka = keys, *va = vals, *kb = c->sort.keys_alt, *vb = c->sort.vals_alt;
  for (int shift = 0; shift < 32; shift += 8) {
    hipLaunchKernelGGL(k_hist, dim3(nblocks), dim3(kBlock), 0, c->stream, ka, n, shift, c->sort.hist,
                       nblocks);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, c->stream, c->sort.hist, (int64_t)256 * nblocks);
    hipLaunchKernelGGL(k_scatter, dim3(nblocks), dim3(kBlock), 0, c->stream, ka, va, n, shift,
                       c->sort.hist, nblocks, kb, vb);
    uint32_t* t = ka; ka = kb; kb = t;
    t = va; va = vb; vb = t;
  }
  // four passes: the result is back in the caller's buffers
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

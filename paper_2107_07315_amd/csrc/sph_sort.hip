// Stable LSD radix sort of (32-bit key, 32-bit value) pairs, 8-bit digits, for the cell build.
// Per pass: block histograms -> exclusive scan over (digit, block) in two small kernels ->
// stable scatter.  The
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

// Block-wide exclusive scan of one value per thread (256 threads = 4 waves).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t o = __shfl_up(inc, off, 64);
    if (lane >= off) inc += o;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();
  return before + inc - v;
}

// Row scan: block d turns hist[d][0..nblocks) into exclusive prefixes and stores the row total.
__global__ __launch_bounds__(256) void k_scan_rows(uint32_t* __restrict__ hist, int nblocks,
                                                   uint32_t* __restrict__ rowtot) {
  __shared__ uint32_t wsum[4];
  uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
  uint32_t carry = 0;
  for (int base = 0; base < nblocks; base += 256) {
    int i = base + threadIdx.x;
    uint32_t v = i < nblocks ? row[i] : 0u;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(v, wsum, tot);
    if (i < nblocks) row[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) rowtot[blockIdx.x] = carry;
}

// Exclusive scan of the 256 row totals (digit offsets).
__global__ __launch_bounds__(256) void k_scan_totals(uint32_t* __restrict__ rowtot) {
  __shared__ uint32_t wsum[4];
  uint32_t tot;
  uint32_t v = rowtot[threadIdx.x];
  uint32_t ex = block_exclusive_scan(v, wsum, tot);
  rowtot[threadIdx.x] = ex;
}

__global__ __launch_bounds__(kBlock) void k_scatter(const uint32_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ vals, int64_t n,
                                                    int shift, const uint32_t* __restrict__ offs,
                                                    const uint32_t* __restrict__ digit_off,
                                                    int nblocks, uint32_t* __restrict__ keys_out,
                                                    uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wave_cnt[4][256];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  base[threadIdx.x] = digit_off[threadIdx.x] + offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
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

// Generic exclusive scan, 1024 elements per block: block sums -> scan of the sums -> apply.
__global__ __launch_bounds__(256) void k_scan_bsum(const uint32_t* __restrict__ in, int64_t n,
                                                   uint32_t* __restrict__ bsum) {
  __shared__ uint32_t wsum[4];
  int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  uint32_t v = 0;
  for (int k = 0; k < 4; ++k)
    if (base + k < n) v += in[base + k];
  uint32_t tot;
  block_exclusive_scan(v, wsum, tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ in, int64_t n,
                                                    const uint32_t* __restrict__ boff, uint32_t* __restrict__ out) {
  __shared__ uint32_t wsum[4];
  int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  uint32_t v[4], s = 0;
  for (int k = 0; k < 4; ++k) {
    v[k] = base + k < n ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t ex = block_exclusive_scan(s, wsum, tot) + boff[blockIdx.x];
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
}

}  // namespace

// out = exclusive prefix sum of in[0..n); *total (device) = sum.  in and out may alias.
sph_status sph_scan_u32(sph_ctx* c, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total) {
  if (n <= 0) return SPH_OK;
  const int64_t nb = (n + 1023) / 1024;
  if (nb > c->sort.scan_cap) return SPH_E_ARG;
  hipLaunchKernelGGL(k_scan_bsum, dim3((unsigned)nb), dim3(256), 0, c->stream, in, n, c->sort.scan_bsum);
  hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(256), 0, c->stream, c->sort.scan_bsum, (int)nb, total);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, c->stream, in, n, c->sort.scan_bsum, out);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

// Sorts keys[0..n) ascending, carrying vals; on return keys/vals hold the sorted pairs.
sph_status sph_sort_pairs(sph_ctx* c, uint32_t* keys, uint32_t* vals, int64_t n) {
  if (n <= 1) return SPH_OK;
  int nblocks = (int)((n + kTile - 1) / kTile);
  if (nblocks > c->sort.max_blocks) return SPH_E_ARG;
  uint32_t *ka = keys, *va = vals, *kb = c->sort.keys_alt, *vb = c->sort.vals_alt;
  for (int shift = 0; shift < 32; shift += 8) {
    hipLaunchKernelGGL(k_hist, dim3(nblocks), dim3(kBlock), 0, c->stream, ka, n, shift, c->sort.hist,
                       nblocks);
    hipLaunchKernelGGL(k_scan_rows, dim3(256), dim3(256), 0, c->stream, c->sort.hist, nblocks, c->sort.rowtot);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(256), 0, c->stream, c->sort.rowtot);
    hipLaunchKernelGGL(k_scatter, dim3(nblocks), dim3(kBlock), 0, c->stream, ka, va, n, shift,
                       c->sort.hist, c->sort.rowtot, nblocks, kb, vb);
    uint32_t* t = ka; ka = kb; kb = t;
    t = va; va = vb; vb = t;
  }
  // four passes: the result is back in the caller's buffers
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

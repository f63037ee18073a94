// Cell build and neighbour lists.
//
// The paper's sums run over "particles within the support radius" (section "Solid SPH
// Equations"); with support h_a + h_b the neighbour set is
//   N(a) = { b != a : |x_a - x_b|^2 < (h_a + h_b)^2 }.
// Smoothing lengths in a star vary about tenfold from the centre to the surface, so particles
// are binned into up to four levels by h (factor 2 per level), each with its own uniform grid
// (cell size 2 hmax_l / cell_div).  A particle searches every level l within h_a + hmax_l and
// skips cells whose box lies farther away.  Cells are addressed by Morton codes so that the
// sorted particle order is spatially compact.  The list build writes exact FP64 lists that all
// later passes read; the lists are interleaved by wavefront so that lane a of a wave reading its
// k-th neighbour touches one contiguous 256-byte segment.
#include "sph_internal.h"

namespace {

constexpr int kB = 256;

__global__ void k_grid_reset(GridInfo* g) {
  for (int d = 0; d < 3; ++d) { g->enc_lo[d] = ~0ull; g->enc_hi[d] = 0ull; }
  g->enc_hmin = ~0ull;
  g->enc_hmax = 0ull;
  for (int l = 0; l < SPH_MAX_LEV; ++l) g->hlev_bits[l] = 0ull;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Bounding box (positions relative to their star centre) and the h range.
__global__ __launch_bounds__(kB) void k_bounds(const double4* __restrict__ pos4, int64_t n, GridInfo* g) {
  unsigned long long lo[3] = {~0ull, ~0ull, ~0ull}, hi[3] = {0, 0, 0}, hmn = ~0ull, hmx = 0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n;
       a += (int64_t)gridDim.x * blockDim.x) {
    double4 p = pos4[a];
    double q[3] = {p.x, p.y, p.z};
    for (int d = 0; d < 3; ++d) {
      unsigned long long e = enc_double(q[d]);
      lo[d] = e < lo[d] ? e : lo[d];
      hi[d] = e > hi[d] ? e : hi[d];
    }
    unsigned long long e = enc_double(p.w);
    hmn = e < hmn ? e : hmn;
    hmx = e > hmx ? e : hmx;
  }
  for (int d = 0; d < 3; ++d) { lo[d] = wave_min_u64(lo[d]); hi[d] = wave_max_u64(hi[d]); }
  hmn = wave_min_u64(hmn);
  hmx = wave_max_u64(hmx);
  if ((threadIdx.x & 63) == 0) {
    for (int d = 0; d < 3; ++d) { atomicMin(&g->enc_lo[d], lo[d]); atomicMax(&g->enc_hi[d], hi[d]); }
    atomicMin(&g->enc_hmin, hmn);
    atomicMax(&g->enc_hmax, hmx);
  }
}

__global__ void k_grid_setup1(GridInfo* g, int periodic, double box, DevStatus* st) {
  g->periodic = periodic;
  g->box = box;
  for (int d = 0; d < 3; ++d) g->lo[d] = periodic ? 0.0 : dec_double(g->enc_lo[d]);
  g->hmin = dec_double(g->enc_hmin);
  g->hmax = dec_double(g->enc_hmax);
  // minimum image needs h_a + h_b < box / 2 for every pair; non-positive h is invalid
  if ((periodic && !(2.0 * g->hmax < 0.5 * box)) || !(g->hmin > 0.0)) latch_error(st, SPH_E_ARG, -1);
  int L = 1;
  while (L < SPH_MAX_LEV && g->hmax >= g->hmin * (double)(1 << L)) ++L;
  g->nlev = L;
}

__global__ __launch_bounds__(kB) void k_level_hmax(const double4* __restrict__ pos4, int64_t n, GridInfo* g) {
  __shared__ unsigned long long m[SPH_MAX_LEV];
  if (threadIdx.x < SPH_MAX_LEV) m[threadIdx.x] = 0ull;
  __syncthreads();
  GridInfo G = *g;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n;
       a += (int64_t)gridDim.x * blockDim.x) {
    double h = pos4[a].w;
    int l = particle_level(h, G);
    atomicMax(&m[l], (unsigned long long)__double_as_longlong(h));
  }
  __syncthreads();
  if (threadIdx.x < SPH_MAX_LEV && m[threadIdx.x]) atomicMax(&g->hlev_bits[threadIdx.x], m[threadIdx.x]);
}

__global__ void k_grid_setup2(GridInfo* g, int cell_div, int64_t max_cells, DevStatus* st) {
  double hi[3];
  for (int d = 0; d < 3; ++d) hi[d] = g->periodic ? g->box : dec_double(g->enc_hi[d]);
  double grow = 1.0;
  for (int attempt = 0; attempt < 64; ++attempt) {
    uint64_t total = 0;
    bool ok = true;
    for (int l = 0; l < g->nlev; ++l) {
      double hl = __longlong_as_double((long long)g->hlev_bits[l]);
      if (!(hl > 0.0)) hl = g->hmin * (double)(1 << l);
      g->hlev[l] = hl;
      double c = 2.0 * hl / (double)cell_div * grow;
      int bmax = 0;
      for (int d = 0; d < 3; ++d) {
        int dim;
        if (g->periodic) {
          dim = (int)floor(g->box / c);
          if (dim < 1) dim = 1;
        } else {
          double ext = hi[d] - g->lo[d];
          dim = (int)floor(ext / c) + 1;
        }
        if (dim > 1024) ok = false;
        g->dims[l][d] = dim;
        int b = 0;
        while ((1 << b) < dim) ++b;
        bmax = b > bmax ? b : bmax;
      }
      g->cell[l] = g->periodic ? 0.0 : c;   // periodic: per-dimension sizes below
      g->bits[l] = bmax;
      g->base[l] = (uint32_t)total;
      total += 1ull << (3 * bmax);
    }
    if (ok && total <= (uint64_t)max_cells) {
      g->base[g->nlev] = (uint32_t)total;
      if (g->periodic)
        for (int l = 0; l < g->nlev; ++l) g->cell[l] = g->box / (double)g->dims[l][0];
      return;
    }
    grow *= 1.25;
  }
  // No grid fits: fall back to a single cell (every key 0, memory-safe) and report the error.
  latch_error(st, SPH_E_ARG, -1);
  g->nlev = 1;
  g->cell[0] = 1e300;
  g->dims[0][0] = g->dims[0][1] = g->dims[0][2] = 1;
  g->bits[0] = 0;
  g->base[0] = 0;
  g->base[1] = 1;
}

__device__ __forceinline__ int cell_coord(double x, double lo, double c, int dim) {
  int k = (int)floor((x - lo) / c);
  return k < 0 ? 0 : (k > dim - 1 ? dim - 1 : k);
}

__global__ __launch_bounds__(kB) void k_keys(const double4* __restrict__ pos4, int64_t n,
                                             const GridInfo* __restrict__ gp, uint32_t* __restrict__ keys,
                                             uint32_t* __restrict__ vals) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const GridInfo& g = *gp;
  double4 p = pos4[a];
  int l = particle_level(p.w, g);
  double c = g.cell[l];
  uint32_t ix = (uint32_t)cell_coord(p.x, g.lo[0], c, g.dims[l][0]);
  uint32_t iy = (uint32_t)cell_coord(p.y, g.lo[1], c, g.dims[l][1]);
  uint32_t iz = (uint32_t)cell_coord(p.z, g.lo[2], c, g.dims[l][2]);
  keys[a] = g.base[l] + (spread3(ix) | (spread3(iy) << 1) | (spread3(iz) << 2));
  vals[a] = (uint32_t)a;
}

__global__ __launch_bounds__(kB) void k_cell_ranges(const uint32_t* __restrict__ keys, int64_t n,
                                                    int32_t* __restrict__ cstart, int32_t* __restrict__ cend) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t k = keys[i];
  if (i == 0 || keys[i - 1] != k) cstart[k] = (int32_t)i;
  if (i == n - 1 || keys[i + 1] != k) cend[k] = (int32_t)(i + 1);
}

template <typename T>
__global__ __launch_bounds__(kB) void k_gather(const T* __restrict__ src, const uint32_t* __restrict__ perm,
                                               int64_t n, T* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

__global__ __launch_bounds__(kB) void k_identity(uint32_t* __restrict__ v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (uint32_t)i;
}

// pos4: absolute position and h (FP64 pair passes); pos4f: position relative to the
// particle's star centre and h (FP32 pair passes keep full precision near each star).
__global__ __launch_bounds__(kB) void k_pack_pos(const double* __restrict__ x, const double* __restrict__ y,
                                                 const double* __restrict__ z, const double* __restrict__ h,
                                                 const int32_t* __restrict__ star,
                                                 const StarInfo* __restrict__ stars, int64_t n,
                                                 double4* __restrict__ pos4, float4* __restrict__ pos4f) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double cx = 0, cy = 0, cz = 0;
  if (star && stars) {
    StarInfo s = stars[star[a]];
    cx = s.cx; cy = s.cy; cz = s.cz;
  }
  pos4[a] = make_double4(x[a], y[a], z[a], h[a]);
  if (pos4f) pos4f[a] = make_float4((float)(x[a] - cx), (float)(y[a] - cy), (float)(z[a] - cz), (float)h[a]);
}

// Ensemble stars occupy disjoint regions of one coordinate frame: the search runs in that
// frame, so the positions used for binning and testing are the absolute ones.
__global__ __launch_bounds__(kB) void k_build_lists(const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ z, const double* __restrict__ h,
                                                    int64_t n, const GridInfo* __restrict__ gp,
                                                    const uint32_t* __restrict__ skeys,
                                                    const uint32_t* __restrict__ perm, int identity,
                                                    const int32_t* __restrict__ cstart,
                                                    const int32_t* __restrict__ cend, int cap,
                                                    int32_t* __restrict__ nbr, int32_t* __restrict__ count,
                                                    DevStatus* status) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const GridInfo& g = *gp;
  const double xa = x[a], ya = y[a], za = z[a], ha = h[a];
  int32_t* out = nbr + ((a >> 6) * (int64_t)cap) * 64 + (a & 63);
  int cnt = 0;
  const int periodic = g.periodic;
  const double box = g.box;
  for (int l = 0; l < g.nlev; ++l) {
    const double c = g.cell[l];
    const double R = (ha + g.hlev[l]) * (1.0 + 1e-9);
    const double R2 = R * R;
    int lo3[3], hi3[3];
    bool wrap[3];
    const double q[3] = {xa, ya, za};
    for (int d = 0; d < 3; ++d) {
      int dim = g.dims[l][d];
      int l0 = (int)floor((q[d] - R - g.lo[d]) / c);
      int h0 = (int)floor((q[d] + R - g.lo[d]) / c);
      wrap[d] = false;
      if (periodic) {
        if (h0 - l0 + 1 >= dim) { l0 = 0; h0 = dim - 1; }
        else wrap[d] = true;
      } else {
        l0 = l0 < 0 ? 0 : l0;
        h0 = h0 > dim - 1 ? dim - 1 : h0;
      }
      lo3[d] = l0;
      hi3[d] = h0;
    }
    const uint32_t base = g.base[l];
    for (int kz = lo3[2]; kz <= hi3[2]; ++kz) {
      double dz = 0.0;
      if (!periodic || wrap[2]) {
        double b0 = g.lo[2] + kz * c, b1 = b0 + c;
        dz = za < b0 ? b0 - za : (za > b1 ? za - b1 : 0.0);
      }
      int cz = kz;
      if (wrap[2]) cz = (kz % g.dims[l][2] + g.dims[l][2]) % g.dims[l][2];
      const uint32_t mz = spread3((uint32_t)cz) << 2;
      for (int ky = lo3[1]; ky <= hi3[1]; ++ky) {
        double dy = 0.0;
        if (!periodic || wrap[1]) {
          double b0 = g.lo[1] + ky * c, b1 = b0 + c;
          dy = ya < b0 ? b0 - ya : (ya > b1 ? ya - b1 : 0.0);
        }
        if (dz * dz + dy * dy >= R2) continue;
        int cy = ky;
        if (wrap[1]) cy = (ky % g.dims[l][1] + g.dims[l][1]) % g.dims[l][1];
        const uint32_t myz = mz | (spread3((uint32_t)cy) << 1);
        for (int kx = lo3[0]; kx <= hi3[0]; ++kx) {
          double dx = 0.0;
          if (!periodic || wrap[0]) {
            double b0 = g.lo[0] + kx * c, b1 = b0 + c;
            dx = xa < b0 ? b0 - xa : (xa > b1 ? xa - b1 : 0.0);
          }
          if (dz * dz + dy * dy + dx * dx >= R2) continue;
          int cx = kx;
          if (wrap[0]) cx = (kx % g.dims[l][0] + g.dims[l][0]) % g.dims[l][0];
          const uint32_t key = base + (myz | spread3((uint32_t)cx));
          int32_t s = cstart[key];
          if (s < 0 || s >= n || skeys[s] != key) continue;
          int32_t e = cend[key];
          for (int32_t p = s; p < e; ++p) {
            int64_t b = identity ? p : (int64_t)perm[p];
            if (b == a) continue;
            double ddx = min_image(xa - x[b], periodic, box);
            double ddy = min_image(ya - y[b], periodic, box);
            double ddz = min_image(za - z[b], periodic, box);
            if (!neighbour_test(ddx, ddy, ddz, ha, h[b])) continue;
            if (cnt < cap) out[(int64_t)cnt * 64] = (int32_t)b;
            ++cnt;
          }
        }
      }
    }
  }
  count[a] = cnt < cap ? cnt : cap;
  if (cnt > cap) latch_error(status, SPH_E_NGB_CAPACITY, (int)a);
}

template <typename T>
sph_status permute_array(sph_ctx* c, T* arr, int64_t n) {
  if (!arr) return SPH_OK;
  T* tmp = reinterpret_cast<T*>(c->tmp);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gather<T>), dim3(grid_for(n, kB)), dim3(kB), 0, c->stream, arr,
                     c->vals, n, tmp);
  HIP_TRY(hipMemcpyAsync(arr, tmp, sizeof(T) * n, hipMemcpyDeviceToDevice, c->stream));
  return SPH_OK;
}

}  // namespace

// Bin particles into the multi-level grid and build the neighbour lists.  With permute, every
// particle array of the state (and the half-step copies) is reordered into cell order first.
sph_status sph_rebin(sph_ctx* c, sph_state* st, bool permute) {
  const int64_t n = st->n;
  hipStream_t s = c->stream;
  const unsigned nb = grid_for(n, kB);
  unsigned nred = nb < 1024 ? nb : 1024;
  // absolute positions for binning (ensemble stars are placed apart in one frame)
  hipLaunchKernelGGL(k_pack_pos, dim3(nb), dim3(kB), 0, s, st->x, st->y, st->z, st->h,
                     (const int32_t*)nullptr, (const StarInfo*)nullptr, n, c->pos4, (float4*)nullptr);
  hipLaunchKernelGGL(k_grid_reset, dim3(1), dim3(1), 0, s, c->grid);
  hipLaunchKernelGGL(k_bounds, dim3(nred), dim3(kB), 0, s, c->pos4, n, c->grid);
  hipLaunchKernelGGL(k_grid_setup1, dim3(1), dim3(1), 0, s, c->grid, c->p.periodic, c->p.box, c->status);
  hipLaunchKernelGGL(k_level_hmax, dim3(nred), dim3(kB), 0, s, c->pos4, n, c->grid);
  hipLaunchKernelGGL(k_grid_setup2, dim3(1), dim3(1), 0, s, c->grid, c->p.cell_div > 0 ? c->p.cell_div : 2,
                     c->max_cells, c->status);
  hipLaunchKernelGGL(k_keys, dim3(nb), dim3(kB), 0, s, c->pos4, n, c->grid, c->keys, c->vals);
  sph_status e = sph_sort_pairs(c, c->keys, c->vals, n);
  if (e) return e;
  if (permute) {
    double* d64[] = {st->x, st->y, st->z, st->vx, st->vy, st->vz, st->u, st->h, st->D, st->rho,
                     st->P, st->cs, st->ax, st->ay, st->az, st->dudt};
    for (double* a : d64)
      if ((e = permute_array(c, a, n))) return e;
    for (int k = 0; k < 6; ++k) {
      if ((e = permute_array(c, st->S + k * n, n))) return e;
      if ((e = permute_array(c, st->dSdt + k * n, n))) return e;
    }
    for (int k = 0; k < 10; ++k)
      if ((e = permute_array(c, c->half + (int64_t)k * c->capacity, n))) return e;
    if ((e = permute_array(c, st->type, n))) return e;
    if ((e = permute_array(c, st->broken, n))) return e;
    if ((e = permute_array(c, st->id, n))) return e;
    if ((e = permute_array(c, st->star, n))) return e;
    hipLaunchKernelGGL(k_identity, dim3(nb), dim3(kB), 0, s, c->vals, n);
    c->identity_perm = 1;
  } else {
    c->identity_perm = 0;
  }
  hipLaunchKernelGGL(k_cell_ranges, dim3(nb), dim3(kB), 0, s, c->keys, n, c->cell_start, c->cell_end);
  hipLaunchKernelGGL(k_build_lists, dim3(nb), dim3(kB), 0, s, st->x, st->y, st->z, st->h, n, c->grid,
                     c->keys, c->vals, c->identity_perm, c->cell_start, c->cell_end, c->cap, c->nbr,
                     c->nbr_count, c->status);
  HIP_TRY(hipGetLastError());
  return launch_pack(c, st);
}

// Pack the position records the pair passes read, in the current particle order.
sph_status launch_pack(sph_ctx* c, sph_state* st) {
  const int64_t n = st->n;
  hipLaunchKernelGGL(k_pack_pos, dim3(grid_for(n, kB)), dim3(kB), 0, c->stream, st->x, st->y, st->z, st->h,
                     st->star, c->stars, n, c->pos4, c->p.precision == SPH_FP32 ? c->pos4f : nullptr);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

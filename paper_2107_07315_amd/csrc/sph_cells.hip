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
// later passes read, grouped in tiles of 64 particles (see k_build_tiles).
#include <stddef.h>
#include <string.h>

#include <mutex>

#include "sph_internal.h"

namespace {

constexpr int kB = 256;

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

// Bounding box and h range: one partial per block (8 encoded values), reduced in set-up.
__global__ __launch_bounds__(kB) void k_bounds(const double4* __restrict__ pos4, int64_t n,
                                               unsigned long long* __restrict__ partial) {
  __shared__ unsigned long long red[4][8];
  unsigned long long v[8] = {~0ull, ~0ull, ~0ull, 0ull, 0ull, 0ull, ~0ull, 0ull};  // lo xyz, hi xyz, hmin, hmax
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n;
       a += (int64_t)gridDim.x * blockDim.x) {
    double4 p = pos4[a];
    double q[3] = {p.x, p.y, p.z};
    for (int d = 0; d < 3; ++d) {
      unsigned long long e = enc_double(q[d]);
      v[d] = e < v[d] ? e : v[d];
      v[3 + d] = e > v[3 + d] ? e : v[3 + d];
    }
    unsigned long long e = enc_double(p.w);
    v[6] = e < v[6] ? e : v[6];
    v[7] = e > v[7] ? e : v[7];
  }
  for (int k = 0; k < 8; ++k) {
    bool mx = (k >= 3 && k < 6) || k == 7;
    v[k] = mx ? wave_max_u64(v[k]) : wave_min_u64(v[k]);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 8; ++k) red[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 8) {
    int k = threadIdx.x;
    bool mx = (k >= 3 && k < 6) || k == 7;
    unsigned long long r = red[0][k];
    for (int w = 1; w < 4; ++w) r = mx ? (red[w][k] > r ? red[w][k] : r) : (red[w][k] < r ? red[w][k] : r);
    partial[(int64_t)blockIdx.x * 8 + k] = r;
  }
}

__global__ __launch_bounds__(64) void k_grid_setup1(GridInfo* g, const unsigned long long* __restrict__ partial,
                                                    int nblocks, int periodic, double box, double skin,
                                                    DevStatus* st) {
  unsigned long long v[8] = {~0ull, ~0ull, ~0ull, 0ull, 0ull, 0ull, ~0ull, 0ull};
  for (int b = threadIdx.x; b < nblocks; b += 64)
    for (int k = 0; k < 8; ++k) {
      unsigned long long e = partial[(int64_t)b * 8 + k];
      bool mx = (k >= 3 && k < 6) || k == 7;
      v[k] = mx ? (e > v[k] ? e : v[k]) : (e < v[k] ? e : v[k]);
    }
  for (int k = 0; k < 8; ++k) {
    bool mx = (k >= 3 && k < 6) || k == 7;
    v[k] = mx ? wave_max_u64(v[k]) : wave_min_u64(v[k]);
  }
  if (threadIdx.x != 0) return;
  for (int d = 0; d < 3; ++d) { g->enc_lo[d] = v[d]; g->enc_hi[d] = v[3 + d]; }
  g->enc_hmin = v[6];
  g->enc_hmax = v[7];
  for (int l = 0; l < SPH_MAX_LEV; ++l) {
    g->hlev_bits[l] = 0ull;
    for (int d = 0; d < 3; ++d) {
      g->lev_lo[l][d] = ~0ull;
      g->lev_hi[l][d] = 0ull;
    }
  }
  g->periodic = periodic;
  g->box = box;
  for (int d = 0; d < 3; ++d) g->lo[d] = periodic ? 0.0 : dec_double(g->enc_lo[d]);
  g->hmin = dec_double(g->enc_hmin);
  g->hmax = dec_double(g->enc_hmax);
  // minimum image needs h_a + h_b < box / 2 for every pair; non-positive h is invalid
  if ((periodic && !(2.0 * g->hmax < 0.5 * box)) || !(g->hmin > 0.0)) latch_error(st, SPH_E_ARG, -1);
  // effective skin: the widened support must stay below half a periodic box
  double s = skin;
  if (periodic) {
    const double smax = 0.5 * box / (2.0 * g->hmax) * (1.0 - 1e-9) - 1.0;
    s = s < smax ? s : smax;
  }
  g->skin = s >= 1e-4 ? s : 0.0;
  int L = 1;
  while (L < SPH_MAX_LEV && g->hmax >= g->hmin * (double)(1 << L)) ++L;
  g->nlev = L;
}

// Per level: largest h and the bounding box of the level's particles (a tile's search at a level
// is clipped to that box, which keeps large-h tiles from enumerating the empty fine cells of
// levels that only occupy the core).
__global__ __launch_bounds__(kB) void k_level_hmax(const double4* __restrict__ pos4, int64_t n, GridInfo* g) {
  __shared__ unsigned long long m[SPH_MAX_LEV];
  __shared__ unsigned long long blo[SPH_MAX_LEV][3], bhi[SPH_MAX_LEV][3];
  if (threadIdx.x < SPH_MAX_LEV) {
    m[threadIdx.x] = 0ull;
    for (int d = 0; d < 3; ++d) {
      blo[threadIdx.x][d] = ~0ull;
      bhi[threadIdx.x][d] = 0ull;
    }
  }
  __syncthreads();
  GridInfo G = *g;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n;
       a += (int64_t)gridDim.x * blockDim.x) {
    const double4 q = pos4[a];
    const int l = particle_level(q.w, G);
    atomicMax(&m[l], (unsigned long long)__double_as_longlong(q.w));
    const double c[3] = {q.x, q.y, q.z};
    for (int d = 0; d < 3; ++d) {
      const unsigned long long e = enc_double(c[d]);
      atomicMin(&blo[l][d], e);
      atomicMax(&bhi[l][d], e);
    }
  }
  __syncthreads();
  if (threadIdx.x < SPH_MAX_LEV && m[threadIdx.x]) {
    const int l = threadIdx.x;
    atomicMax(&g->hlev_bits[l], m[l]);
    for (int d = 0; d < 3; ++d) {
      atomicMin(&g->lev_lo[l][d], blo[l][d]);
      atomicMax(&g->lev_hi[l][d], bhi[l][d]);
    }
  }
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

// Clears the cells in use (base[nlev] entries) to empty ranges.
__global__ __launch_bounds__(kB) void k_cells_clear(int2* __restrict__ se, const GridInfo* __restrict__ gp) {
  const int64_t total = gp->base[gp->nlev];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    se[i] = make_int2(0, 0);
}

__global__ __launch_bounds__(kB) void k_cell_ranges(const uint32_t* __restrict__ keys, int64_t n,
                                                    int2* __restrict__ se) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t k = keys[i];
  if (i == 0 || keys[i - 1] != k) se[k].x = (int32_t)i;
  if (i == n - 1 || keys[i + 1] != k) se[k].y = (int32_t)(i + 1);
}

template <typename T>
__global__ __launch_bounds__(kB) void k_gather(const T* __restrict__ src, const uint32_t* __restrict__ perm,
                                               int64_t n, T* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

// Several arrays of 8-byte elements at once: dst[k][i] = src[k][perm[i]] (gather) or
// dst[k][i] = src[k][i] (copy) for k < na, the permutation read once per element.
constexpr int kPermBatch = 16;
struct PermBatch {
  const double* src[kPermBatch];
  double* dst[kPermBatch];
  int na;
};
template <bool GATHER>
__global__ __launch_bounds__(kB) void k_permute_batch(PermBatch B, const uint32_t* __restrict__ perm, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = GATHER ? (int64_t)perm[i] : i;
  for (int k = 0; k < B.na; ++k) B.dst[k][i] = B.src[k][j];
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
  if (pos4f) pos4f[a] = make_float4((float)(x[a] - cx), (float)(y[a] - cy), (float)(z[a] - cz), (float)(0.5 * h[a]));
}

// Global Morton key of a 1024^3 grid over the bounding box: the particle arrays are kept in this
// order (re-sorted every few steps), so any 64 consecutive particles form a compact tile whatever
// the local density; the per-level cell tables index the particles through a permutation.
__global__ __launch_bounds__(kB) void k_gkeys(const double4* __restrict__ pos4, int64_t n,
                                              const GridInfo* __restrict__ gp, uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ vals) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const GridInfo& g = *gp;
  double ext = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double e = g.periodic ? g.box : dec_double(g.enc_hi[d]) - g.lo[d];
    ext = e > ext ? e : ext;
  }
  const double sc = ext > 0.0 ? 1024.0 / ext : 0.0;
  const double4 p = pos4[a];
  uint32_t k3[3];
  const double q[3] = {p.x, p.y, p.z};
  for (int d = 0; d < 3; ++d) {
    int k = (int)floor((q[d] - g.lo[d]) * sc);
    k3[d] = (uint32_t)(k < 0 ? 0 : (k > 1023 ? 1023 : k));
  }
  keys[a] = spread3(k3[0]) | (spread3(k3[1]) << 1) | (spread3(k3[2]) << 2);
  vals[a] = (uint32_t)a;
}

// Tile table, rebuilt at every full re-sort (particles keep their array order in between).  A
// tile starts at every multiple of 64 and wherever the Morton curve jumps: if consecutive keys first
// differ in octree level k, the two particles only share a block of 2^(k+1) fine cells, so a tile
// that spans the boundary could be that large.  Cutting where 2^(k+1) fine cells exceed 4 h keeps
// every tile inside a region about 4 smoothing lengths across, in dense and sparse parts alike
// (the factor is the tile_cut parameter).
__global__ __launch_bounds__(kB) void k_tile_flags(const uint32_t* __restrict__ gkeys, const double4* __restrict__ pos4,
                                                   int64_t n, const GridInfo* __restrict__ gp, double cut,
                                                   uint32_t* __restrict__ flag) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  bool start = (p & 63) == 0;
  if (!start) {
    const GridInfo& g = *gp;
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double e = g.periodic ? g.box : dec_double(g.enc_hi[d]) - g.lo[d];
      ext = e > ext ? e : ext;
    }
    const double fine = ext / 1024.0;
    const uint32_t x = gkeys[p] ^ gkeys[p - 1];
    const int lvl = x ? (31 - __clz(x)) / 3 : -1;
    start = lvl >= 0 && (double)(2 << lvl) * fine > cut * pos4[p].w;
  }
  flag[p] = start ? 1u : 0u;
}

// Work list of the stress pass: the tiles that hold a particle of type 1 (crust).  Breaking only
// removes particles from the stressed set and type never changes, so the list stays a superset
// until the next build.  Every other particle is of type 0, carries no deviatoric stress and has
// zero stress rates, which k_zero_fluid_rates sets once per build (the kicks then skip the stress
// arrays of type-0 particles; the rates of type-1 particles are written by the pass).
__global__ __launch_bounds__(kB) void k_stress_flags(const GridInfo* __restrict__ gp, int64_t cap_tiles,
                                                     const int32_t* __restrict__ tile_start,
                                                     const int32_t* __restrict__ tile_cnt,
                                                     const int8_t* __restrict__ type, uint32_t* __restrict__ flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cap_tiles) return;
  uint32_t f = 0u;
  if (t < (int64_t)gp->ntiles) {
    const int32_t s = tile_start[t], e = s + tile_cnt[t];
    for (int32_t q = s; q < e; ++q) f |= type[q] == 1 ? 1u : 0u;
  }
  flag[t] = f;
}
// Per tile: whether one of its particles or of its union members is of type 1 (one wave a tile).
__global__ __launch_bounds__(64) void k_tile_union_type(const GridInfo* __restrict__ gp, const int32_t* __restrict__ tile_start,
                                                       const int32_t* __restrict__ tile_cnt,
                                                       const uint32_t* __restrict__ tile_uoff,
                                                       const int32_t* __restrict__ tile_usize,
                                                       const int32_t* __restrict__ tile_u,
                                                       const int8_t* __restrict__ type, uint32_t* __restrict__ flag) {
  const int lane = threadIdx.x;
  const int64_t nt = gp->ntiles;
  for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    bool f = lane < tile_cnt[t] && type[tile_start[t] + lane] == 1;
    const int32_t us = tile_usize[t];
    const int32_t* U = tile_u + tile_uoff[t];
    for (int j = lane; j < us && !f; j += 64) f = type[U[j]] == 1;
    const unsigned long long m = __ballot(f);
    if (lane == 0) flag[t] = m ? 1u : 0u;
  }
}
__global__ __launch_bounds__(kB) void k_stress_list(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ idx,
                                                    int64_t cap_tiles, int32_t* __restrict__ list) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cap_tiles && flag[t]) list[idx[t]] = (int32_t)t;
}
__global__ __launch_bounds__(kB) void k_zero_fluid_rates(const int8_t* __restrict__ type, int64_t n,
                                                         double* __restrict__ S, double* __restrict__ dSdt,
                                                         double* __restrict__ sdot) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n || type[a] == 1) return;
  for (int c = 0; c < 6; ++c) {
    S[c * n + a] = 0.0;   // fluid (type 0) carries no deviatoric stress
    dSdt[c * n + a] = 0.0;
  }
  sdot[a] = 0.0;
}

__global__ __launch_bounds__(kB) void k_tile_fill(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ idx,
                                                  int64_t n, int32_t* __restrict__ tile_start) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (flag[p]) tile_start[idx[p]] = (int32_t)p;
}

// tile lengths and each tile's reservation in the union pool: min(ucap, cnt * cap) entries
__global__ __launch_bounds__(kB) void k_tile_len(const GridInfo* __restrict__ gp, int64_t n, int64_t cap_tiles,
                                                 const int32_t* __restrict__ tile_start, int32_t* __restrict__ tile_cnt,
                                                 int cap, int ucap, uint32_t* __restrict__ ub) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cap_tiles) return;
  const int64_t nt = gp->ntiles;
  uint32_t v = 0;
  if (t < nt) {
    const int64_t e = t + 1 < nt ? tile_start[t + 1] : n;
    const int32_t cnt = (int32_t)(e - tile_start[t]);
    tile_cnt[t] = cnt;
    const int64_t b = (int64_t)cnt * cap;
    v = (uint32_t)(b < ucap ? b : ucap);
  }
  ub[t] = v;
}

// Tile neighbour lists.  Each tile is handled by one wavefront (one lane per target), in three
// latency-friendly phases per block of 64 candidate cells:
//  1. the 64 lanes enumerate 64 cells of the search box at once, cull them against the tile's
//     bounding box and look up their particle ranges (parallel loads);
//  2. the wave gathers the cells' particles 64 at a time (a wave-wide prefix sum maps lanes to
//     (cell, offset)), pre-tests each against the tile box and appends survivors to an LDS batch;
//  3. per batch of 64 candidates every lane runs the exact FP64 test against all of them,
//     building a 64-bit hit mask; the OR of the masks gives the batch's new union members (in
//     candidate order) and each lane appends the local indices of its hits.
// Tile t is particles [tile_start[t], tile_start[t] + tile_cnt[t]) of the array order (at most 64).
// Candidates enter batches in a fixed order (level, cell, cell-sorted position), so U and the
// lists are deterministic and each list is ascending in local index.
struct BuildArgs {
  const double4* __restrict__ pos4;
  int64_t n;
  const GridInfo* __restrict__ grid;
  const uint32_t* __restrict__ perm;   // cell-sorted position -> particle index
  const double4* __restrict__ pos_sorted;
  const int2* __restrict__ cell_se;
  const int32_t* __restrict__ tile_start;
  const int32_t* __restrict__ tile_cnt;
  const uint32_t* __restrict__ tile_uoff;
  int64_t capw, upool;
  int cap, ucap;
  int32_t* __restrict__ tile_u;
  int32_t* __restrict__ tile_usize;
  uint16_t* __restrict__ nbr16;     // candidate slot lists
  int32_t* __restrict__ count;       // candidates per particle
  int lanes;                         // slots per particle (lanes per target of the pair passes)
  int cap_sl;                        // entries a slot holds
  DevStatus* status;
};

__device__ __forceinline__ double wave_min_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
// min / max over aligned groups of 8 lanes
__device__ __forceinline__ double grp8_min(double v) {
  for (int off = 1; off < 8; off <<= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double grp8_max(double v) {
  for (int off = 1; off < 8; off <<= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ unsigned long long wave_or_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off, 64);
  return v;
}

struct TileState {
  int64_t a;
  int32_t a32;               // a as a 32-bit index (candidate indices are 32-bit), -1 if not valid
  bool valid;
  unsigned long long vmask;  // the wave's valid lanes
  double xa, ya, za, ha;
  double hs;                 // ha (1 + skin)(1 + 2^-40), the candidate test's scaled h
  int usize, cnt, ucap;
  int32_t* U;
  uint16_t* row;             // the lane's staging row in LDS (8 entries of each of the L slots)
  uint4* slot0;              // group 0 of the lane's first slot
  int64_t gstride;           // groups between consecutive groups of one slot (capw * lanes)
};

// Candidate k of a particle goes to its slot k % L, as entry k / L (L = lanes per target of the
// pair passes): each lane of the density pass then walks one contiguous slot list.  The lane's
// LDS row holds 8 L consecutive candidates in arrival order (candidate k at k mod 8 L, so entry p
// of slot s of the row's group sits at p L + s); when the row is full every slot has a complete
// group of 8, and the row is stored as L groups (group g of slot s at g * capw * L + s), each
// gathered from the row by byte permutes.  A row holds group g = k / (8 L) of every slot.
template <int L>
__device__ __forceinline__ void store_row_groups(const TileState& T, int g, int nslots) {
  uint32_t D[4 * L];
  __builtin_memcpy(D, T.row, sizeof(D));
#pragma unroll
  for (int s = 0; s < L; ++s) {
    if (s >= nslots) break;
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if constexpr (L == 1) {
        w[k] = D[k];
      } else {
        const int i0 = 2 * k * L + s, i1 = (2 * k + 1) * L + s;   // entries 2k, 2k+1 of slot s
        const uint32_t sel = ((i0 & 1) ? 0x0302u : 0x0100u) | ((i1 & 1) ? 0x07060000u : 0x05040000u);
        w[k] = __builtin_amdgcn_perm(D[i1 >> 1], D[i0 >> 1], sel);
      }
    }
    T.slot0[(int64_t)g * T.gstride + s] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}
template <int L>
__device__ __forceinline__ void append_candidate(const BuildArgs& B, TileState& T, int loc) {
  const unsigned k = (unsigned)T.cnt;
  const uint16_t v = (uint16_t)loc;
  __builtin_memcpy(T.row + (k & (8 * L - 1)), &v, sizeof(v));
  ++T.cnt;
  if ((k & (8 * L - 1)) == 8 * L - 1 && (int)(k / (8 * L)) * 8 < B.cap_sl) store_row_groups<L>(T, (int)(k / (8 * L)), L);
}

// candidate test (skin-widened, FP64) of every lane's target against batch candidates cb[0..nb),
// nb <= 64; NB > 0 fixes nb at compile time (full batches).  The test is
// r^2 < (h_a' + h_b')^2 with h' = h (1 + skin)(1 + 2^-40) (T.hs, cb[j].w) and r^2 by FMA: the
// factor 1 + 2^-40 exceeds the few ulp by which this rounding can differ from the exact decision
// of the density pass, so the candidates always contain every pair that test can accept (with a
// positive skin the rebuild test's own margin of 1e-9 is larger still).
// Candidates are taken one at a time: the wave's ballot decides at once whether candidate j joins
// the union (as its next member), and the lanes that hit it append that local index, so the
// lists come out ascending in local index and U in candidate order.
template <int L, int NB, bool PER>
__device__ __forceinline__ void run_batch(const BuildArgs& B, TileState& T, const double4* cb, const int32_t* cbi,
                                          int nb, double box) {
  const int lane = threadIdx.x;
  unsigned long long um = 0ull;   // the batch's union members (wave-uniform)
  int nm = 0;
  // the lane's decision (hit) and the wave's mask of it, the mask from the compares themselves
  // (ballot of the combined flag would first widen it to a vector register)
  struct Hit { bool hit; unsigned long long m; };
  auto test = [&](const double4& pb, int32_t bj) -> Hit {
    const double dx = min_image(T.xa - pb.x, (int)PER, box), dy = min_image(T.ya - pb.y, (int)PER, box),
                 dz = min_image(T.za - pb.z, (int)PER, box);
    const double H = T.hs + pb.w;
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx)), H2 = H * H;
    return Hit{T.valid && bj != T.a32 && r2 < H2,
               __builtin_amdgcn_fcmp(r2, H2, 4 /* ordered less than */) &
                   __builtin_amdgcn_uicmp(bj, T.a32, 33 /* not equal */) & T.vmask};
  };
  auto take = [&](int j, const Hit& t) {
    const bool hit = t.hit;
    if (t.m) {
      um |= 1ull << j;
      int loc = T.usize + nm;
      ++nm;
      loc = loc < T.ucap ? loc : T.ucap - 1;   // union overflow: keep reads in range, error latched
      if (hit) append_candidate<L>(B, T, loc);
    }
  };
  if constexpr (NB > 0) {
    // the next candidate's record is read from LDS while this one is tested and appended
    double4 nx = cb[0];
    int32_t nbi = cbi[0];
#pragma unroll 1
    for (int jb = 0; jb < NB; jb += 8) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double4 pb = nx;
        const int32_t bj = nbi;
        if (jb + k + 1 < NB) {
          nx = cb[jb + k + 1];
          nbi = cbi[jb + k + 1];
        }
        take(jb + k, test(pb, bj));
      }
    }
  } else {
    for (int j = 0; j < nb; ++j) take(j, test(cb[j], cbi[j]));
  }
  if (!um) return;
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  if ((um >> lane) & 1ull) {
    const int loc = T.usize + __popcll(um & lt);
    if (loc < T.ucap) T.U[loc] = cbi[lane];
  }
  T.usize += nm;
}

// Geometry of one tile, shared by the cost and build kernels: whole-tile box and max h
// (wave-uniform), and in LDS the sub-boxes of the 8 groups of 8 consecutive particles with their
// own max h.  Candidates and cells are tested against the sub-boxes, which stays tight where a
// tile mixes small and large h (a candidate within (h_a + h_b)(1 + skin) of a particle a is that
// close to a's sub-box).
struct TileGeom {
  double lo[3], hi[3], hmx;
};

__device__ __forceinline__ void tile_geometry(const double4 pa, bool valid, TileGeom& G, double (*sub)[8]) {
  const int lane = threadIdx.x;
  const double big = 1e300;
  const double q[3] = {pa.x, pa.y, pa.z};
  for (int d = 0; d < 3; ++d) {
    G.lo[d] = wave_min_d(valid ? q[d] : big);
    G.hi[d] = wave_max_d(valid ? q[d] : -big);
  }
  G.hmx = wave_max_d(valid ? pa.w : 0.0);
  double gl[3], gh[3];
  for (int d = 0; d < 3; ++d) {
    gl[d] = grp8_min(valid ? q[d] : big);
    gh[d] = grp8_max(valid ? q[d] : -big);
  }
  const double gx = grp8_max(valid ? pa.w : 0.0);
  __syncthreads();
  if ((lane & 7) == 0) {
    for (int d = 0; d < 3; ++d) {
      sub[lane >> 3][d] = 0.5 * (gl[d] + gh[d]);
      sub[lane >> 3][3 + d] = 0.5 * (gh[d] - gl[d]);
    }
    sub[lane >> 3][6] = gx;
  }
  __syncthreads();
}

// Cells of level l that can hold candidates of the tile: the tile box widened by
// (hmx + hlev[l])(1 + skin), clipped to the cells that hold the level's particles.
struct LevelBox {
  int lo3[3], ext[3];
  bool wrap[3];
  int64_t total;
  double c;
  uint32_t base;
};

template <bool PER>
__device__ __forceinline__ bool level_box(const GridInfo& g, int l, const TileGeom& G, double s1, LevelBox& L) {
  if (!g.hlev_bits[l]) return false;   // no particles at this level
  L.c = g.cell[l];
  L.base = g.base[l];
  const double R = (G.hmx + g.hlev[l]) * s1 * (1.0 + 1e-9);
  for (int d = 0; d < 3; ++d) {
    const int dim = g.dims[l][d];
    int l0 = (int)floor((G.lo[d] - R - g.lo[d]) / L.c);
    int h0 = (int)floor((G.hi[d] + R - g.lo[d]) / L.c);
    L.wrap[d] = false;
    if (PER) {
      if (h0 - l0 + 1 >= dim) { l0 = 0; h0 = dim - 1; }
      else L.wrap[d] = true;
    } else {
      const int b0 = cell_coord(dec_double(g.lev_lo[l][d]), g.lo[d], L.c, dim);
      const int b1 = cell_coord(dec_double(g.lev_hi[l][d]), g.lo[d], L.c, dim);
      l0 = l0 < b0 ? b0 : l0;
      h0 = h0 > b1 ? b1 : h0;
    }
    L.lo3[d] = l0;
    L.ext[d] = h0 >= l0 ? h0 - l0 + 1 : 0;
  }
  L.total = (int64_t)L.ext[0] * L.ext[1] * L.ext[2];
  return L.total > 0;
}

// Particle range [s, e) of the cell with linear index j of the level box (empty if the cell is
// farther than (hmax_g + hlev[l])(1 + skin) from every sub-box).  UNR: sub-boxes tested per
// unrolled step (their LDS reads issued together; more registers).
template <bool PER, int UNR>
__device__ __forceinline__ void cell_range(const GridInfo& g, int l, const LevelBox& L, int64_t j, double s1,
                                           const double (*sub)[8], const int2* __restrict__ cell_se, int& s, int& e) {
  s = e = 0;
  if (j >= L.total) return;
  // the box holds at most 2^30 cells (10 bits per axis), so 32-bit index arithmetic suffices
  const unsigned jj = (unsigned)j, e0 = (unsigned)L.ext[0], e1 = (unsigned)L.ext[1];
  const unsigned j1 = jj / e0;
  const int kk[3] = {L.lo3[0] + (int)(jj - j1 * e0), L.lo3[1] + (int)(j1 % e1), L.lo3[2] + (int)(j1 / e1)};
  int cc[3];
  double b0[3], b1[3];
  bool gapd[3];
  for (int d = 0; d < 3; ++d) {
    gapd[d] = !PER || L.wrap[d];
    b0[d] = g.lo[d] + kk[d] * L.c;
    b1[d] = b0[d] + L.c;
    const int dim = g.dims[l][d];
    cc[d] = L.wrap[d] ? ((kk[d] % dim) + dim) % dim : kk[d];
  }
  bool need = false;
#pragma unroll UNR
  for (int gi = 0; gi < 8; ++gi) {
    double gap2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double gd = fmax(0.0, fmax(b0[d] - (sub[gi][d] + sub[gi][3 + d]), (sub[gi][d] - sub[gi][3 + d]) - b1[d]));
      gap2 += gapd[d] ? gd * gd : 0.0;
    }
    const double Rg = (sub[gi][6] + g.hlev[l]) * s1 * (1.0 + 1e-9);
    need |= gap2 < Rg * Rg && sub[gi][6] > 0.0;
  }
  if (need) {
    const uint32_t key = L.base + (spread3((uint32_t)cc[0]) | (spread3((uint32_t)cc[1]) << 1) |
                                   (spread3((uint32_t)cc[2]) << 2));
    const int2 se = cell_se[key];
    s = se.x;
    e = se.y;
  }
}

// Cost estimate of each tile: the number of particles in the cells its build would gather.
template <bool PER>
__global__ __launch_bounds__(64) void k_tile_cost(const double4* __restrict__ pos4, const GridInfo* __restrict__ gp,
                                                  const int32_t* __restrict__ tile_start,
                                                  const int32_t* __restrict__ tile_cnt, const int2* __restrict__ cell_se,
                                                  int32_t* __restrict__ cost) {
  __shared__ double sub[8][8];
  const int lane = threadIdx.x;
  const GridInfo& g = *gp;
  const double s1 = 1.0 + g.skin;
  const int64_t ntiles = g.ntiles;
  for (int64_t k_ = blockIdx.x / SPH_XCD, chunk_ = xcd_chunk(ntiles); k_ < chunk_; k_ += gridDim.x / SPH_XCD) {
    const int64_t t = (int64_t)(blockIdx.x % SPH_XCD) * chunk_ + k_;
    if (t >= ntiles) break;
    const bool valid = lane < tile_cnt[t];
    const double4 pa = valid ? pos4[tile_start[t] + lane] : make_double4(0.0, 0.0, 0.0, 0.0);
    TileGeom G;
    tile_geometry(pa, valid, G, sub);
    int64_t tot = 0;
    for (int l = 0; l < g.nlev; ++l) {
      LevelBox L;
      if (!level_box<PER>(g, l, G, s1, L)) continue;
      for (int64_t q = 0; q < L.total; q += 64) {
        int s, e;
        cell_range<PER, 4>(g, l, L, q + lane, s1, sub, cell_se, s, e);
        tot += e - s;
      }
    }
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
    if (lane == 0) cost[t] = (int32_t)(tot < 0x7fffffff ? tot : 0x7fffffff);
    __syncthreads();
  }
}

// Splits expensive tiles: a particle also starts a tile at every 16th (cost > kSplit16 / cdiv) or
// 8th (cost > kSplit8 / cdiv) position of its tile.  The cost counts the particles of the cells a
// build gathers, which shrinks with finer cells (cdiv cells per smoothing diameter).  Reads the
// tile of p from the scan of the old flags.
constexpr int32_t kSplit16 = 12000, kSplit8 = 40000;
__global__ __launch_bounds__(kB) void k_tile_split(uint32_t* __restrict__ flag, const uint32_t* __restrict__ idx,
                                                   int64_t n, const int32_t* __restrict__ tile_start,
                                                   const int32_t* __restrict__ cost, int cdiv) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t f = flag[p];
  const int64_t t = (int64_t)idx[p] + f - 1;
  const int32_t c = cost[t];
  const int64_t off = p - tile_start[t];
  const int size = c > kSplit8 / cdiv ? 8 : (c > kSplit16 / cdiv ? 16 : 64);
  flag[p] = (f || (off % size) == 0) ? 1u : 0u;
}

// Tile neighbour lists.  Each tile is handled by one wavefront (one lane per target), in three
// latency-friendly phases per block of 64 candidate cells:
//  1. the 64 lanes take 64 cells of the level box at once, cull them against the sub-boxes and
//     load their particle ranges;
//  2. the wave gathers the cells' particles 64 at a time (a wave-wide prefix sum maps lanes to
//     (cell, offset)), pre-tests each against the sub-boxes and appends survivors to an LDS batch;
//  3. per batch of 64 candidates every lane runs the skin-widened FP64 test against all of them,
//     building a 64-bit hit mask; the OR of the masks gives the batch's new union members (in
//     candidate order) and each lane appends the local indices of its hits.
// Tile t is particles [tile_start[t], tile_start[t] + tile_cnt[t]) of the array order (at most 64).
// Candidates enter batches in a fixed order (level, cell, cell-sorted position), so U and the
// lists are deterministic and each list is ascending in local index.
template <bool PER, int NL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_build_tiles(BuildArgs B) {
  __shared__ int32_t c_s[64], c_o[64];
  __shared__ double sub[8][8];   // per group of 8 tile particles: centre xyz, half-width xyz, max h
  __shared__ double4 tp[16];     // the particles of a small tile (its exact pre-filter)
  __shared__ double4 cb[128];
  __shared__ int32_t cbi[128];
  __shared__ __align__(16) uint16_t crow[64][8 * NL];   // per lane: staging of the candidate lists
  const int lane = threadIdx.x;
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const GridInfo& g = *B.grid;
  const double box = g.box;
  const double s1 = 1.0 + g.skin;
  const double s1w = s1 * (1.0 + 0x1p-40);   // the batch test's widened factor
  const int64_t ntiles = g.ntiles;
  for (int64_t k_ = blockIdx.x / SPH_XCD, chunk_ = xcd_chunk(ntiles); k_ < chunk_; k_ += gridDim.x / SPH_XCD) {
    const int64_t t = (int64_t)(blockIdx.x % SPH_XCD) * chunk_ + k_;
    if (t >= ntiles) break;
    const int32_t tcnt = B.tile_cnt[t];
    const int64_t p = (int64_t)B.tile_start[t] + lane;
    TileState T;
    T.valid = lane < tcnt;
    T.a = T.valid ? p : -1;
    T.a32 = (int32_t)T.a;
    T.vmask = __builtin_amdgcn_ballot_w64(T.valid);
    const double4 pa = T.valid ? B.pos4[T.a] : make_double4(0.0, 0.0, 0.0, 0.0);
    T.xa = pa.x; T.ya = pa.y; T.za = pa.z; T.ha = pa.w; T.hs = pa.w * s1w;
    TileGeom G;
    tile_geometry(pa, T.valid, G, sub);
    if (lane < 16) tp[lane] = pa;
    // small tiles (split because they are expensive) pre-filter candidates exactly against
    // their own particles: far fewer batches, each of which would use only tcnt lanes
    const bool small = tcnt <= 16;
    const uint32_t uoff = B.tile_uoff[t];
    T.ucap = (int)((int64_t)tcnt * B.cap < B.ucap ? (int64_t)tcnt * B.cap : B.ucap);
    if ((int64_t)uoff + T.ucap > B.upool) {
      T.ucap = 0;
      if (lane == 0) latch_error(B.status, SPH_E_NGB_CAPACITY, -1);
    }
    T.U = B.tile_u + uoff;
    T.usize = 0; T.cnt = 0;
    T.row = crow[lane];
    T.slot0 = reinterpret_cast<uint4*>(B.nbr16) + (T.valid ? p : 0) * NL;
    T.gstride = B.capw * NL;
    int pend = 0;   // candidates waiting in cb (wave-uniform)
    for (int l = 0; l < g.nlev; ++l) {
      LevelBox L;
      if (!level_box<PER>(g, l, G, s1, L)) continue;
      for (int64_t q = 0; q < L.total; q += 64) {
        // phase 1: 64 cells at once; lanes take the block's cells in bit-reversed order so that
        // consecutive union members come from all over the neighbourhood and every target's
        // neighbours spread evenly over the LDS chunks of the pair passes
        int s, e;
        cell_range<PER, 2>(g, l, L, q + (int64_t)(__brev((unsigned)lane) >> 26), s1, sub, B.cell_se, s, e);
        // wave prefix sum of the cells' particle counts
        const int cntc = e - s;
        int inc = cntc;
        for (int off = 1; off < 64; off <<= 1) {
          const int o = __shfl_up(inc, off, 64);
          if (lane >= off) inc += o;
        }
        const int Tc = __shfl(inc, 63, 64);
        __syncthreads();
        c_s[lane] = s;
        c_o[lane] = inc - cntc;
        __syncthreads();
        // phase 2: gather candidates, 4 rounds of 64 per pass (loads of all 4 issued together),
        // pre-test against the sub-boxes (small tiles: against their particles) and append the
        // survivors to the batch in slot order
        for (int q0 = 0; q0 < Tc; q0 += 256) {
          double4 pbu[4];
          int32_t bu[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int slot = q0 + 64 * u + lane;
            pbu[u] = make_double4(0.0, 0.0, 0.0, 0.0);
            bu[u] = -1;
            if (slot < Tc) {
              int lo_i = 0, hi_i = 63;   // last cell with c_o <= slot
              while (lo_i < hi_i) {
                const int mid = (lo_i + hi_i + 1) >> 1;
                if (c_o[mid] <= slot) lo_i = mid;
                else hi_i = mid - 1;
              }
              const int32_t sp = c_s[lo_i] + (slot - c_o[lo_i]);
              bu[u] = (int32_t)B.perm[sp];
              pbu[u] = B.pos_sorted[sp];
            }
          }
          // pre-test of the 4 rounds: each sub-box (particle) is read from LDS once for all 4
          bool pass[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) pass[u] = false;
          if (small) {
            for (int k = 0; k < tcnt; ++k) {
              const double4 q = tp[k];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const double4 pb = pbu[u];
                pass[u] |= candidate_test(min_image(q.x - pb.x, (int)PER, box), min_image(q.y - pb.y, (int)PER, box),
                                          min_image(q.z - pb.z, (int)PER, box), q.w, pb.w, s1);
              }
            }
          } else {
#pragma unroll 1
            for (int gi = 0; gi < 8; ++gi) {
              const double cx = sub[gi][0], cy = sub[gi][1], cz = sub[gi][2];
              const double wx = sub[gi][3], wy = sub[gi][4], wz = sub[gi][5], hg = sub[gi][6];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const double4 pb = pbu[u];
                const double ex = fmax(0.0, fabs(min_image(pb.x - cx, (int)PER, box)) - wx);
                const double ey = fmax(0.0, fabs(min_image(pb.y - cy, (int)PER, box)) - wy);
                const double ez = fmax(0.0, fabs(min_image(pb.z - cz, (int)PER, box)) - wz);
                const double Rb = (hg + pb.w) * s1 * (1.0 + 1e-9);
                pass[u] |= ex * ex + ey * ey + ez * ez < Rb * Rb && hg > 0.0;
              }
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (q0 + 64 * u >= Tc) break;
            const double4 pb = pbu[u];
            pass[u] = pass[u] && bu[u] >= 0;
            const unsigned long long m = __ballot(pass[u]);
            if (pass[u]) {
              const int k = pend + __popcll(m & lt);
              cb[k] = make_double4(pb.x, pb.y, pb.z, pb.w * s1w);
              cbi[k] = bu[u];
            }
            pend += __popcll(m);
            __syncthreads();
            if (pend >= 64) {   // phase 3 on a full batch
              run_batch<NL, 64, PER>(B, T, cb, cbi, 64, box);
              const int rest = pend - 64;
              double4 mv = make_double4(0.0, 0.0, 0.0, 0.0);
              int32_t mi = 0;
              if (lane < rest) { mv = cb[64 + lane]; mi = cbi[64 + lane]; }
              __syncthreads();
              if (lane < rest) { cb[lane] = mv; cbi[lane] = mi; }
              pend = rest;
              __syncthreads();
            }
          }
        }
      }
    }
    if (pend > 0) run_batch<NL, 0, PER>(B, T, cb, cbi, pend, box);
    __syncthreads();
    if (T.valid && T.cnt <= B.cap && (T.cnt & (8 * NL - 1))) {
      // the partly filled last row: slots s < r hold a partial last group g (a slot's count is at
      // most that of slot 0, so the capacity test of slot 0 covers them all)
      const int r = T.cnt & (8 * NL - 1), g = T.cnt / (8 * NL);
      if ((T.cnt + NL - 1) / NL <= B.cap_sl) store_row_groups<NL>(T, g, r < NL ? r : NL);
    }
    if (T.valid) B.count[p] = T.cnt < B.cap ? T.cnt : B.cap;
    if (lane == 0) B.tile_usize[t] = T.usize < T.ucap ? T.usize : T.ucap;
    if (T.usize > T.ucap || T.cnt > B.cap) latch_error(B.status, SPH_E_NGB_CAPACITY, (int)(T.valid ? T.a : -1));
  }
}

__global__ __launch_bounds__(kB) void k_count_stats(const int32_t* __restrict__ cnt, int64_t n,
                                                    unsigned long long* total, int32_t* mx) {
  unsigned long long s = 0;
  int m = 0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
    s += (unsigned long long)cnt[a];
    m = cnt[a] > m ? cnt[a] : m;
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    int o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(total, s);
    atomicMax(mx, m);
  }
}

// Permutes the 8-byte arrays arr[0, m) in place along c->vals: batches of up to kPermBatch go
// through a staging area in one gather and one copy launch each.  The staging is the candidate-list
// buffer, whose lists the build that follows rewrites (c->tmp, one array, where it is smaller).
static sph_status permute_arrays(sph_ctx* c, double* const* arr, int m, int64_t n) {
  if (n <= 0) return SPH_OK;
  const size_t big = (size_t)c->capw * (size_t)(c->cap_s + 32) * sizeof(uint16_t);
  double* stage = reinterpret_cast<double*>(c->nbr16s);
  int per = (int)(big / (sizeof(double) * (size_t)n));
  if (per < 1) { stage = c->tmp; per = 1; }
  per = per < kPermBatch ? per : kPermBatch;
  const unsigned nb = grid_for(n, kB);
  for (int k0 = 0; k0 < m; k0 += per) {
    PermBatch G{}, C{};
    G.na = C.na = (m - k0) < per ? (m - k0) : per;
    for (int k = 0; k < G.na; ++k) {
      G.src[k] = arr[k0 + k];
      G.dst[k] = stage + (int64_t)k * n;
      C.src[k] = G.dst[k];
      C.dst[k] = arr[k0 + k];
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_permute_batch<true>), dim3(nb), dim3(kB), 0, c->stream, G, c->vals, n);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_permute_batch<false>), dim3(nb), dim3(kB), 0, c->stream, C, c->vals, n);
  }
  HIP_TRY(hipGetLastError());
  return SPH_OK;
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

// The union pool is sized to what the tiles reserve: read the reservation total and grow the
// pool (by a quarter more than needed) when it does not fit.  Waits for the stream.
static sph_status ensure_pool(sph_ctx* c) {
  // ntiles, upool_used and nstress are adjacent in GridInfo: one copy brings all three
  static_assert(offsetof(GridInfo, upool_used) == offsetof(GridInfo, ntiles) + 4 &&
                    offsetof(GridInfo, nstress) == offsetof(GridInfo, ntiles) + 8,
                "GridInfo layout");
  HIP_TRY(hipMemcpyAsync(c->drift_host, &c->grid->ntiles, 3 * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const uint32_t used = c->drift_host[1];
  c->stress_heavy = 2ull * c->drift_host[2] > (unsigned long long)c->drift_host[0];
  if ((int64_t)used <= c->upool) return SPH_OK;
  int64_t want = (int64_t)used + (int64_t)used / 4;
  if (want > (int64_t)0xffffffffll) want = (int64_t)0xffffffffll;
  HIP_TRY(hipFree(c->tile_u));
  c->tile_u = nullptr;
  c->upool = 0;
  if (hipMalloc((void**)&c->tile_u, sizeof(int32_t) * (size_t)want) != hipSuccess) {
    c->tile_u = nullptr;
    return SPH_E_OOM;
  }
  c->upool = want;
  ++c->graph_epoch;   // captured kernels hold the old pool pointer
  return SPH_OK;
}

// Cells per smoothing diameter of the finest level (default 1: cells of 2 hmax_l).  Measured on
// the 2M-particle star, 1 against 2 takes a list build from 6.2 to 5.3 ms (8x fewer cells to
// cull, at 1.5x more particles to pre-test) and the FP32 step from 1.335 to 1.288 ms.
static int cell_div_of(const sph_params& p) { return p.cell_div > 0 ? p.cell_div : 1; }

static unsigned tile_grid(int64_t cap_tiles) {
  return (unsigned)(cap_tiles < 65536 ? cap_tiles : 65536);
}

template <bool PER>
static void launch_build_per(const BuildArgs& B, dim3 grid, hipStream_t s) {
  if (B.lanes == 1)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_build_tiles<PER, 1>), grid, dim3(64), 0, s, B);
  else if (B.lanes == 2)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_build_tiles<PER, 2>), grid, dim3(64), 0, s, B);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_build_tiles<PER, 4>), grid, dim3(64), 0, s, B);
}
static void launch_build(const BuildArgs& B, bool per, dim3 grid, hipStream_t s) {
  if (per) launch_build_per<true>(B, grid, s);
  else launch_build_per<false>(B, grid, s);
}

// Candidate-list build: every particle array of the state (and the half-step copies) is reordered
// along the global Morton curve (the outputs only when outputs_recomputed is false), tiles are cut
// from that order, particles are binned into the multi-level grid and each tile's candidates are
// collected; the positions and h at the list build are kept for the drift test.
sph_status sph_rebin(sph_ctx* c, sph_state* st, bool outputs_recomputed) {
  const int64_t n = st->n;
  hipStream_t s = c->stream;
  const unsigned nb = grid_for(n, kB);
  unsigned nred = nb < 1024 ? nb : 1024;
  sph_status e;
  hipLaunchKernelGGL(k_pack_pos, dim3(nb), dim3(kB), 0, s, st->x, st->y, st->z, st->h,
                     (const int32_t*)nullptr, (const StarInfo*)nullptr, n, c->pos4, (float4*)nullptr);
  hipLaunchKernelGGL(k_bounds, dim3(nred), dim3(kB), 0, s, c->pos4, n, c->sort.partial);
  hipLaunchKernelGGL(k_grid_setup1, dim3(1), dim3(64), 0, s, c->grid, c->sort.partial, (int)nred, c->p.periodic,
                     c->p.box, c->p.skin, c->status);
  {
    hipLaunchKernelGGL(k_gkeys, dim3(nb), dim3(kB), 0, s, c->pos4, n, c->grid, c->keys, c->vals);
    if ((e = sph_sort_pairs(c, c->keys, c->vals, n))) return e;
    double* d64[64];
    int m = 0;
    for (double* a : {st->x, st->y, st->z, st->vx, st->vy, st->vz, st->u, st->h}) d64[m++] = a;
    for (int k = 0; k < 6; ++k) d64[m++] = st->S + k * n;
    if (!outputs_recomputed) {
      for (double* a : {st->D, st->rho, st->P, st->cs, st->ax, st->ay, st->az, st->dudt}) d64[m++] = a;
      for (int k = 0; k < 6; ++k) d64[m++] = st->dSdt + k * n;
    } else {   // state that the next evaluation reads although it is an output
      if (c->p.density_mode == SPH_DENS_CONTINUITY) d64[m++] = st->D;
      if (c->p.dtP_mode == SPH_DTP_LAGGED) d64[m++] = st->P;
    }
    for (int k = 0; k < SPH_HALF_FIELDS; ++k) d64[m++] = c->half + (int64_t)k * c->capacity;
    if ((e = permute_arrays(c, d64, m, n))) return e;
    if ((e = permute_array(c, st->type, n))) return e;
    if ((e = permute_array(c, st->broken, n))) return e;
    if ((e = permute_array(c, st->id, n))) return e;
    if ((e = permute_array(c, st->star, n))) return e;
    hipLaunchKernelGGL(k_pack_pos, dim3(nb), dim3(kB), 0, s, st->x, st->y, st->z, st->h,
                       (const int32_t*)nullptr, (const StarInfo*)nullptr, n, c->pos4, (float4*)nullptr);
  }
  // tile starts along the Morton order (the keys are overwritten by the cell sort below)
  uint32_t* flag = reinterpret_cast<uint32_t*>(c->tmp);
  uint32_t* idx = flag + c->capw;
  hipLaunchKernelGGL(k_tile_flags, dim3(nb), dim3(kB), 0, s, c->keys, c->pos4, n, c->grid,
                     tile_cut_of(c->p), flag);
  hipLaunchKernelGGL(k_level_hmax, dim3(nred), dim3(kB), 0, s, c->pos4, n, c->grid);
  hipLaunchKernelGGL(k_grid_setup2, dim3(1), dim3(1), 0, s, c->grid, cell_div_of(c->p),
                     c->max_cells, c->status);
  hipLaunchKernelGGL(k_keys, dim3(nb), dim3(kB), 0, s, c->pos4, n, c->grid, c->keys, c->vals);
  if ((e = sph_sort_pairs(c, c->keys, c->vals, n))) return e;
  hipLaunchKernelGGL(k_cells_clear, dim3(2048), dim3(kB), 0, s, c->cell_se, c->grid);
  hipLaunchKernelGGL(k_cell_ranges, dim3(nb), dim3(kB), 0, s, c->keys, n, c->cell_se);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gather<double4>), dim3(nb), dim3(kB), 0, s, c->pos4, c->vals, n, c->pos_sorted);
  // tile table: Morton cuts, then tiles whose candidate cells hold many particles are split
  const bool per = c->p.periodic != 0;
  for (int pass = 0; pass < 2; ++pass) {
    if ((e = sph_scan_u32(c, flag, idx, n, &c->grid->ntiles))) return e;
    hipLaunchKernelGGL(k_tile_fill, dim3(nb), dim3(kB), 0, s, flag, idx, n, c->tile_start);
    hipLaunchKernelGGL(k_tile_len, dim3(grid_for(c->cap_tiles, kB)), dim3(kB), 0, s, c->grid, n, c->cap_tiles,
                       c->tile_start, c->tile_cnt, c->cap_s, c->ucap, c->tile_uoff);
    if (pass == 1) break;
    if (per)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tile_cost<true>), dim3(tile_grid(c->cap_tiles)), dim3(64), 0, s, c->pos4,
                         c->grid, c->tile_start, c->tile_cnt, c->cell_se, c->tile_usize);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tile_cost<false>), dim3(tile_grid(c->cap_tiles)), dim3(64), 0, s, c->pos4,
                         c->grid, c->tile_start, c->tile_cnt, c->cell_se, c->tile_usize);
    hipLaunchKernelGGL(k_tile_split, dim3(nb), dim3(kB), 0, s, flag, idx, n, c->tile_start, c->tile_usize,
                       cell_div_of(c->p));
  }
  if ((e = sph_scan_u32(c, c->tile_uoff, c->tile_uoff, c->cap_tiles, &c->grid->upool_used))) return e;
  // stress-pass work list (tiles with a type-1 particle), read back with the pool size
  hipLaunchKernelGGL(k_stress_flags, dim3(grid_for(c->cap_tiles, kB)), dim3(kB), 0, s, c->grid, c->cap_tiles,
                     c->tile_start, c->tile_cnt, st->type, flag);
  if ((e = sph_scan_u32(c, flag, idx, c->cap_tiles, &c->grid->nstress))) return e;
  hipLaunchKernelGGL(k_stress_list, dim3(grid_for(c->cap_tiles, kB)), dim3(kB), 0, s, flag, idx, c->cap_tiles,
                     c->stress_tiles);
  if ((e = ensure_pool(c))) return e;
  BuildArgs B;
  B.pos4 = c->pos4; B.n = n; B.grid = c->grid; B.perm = c->vals; B.pos_sorted = c->pos_sorted;
  B.cell_se = c->cell_se; B.capw = c->capw; B.cap = c->cap_s; B.ucap = c->ucap;
  B.lanes = pass_lanes(c->p); B.cap_sl = cand_slot_capacity(c->cap_s, B.lanes);
  B.tile_start = c->tile_start; B.tile_cnt = c->tile_cnt; B.tile_uoff = c->tile_uoff; B.upool = c->upool;
  B.tile_u = c->tile_u; B.tile_usize = c->tile_usize; B.nbr16 = c->nbr16s; B.count = c->nbr_count_s;
  B.status = c->status;
  launch_build(B, per, dim3(tile_grid(c->cap_tiles)), s);
  hipLaunchKernelGGL(k_tile_union_type, dim3(tile_grid(c->cap_tiles)), dim3(64), 0, s, c->grid, c->tile_start,
                     c->tile_cnt, c->tile_uoff, c->tile_usize, c->tile_u, st->type, c->tile_st);
  HIP_TRY(hipGetLastError());
  // the zero rates of every type-0 particle
  hipLaunchKernelGGL(k_zero_fluid_rates, dim3(grid_for(n, kB)), dim3(kB), 0, s, st->type, n, st->S, st->dSdt,
                     c->sdot);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(c->pos_build, c->pos4, sizeof(double4) * n, hipMemcpyDeviceToDevice, s));
  return launch_pack(c, st);
}

// Skin test of the current positions and h against the last build (for sph_build_cells; inside
// sph_step the test is fused into the drift kernel).
__global__ __launch_bounds__(kB) void k_drift_check(const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ z, const double* __restrict__ h,
                                                    const double4* __restrict__ pb, int64_t n,
                                                    const GridInfo* __restrict__ gp, uint32_t id,
                                                    uint32_t* __restrict__ flag) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const GridInfo& g = *gp;
  const double4 b = pb[a];
  if (skin_exceeded(min_image(x[a] - b.x, g.periodic, g.box), min_image(y[a] - b.y, g.periodic, g.box),
                    min_image(z[a] - b.z, g.periodic, g.box), h[a], b, g.skin))
    atomicMax(flag, id);
}

sph_status launch_drift_check(sph_ctx* c, sph_state* st) {
  hipLaunchKernelGGL(k_drift_check, dim3(grid_for(st->n, kB)), dim3(kB), 0, c->stream, st->x, st->y, st->z,
                     st->h, c->pos_build, st->n, c->grid, c->check_id, c->drift_flag);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

// Pack the position records the pair passes read, in the current particle order.
sph_status launch_pack(sph_ctx* c, sph_state* st) {
  const int64_t n = st->n;
  hipLaunchKernelGGL(k_pack_pos, dim3(grid_for(n, kB)), dim3(kB), 0, c->stream, st->x, st->y, st->z, st->h,
                     st->star, c->stars, n, c->pos4, c->p.precision == SPH_FP32 ? c->pos4f : nullptr);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

__global__ __launch_bounds__(kB) void k_union_stats(const int32_t* __restrict__ usize, const GridInfo* __restrict__ gp,
                                                    unsigned long long* total) {
  unsigned long long s = 0;
  const int64_t nt = gp->ntiles;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x)
    s += (unsigned long long)usize[t];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(total, s);
}

sph_status sph_count_stats(sph_ctx* c, sph_list_stats* out) {
  struct R { unsigned long long t, u, cs; int32_t m, ms; };
  R* d = nullptr;
  if (hipMalloc((void**)&d, sizeof(R)) != hipSuccess) return SPH_E_OOM;
  R h = {0ull, 0ull, 0ull, 0, 0};
  sph_status e = SPH_OK;
  if (hipMemcpy(d, &h, sizeof(R), hipMemcpyHostToDevice) != hipSuccess) e = SPH_E_HIP;
  if (!e && c->n > 0 && c->lists_valid) {
    unsigned nb = grid_for(c->n, kB);
    nb = nb < 1024 ? nb : 1024;
    if (c->gen >= 2)
      hipLaunchKernelGGL(k_count_stats, dim3(nb), dim3(kB), 0, c->stream, c->nbr_count, c->n, &d->t, &d->m);
    hipLaunchKernelGGL(k_count_stats, dim3(nb), dim3(kB), 0, c->stream, c->nbr_count_s, c->n, &d->cs, &d->ms);
    hipLaunchKernelGGL(k_union_stats, dim3(256), dim3(kB), 0, c->stream, c->tile_usize, c->grid, &d->u);
    if (hipStreamSynchronize(c->stream) != hipSuccess) e = SPH_E_HIP;
  }
  if (!e && hipMemcpy(&h, d, sizeof(R), hipMemcpyDeviceToHost) != hipSuccess) e = SPH_E_HIP;
  (void)hipFree(d);
  out->pairs = (int64_t)h.t;
  out->max_count = h.m;
  out->pad = 0;
  out->union_total = (int64_t)h.u;
  out->candidates = (int64_t)h.cs;
  out->rebuilds = c->rebuilds;
  out->tiles = 0;
  if (!e && c->n > 0 && c->lists_valid) {
    GridInfo g;
    if (hipMemcpy(&g, c->grid, sizeof(g), hipMemcpyDeviceToHost) != hipSuccess) return SPH_E_HIP;
    out->tiles = (int64_t)g.ntiles;
  }
  return e;
}

// ---- list statistics without device allocation ------------------------------------------------
// Counters of sph_neighbour_stats_noalloc: exact pairs, union members, candidates (64-bit) and
// the longest exact and candidate lists (32-bit, in the fourth and fifth words).  One copy per
// GPU, held until the process ends; every call on a GPU uses that GPU's copy.  Host code never
// names the array in a kernel argument or copy: it uses the device address looked up once per
// device by stats_scratch_init.
constexpr int kStatWords = 8;
static __device__ __align__(256) unsigned long long scratch[kStatWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_addr[kMaxDevices] = {};

__global__ void k_clear_words(unsigned long long* __restrict__ w, int n) {
  if ((int)threadIdx.x < n) w[threadIdx.x] = 0ull;
}
}  // namespace

sph_status stats_scratch_init(sph_ctx* c) {
  if (c->device < 0 || c->device >= kMaxDevices) return SPH_E_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[c->device]) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != c->device) HIP_TRY(hipSetDevice(c->device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != c->device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) return SPH_E_HIP;
    g_scratch_addr[c->device] = (unsigned long long*)ptr;
  }
  c->stats_scratch = g_scratch_addr[c->device];
  return SPH_OK;
}

extern "C" sph_status sph_neighbour_stats_noalloc(sph_ctx* c, sph_list_stats* out) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (!out) return note(c, SPH_E_ARG, "out is NULL");
  unsigned long long* d = c->stats_scratch;
  if (!d) return note(c, SPH_E_HIP, "no statistics scratch address for device %d", c->device);
  hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, c->stream, d, kStatWords);
  int32_t* mx = reinterpret_cast<int32_t*>(d + 3);   // words 3 and 4 hold the two maxima
  if (c->n > 0 && c->lists_valid) {
    unsigned nb = grid_for(c->n, kB);
    nb = nb < 1024 ? nb : 1024;
    if (c->gen >= 2) hipLaunchKernelGGL(k_count_stats, dim3(nb), dim3(kB), 0, c->stream, c->nbr_count, c->n, d, mx);
    hipLaunchKernelGGL(k_count_stats, dim3(nb), dim3(kB), 0, c->stream, c->nbr_count_s, c->n, d + 2, mx + 2);
    hipLaunchKernelGGL(k_union_stats, dim3(256), dim3(kB), 0, c->stream, c->tile_usize, c->grid, d + 1);
  }
  hipError_t he = hipGetLastError();
  unsigned long long h[kStatWords];
  GridInfo g;
  if (he == hipSuccess) he = hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (he == hipSuccess && c->n > 0 && c->lists_valid)
    he = hipMemcpyAsync(&g, c->grid, sizeof(g), hipMemcpyDeviceToHost, c->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
  if (he != hipSuccess) return note(c, SPH_E_HIP, "statistics: %s", hipGetErrorString(he));
  int32_t m[4];
  memcpy(m, h + 3, sizeof(m));
  out->pairs = (int64_t)h[0];
  out->union_total = (int64_t)h[1];
  out->candidates = (int64_t)h[2];
  out->max_count = m[0];
  out->pad = 0;
  out->rebuilds = c->rebuilds;
  out->tiles = (c->n > 0 && c->lists_valid) ? (int64_t)g.ntiles : 0;
  return SPH_OK;
}

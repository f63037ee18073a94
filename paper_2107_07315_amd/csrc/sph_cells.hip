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
  for (int l = 0; l < SPH_MAX_LEV; ++l) g->hlev_bits[l] = 0ull;
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
  const uint32_t* __restrict__ skeys;
  const uint32_t* __restrict__ perm;   // cell-sorted position -> particle index
  const int32_t* __restrict__ cstart;
  const int32_t* __restrict__ cend;
  const int32_t* __restrict__ tile_start;
  const int32_t* __restrict__ tile_cnt;
  const uint32_t* __restrict__ tile_uoff;
  int64_t capw, upool;
  int cap, ucap;
  int32_t* __restrict__ tile_u;
  int32_t* __restrict__ tile_usize;
  uint16_t* __restrict__ nbr16;
  int32_t* __restrict__ count;
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
__device__ __forceinline__ unsigned long long wave_or_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off, 64);
  return v;
}

struct TileState {
  int64_t a;
  bool valid;
  double xa, ya, za, ha;
  int usize, cnt, stored, ucap;
  int64_t p;
  int32_t* U;
};

// candidate test (skin-widened, FP64) of every lane's target against batch candidates cb[0..nb),
// nb <= 64
__device__ __forceinline__ void run_batch(const BuildArgs& B, TileState& T, const double4* cb, const int32_t* cbi,
                                          int nb, int periodic, double box, double s1) {
  const int lane = threadIdx.x;
  unsigned long long hm = 0ull;
  if (T.valid) {
    for (int j = 0; j < nb; ++j) {
      const double4 pb = cb[j];
      const bool hit = cbi[j] != T.a &&
                       candidate_test(min_image(T.xa - pb.x, periodic, box), min_image(T.ya - pb.y, periodic, box),
                                      min_image(T.za - pb.z, periodic, box), T.ha, pb.w, s1);
      hm |= (unsigned long long)hit << j;
    }
  }
  const unsigned long long um = wave_or_u64(hm);
  if (!um) return;
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  if ((um >> lane) & 1ull) {
    const int loc = T.usize + __popcll(um & lt);
    if (loc < T.ucap) T.U[loc] = cbi[lane];
  }
  unsigned long long mm = hm;
  while (mm) {
    const int j = __ffsll((long long)mm) - 1;
    mm &= mm - 1ull;
    const int loc = T.usize + __popcll(um & ((1ull << j) - 1ull));
    if (T.cnt < B.cap && loc < T.ucap) {
      B.nbr16[nbr_index(T.cnt, T.p, B.capw)] = (uint16_t)loc;
      ++T.stored;
    }
    ++T.cnt;
  }
  T.usize += __popcll(um);
}

__global__ __launch_bounds__(64) void k_build_tiles(BuildArgs B) {
  __shared__ int32_t c_s[64], c_o[64];
  __shared__ double4 cb[128];
  __shared__ int32_t cbi[128];
  const int lane = threadIdx.x;
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const GridInfo& g = *B.grid;
  const int periodic = g.periodic;
  const double box = g.box;
  const double s1 = 1.0 + g.skin;
  const int64_t ntiles = g.ntiles;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int32_t tcnt = B.tile_cnt[t];   // (lists below are the candidate lists)
    const int64_t p = (int64_t)B.tile_start[t] + lane;
    TileState T;
    T.valid = lane < tcnt;
    T.a = T.valid ? p : -1;
    double4 pa = T.valid ? B.pos4[T.a] : make_double4(0.0, 0.0, 0.0, 0.0);
    T.xa = pa.x; T.ya = pa.y; T.za = pa.z; T.ha = pa.w;
    const double big = 1e300;
    double lo[3], hi[3];
    lo[0] = wave_min_d(T.valid ? pa.x : big); hi[0] = wave_max_d(T.valid ? pa.x : -big);
    lo[1] = wave_min_d(T.valid ? pa.y : big); hi[1] = wave_max_d(T.valid ? pa.y : -big);
    lo[2] = wave_min_d(T.valid ? pa.z : big); hi[2] = wave_max_d(T.valid ? pa.z : -big);
    const double hmx = wave_max_d(T.valid ? pa.w : 0.0);
    double cen[3], hw[3];
    for (int d = 0; d < 3; ++d) { cen[d] = 0.5 * (lo[d] + hi[d]); hw[d] = 0.5 * (hi[d] - lo[d]); }
    const uint32_t uoff = B.tile_uoff[t];
    T.ucap = (int)((int64_t)tcnt * B.cap < B.ucap ? (int64_t)tcnt * B.cap : B.ucap);
    if ((int64_t)uoff + T.ucap > B.upool) {
      T.ucap = 0;
      if (lane == 0) latch_error(B.status, SPH_E_NGB_CAPACITY, -1);
    }
    T.U = B.tile_u + uoff;
    T.p = T.valid ? p : 0;
    T.usize = 0; T.cnt = 0; T.stored = 0;
    int pend = 0;   // candidates waiting in cb (wave-uniform)
    for (int l = 0; l < g.nlev; ++l) {
      const double c = g.cell[l];
      const double R = (hmx + g.hlev[l]) * s1 * (1.0 + 1e-9);
      const double R2 = R * R;
      int lo3[3], ext[3];
      bool wrap[3];
      for (int d = 0; d < 3; ++d) {
        const int dim = g.dims[l][d];
        int l0 = (int)floor((lo[d] - R - g.lo[d]) / c);
        int h0 = (int)floor((hi[d] + R - g.lo[d]) / c);
        wrap[d] = false;
        if (periodic) {
          if (h0 - l0 + 1 >= dim) { l0 = 0; h0 = dim - 1; }
          else wrap[d] = true;
        } else {
          l0 = l0 < 0 ? 0 : l0;
          h0 = h0 > dim - 1 ? dim - 1 : h0;
        }
        lo3[d] = l0;
        ext[d] = h0 >= l0 ? h0 - l0 + 1 : 0;
      }
      const int64_t total = (int64_t)ext[0] * ext[1] * ext[2];
      const uint32_t base = g.base[l];
      for (int64_t q = 0; q < total; q += 64) {
        // phase 1: 64 cells at once; lanes take the block's cells in bit-reversed order so that
        // consecutive union members come from all over the neighbourhood and every target's
        // neighbours spread evenly over the LDS chunks of the pair passes
        const int64_t j = q + (int64_t)(__brev((unsigned)lane) >> 26);
        int32_t s = 0, e = 0;
        if (j < total) {
          const int kx = lo3[0] + (int)(j % ext[0]);
          const int ky = lo3[1] + (int)((j / ext[0]) % ext[1]);
          const int kz = lo3[2] + (int)(j / ((int64_t)ext[0] * ext[1]));
          const int kk[3] = {kx, ky, kz};
          double gap2 = 0.0;
          int cc[3];
          for (int d = 0; d < 3; ++d) {
            if (!periodic || wrap[d]) {
              const double b0 = g.lo[d] + kk[d] * c, b1 = b0 + c;
              const double gd = fmax(0.0, fmax(b0 - hi[d], lo[d] - b1));
              gap2 += gd * gd;
            }
            const int dim = g.dims[l][d];
            cc[d] = wrap[d] ? ((kk[d] % dim) + dim) % dim : kk[d];
          }
          if (gap2 < R2) {
            const uint32_t key = base + (spread3((uint32_t)cc[0]) | (spread3((uint32_t)cc[1]) << 1) |
                                         (spread3((uint32_t)cc[2]) << 2));
            const int32_t s0 = B.cstart[key];
            if (s0 >= 0 && s0 < B.n && B.skeys[s0] == key) {
              s = s0;
              e = B.cend[key];
            }
          }
        }
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
        // phase 2: gather candidates 64 at a time, pre-test against the tile box
        for (int q0 = 0; q0 < Tc; q0 += 64) {
          const int slot = q0 + lane;
          const bool has = slot < Tc;
          double4 pb = make_double4(0.0, 0.0, 0.0, 0.0);
          int32_t b = 0;
          bool pass = false;
          if (has) {
            int lo_i = 0, hi_i = 63;   // last cell with c_o <= slot
            while (lo_i < hi_i) {
              const int mid = (lo_i + hi_i + 1) >> 1;
              if (c_o[mid] <= slot) lo_i = mid;
              else hi_i = mid - 1;
            }
            const int32_t sp = c_s[lo_i] + (slot - c_o[lo_i]);
            b = (int32_t)B.perm[sp];
            pb = B.pos4[b];
            const double ex = fmax(0.0, fabs(min_image(pb.x - cen[0], periodic, box)) - hw[0]);
            const double ey = fmax(0.0, fabs(min_image(pb.y - cen[1], periodic, box)) - hw[1]);
            const double ez = fmax(0.0, fabs(min_image(pb.z - cen[2], periodic, box)) - hw[2]);
            const double Rb = (hmx + pb.w) * s1 * (1.0 + 1e-9);
            pass = ex * ex + ey * ey + ez * ez < Rb * Rb;
          }
          const unsigned long long m = __ballot(pass);
          if (pass) {
            const int k = pend + __popcll(m & lt);
            cb[k] = pb;
            cbi[k] = b;
          }
          pend += __popcll(m);
          __syncthreads();
          if (pend >= 64) {   // phase 3 on a full batch
            run_batch(B, T, cb, cbi, 64, periodic, box, s1);
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
    if (pend > 0) run_batch(B, T, cb, cbi, pend, periodic, box, s1);
    __syncthreads();
    if (T.valid) B.count[p] = T.stored;
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
  uint32_t used = 0;
  HIP_TRY(hipMemcpyAsync(c->drift_host, &c->grid->upool_used, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  used = *c->drift_host;
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
  return SPH_OK;
}

static unsigned tile_grid(int64_t cap_tiles) {
  return (unsigned)(cap_tiles < 65536 ? cap_tiles : 65536);
}

// Candidate-list build: every particle array of the state (and the half-step copies) is reordered
// along the global Morton curve, tiles are cut from that order, particles are binned into the
// multi-level grid and each tile's candidates are collected; the positions and h of this build
// are kept for the drift test.
sph_status sph_rebin(sph_ctx* c, sph_state* st) {
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
    hipLaunchKernelGGL(k_pack_pos, dim3(nb), dim3(kB), 0, s, st->x, st->y, st->z, st->h,
                       (const int32_t*)nullptr, (const StarInfo*)nullptr, n, c->pos4, (float4*)nullptr);
    // tile table for this order
    uint32_t* flag = reinterpret_cast<uint32_t*>(c->tmp);
    hipLaunchKernelGGL(k_tile_flags, dim3(nb), dim3(kB), 0, s, c->keys, c->pos4, n, c->grid,
                       c->p.tile_cut > 0.0 ? c->p.tile_cut : 6.0, flag);
    uint32_t* idx = flag + c->capw;
    if ((e = sph_scan_u32(c, flag, idx, n, &c->grid->ntiles))) return e;
    hipLaunchKernelGGL(k_tile_fill, dim3(nb), dim3(kB), 0, s, flag, idx, n, c->tile_start);
    hipLaunchKernelGGL(k_tile_len, dim3(grid_for(c->cap_tiles, kB)), dim3(kB), 0, s, c->grid, n, c->cap_tiles,
                       c->tile_start, c->tile_cnt, c->cap_s, c->ucap, c->tile_uoff);
    if ((e = sph_scan_u32(c, c->tile_uoff, c->tile_uoff, c->cap_tiles, &c->grid->upool_used))) return e;
    if ((e = ensure_pool(c))) return e;
  }
  hipLaunchKernelGGL(k_level_hmax, dim3(nred), dim3(kB), 0, s, c->pos4, n, c->grid);
  hipLaunchKernelGGL(k_grid_setup2, dim3(1), dim3(1), 0, s, c->grid, c->p.cell_div > 0 ? c->p.cell_div : 2,
                     c->max_cells, c->status);
  hipLaunchKernelGGL(k_keys, dim3(nb), dim3(kB), 0, s, c->pos4, n, c->grid, c->keys, c->vals);
  if ((e = sph_sort_pairs(c, c->keys, c->vals, n))) return e;
  hipLaunchKernelGGL(k_cell_ranges, dim3(nb), dim3(kB), 0, s, c->keys, n, c->cell_start, c->cell_end);
  BuildArgs B;
  B.pos4 = c->pos4; B.n = n; B.grid = c->grid; B.skeys = c->keys; B.perm = c->vals;
  B.cstart = c->cell_start; B.cend = c->cell_end; B.capw = c->capw; B.cap = c->cap_s; B.ucap = c->ucap;
  B.tile_start = c->tile_start; B.tile_cnt = c->tile_cnt; B.tile_uoff = c->tile_uoff; B.upool = c->upool;
  B.tile_u = c->tile_u; B.tile_usize = c->tile_usize; B.nbr16 = c->nbr16s; B.count = c->nbr_count_s;
  B.status = c->status;
  hipLaunchKernelGGL(k_build_tiles, dim3(tile_grid(c->cap_tiles)), dim3(64), 0, s, B);
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

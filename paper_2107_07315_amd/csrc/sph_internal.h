// Internal declarations of the gfx950 SPH particle loop: device helpers shared by the
// kernel files, the context struct and the host launchers.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/sph.h"

#define SPH_MAX_LEV 4
#define SPH_PI 3.14159265358979323846

// Multi-level cell grid.  Particles are binned into levels by smoothing length
// (level l holds h in [hmin 2^l, hmin 2^(l+1)), the top level takes the rest); each level has
// its own uniform grid whose cells are addressed by a Morton code inside a per-level block of
// 2^(3 bits) entries starting at base[l].  All fields are computed on the device.
struct GridInfo {
  unsigned long long enc_lo[3], enc_hi[3];   // order-preserving encodings for atomics
  unsigned long long enc_hmin, enc_hmax;
  unsigned long long hlev_bits[SPH_MAX_LEV]; // max h per level (positive-double bits)
  unsigned long long lev_lo[SPH_MAX_LEV][3], lev_hi[SPH_MAX_LEV][3];  // per-level bounding boxes (encoded)
  double lo[3];
  double hmin, hmax;
  double hlev[SPH_MAX_LEV];
  double cell[SPH_MAX_LEV];
  int32_t dims[SPH_MAX_LEV][3];
  int32_t bits[SPH_MAX_LEV];
  uint32_t base[SPH_MAX_LEV + 1];
  int32_t nlev;
  int32_t periodic;
  double box;
  double skin;          // relative Verlet skin of the current candidate lists (0 or >= 1e-4)
  uint32_t ntiles;      // tiles of the current array order (written on the device)
  uint32_t upool_used;  // union-pool entries reserved by the tiles
  uint32_t nstress;     // tiles holding a particle of type 1 (the stress pass's work list)
};

// Per-star parameters of an ensemble (centre of the star's background, particle mass and
// crust shear-modulus factor).
struct StarInfo {
  double cx, cy, cz, m, mu_pfactor, pad[3];
};

// Device status word: first error code and the particle that raised it.
struct DevStatus {
  int32_t code;
  int32_t particle;
};

__device__ __forceinline__ void latch_error(DevStatus* s, int code, int particle) {
  if (atomicCAS(&s->code, 0, code) == 0) s->particle = particle;
}

// ---- order-preserving double <-> uint64 (for atomic min/max of signed doubles) ------------
__device__ __forceinline__ unsigned long long enc_double(double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ __forceinline__ double dec_double(unsigned long long e) {
  unsigned long long b = (e & 0x8000000000000000ull) ? (e & 0x7fffffffffffffffull) : ~e;
  double d;
  __builtin_memcpy(&d, &b, 8);
  return d;
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 10 bits -> every third bit
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ int particle_level(double h, const GridInfo& g) {
  double ratio = h / g.hmin;
  int l = 0;
  while (l < g.nlev - 1 && ratio >= (double)(2 << l)) ++l;
  return l;
}

// ---- geometry ---------------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R min_image(R d, int periodic, R box) {
  if (periodic) {
    if (d > (R)0.5 * box) d -= box;
    else if (d < -(R)0.5 * box) d += box;
  }
  return d;
}

// Exact FP64 neighbour decision r^2 < (h_a + h_b)^2 with every operation rounded separately in
// the order ((dx dx + dy dy) + dz dz); contraction is switched off for this scope.
__device__ __forceinline__ bool neighbour_test(double dx, double dy, double dz, double ha, double hb) {
#pragma clang fp contract(off)
  double r2 = (dx * dx + dy * dy) + dz * dz;
  double H = ha + hb;
  return r2 < H * H;
}

// r^2 in the rounding order of neighbour_test (for passes that test and then use r).
__device__ __forceinline__ double pair_r2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

// The same test against the skin-widened support (1 + s)(h_a + h_b); s1 = 1 + s.  With s = 0 it
// is bit-identical to neighbour_test.
__device__ __forceinline__ bool candidate_test(double dx, double dy, double dz, double ha, double hb, double s1) {
#pragma clang fp contract(off)
  double r2 = (dx * dx + dy * dy) + dz * dz;
  double H = (ha + hb) * s1;
  return r2 < H * H;
}

// Verlet-skin test: candidate lists built at positions/h `b` with skin s stay a superset of the
// exact lists while every particle satisfies |x - x_b| + max(0, h - h_b) <= s h_b: for a pair
// now within h_a + h_b, the distance at build time was below
// h_a + h_b + (|dx_a| + dh_a) + (|dx_b| + dh_b) <= (1 + s)(h_a,b + h_b,b).  The factor 1 - 1e-9
// absorbs the rounding of both tests (s >= 1e-4).  NaN counts as exceeded.
__device__ __forceinline__ bool skin_exceeded(double dx, double dy, double dz, double h, double4 b, double s) {
  const double d = sqrt(dx * dx + dy * dy + dz * dz);
  const double dh = h > b.w ? h - b.w : 0.0;
  return !(d + dh <= s * b.w * (1.0 - 1e-9));
}

// ---- XCD-aware tile schedule ------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs of the chip (block b runs on XCD b % 8),
// each with its own L2.  Tile kernels give each XCD a contiguous range of tiles, so the
// neighbour records that consecutive (spatially adjacent) tiles share stay in that XCD's L2.
// Launch grids are multiples of SPH_XCD.
#define SPH_XCD 8
__device__ __forceinline__ int64_t xcd_chunk(int64_t ntiles) { return (ntiles + SPH_XCD - 1) / SPH_XCD; }

// ---- fast reciprocal and square root -----------------------------------------------------------
// FP64: hardware rcp/rsq estimates refined by Newton steps (a few ulp, far inside the parity
// tolerance; the neighbour decision never uses them).  FP32: single hardware instructions.
__device__ __forceinline__ double rcp_fast(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  y = fma(fma(-x, y, 1.0), y, y);
  return y;
}
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
// sqrt: the rsq estimate (relative error near 2^-23) after one Newton step has an error near
// 1.5 e^2; the closing step on r = x y squares it again, to rounding level.
__device__ __forceinline__ double sqrt_fast(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  double r = x * y;
  r = fma(0.5 * y, fma(-r, r, x), r);
  return x > 0.0 ? r : 0.0;
}
__device__ __forceinline__ float sqrt_fast(float x) {
  const float r = x * __builtin_amdgcn_rsqf(x);
  return x > 0.0f ? r : 0.0f;
}

// ---- Wendland kernels with support 2 h_ab: W and F such that grad_a W = F (x_a - x_b) -------
template <typename R>
__device__ __forceinline__ void wendland(int kernel, R r, R hab, R& W, R& F) {
  R ih = rcp_fast(hab);
  R q = r * ih;
  if (q >= (R)2) { W = 0; F = 0; return; }
  R t = (R)1 - (R)0.5 * q;
  R ih2 = ih * ih, ih3 = ih2 * ih, ih5 = ih3 * ih2;
  if (kernel == SPH_WC4) {
    R t2 = t * t, t5 = t2 * t2 * t;
    W = (R)(495.0 / (256.0 * SPH_PI)) * ih3 * t5 * t * ((R)1 + (R)3 * q + (R)(35.0 / 12.0) * q * q);
    F = -(R)(1155.0 / (128.0 * SPH_PI)) * ih5 * t5 * ((R)1 + (R)2.5 * q);
  } else {
    R t3 = t * t * t;
    W = (R)(21.0 / (16.0 * SPH_PI)) * ih3 * t3 * t * ((R)1 + (R)2 * q);
    F = -(R)(105.0 / (16.0 * SPH_PI)) * ih5 * t3;
  }
}

template <typename R>
__device__ __forceinline__ R wendland_self(int kernel, R h) {
  R ih = (R)1 / h;
  R ih3 = ih * ih * ih;
  return kernel == SPH_WC4 ? (R)(495.0 / (256.0 * SPH_PI)) * ih3 : (R)(21.0 / (16.0 * SPH_PI)) * ih3;
}

// ---- tabulated equation of state -------------------------------------------------------------
// Bilinear interpolation of ln P and ln c_s^2 on the uniform (ln rho, ln u) grid.  Returns non-zero
// outside the table or on non-finite nodes; `cell` = i * (nu - 1) + j of the enclosing cell.
__device__ __forceinline__ bool table_bilinear(const double* __restrict__ T, int64_t o, int nu, double a, double b,
                                               double& v) {
  const double f00 = T[o], f01 = T[o + 1], f10 = T[o + nu], f11 = T[o + nu + 1];
  if (!isfinite(f00) || !isfinite(f01) || !isfinite(f10) || !isfinite(f11)) return false;
  v = (1.0 - a) * ((1.0 - b) * f00 + b * f01) + a * ((1.0 - b) * f10 + b * f11);
  return true;
}
__device__ __forceinline__ int eos_table_ln(const sph_params& p, double lnr, double lnu, double& lp, double& lc,
                                            int64_t& cell) {
  const double fr = (lnr - p.tab_lnr0) / p.tab_dlnr;
  const double fu = (lnu - p.tab_lnu0) / p.tab_dlnu;
  if (!(fr >= 0.0) || !(fu >= 0.0) || fr > (double)(p.tab_nr - 1) || fu > (double)(p.tab_nu - 1)) return 1;
  int i = (int)floor(fr), j = (int)floor(fu);
  i = i > p.tab_nr - 2 ? p.tab_nr - 2 : i;
  j = j > p.tab_nu - 2 ? p.tab_nu - 2 : j;
  const double a = fr - (double)i, b = fu - (double)j;
  const int64_t o = (int64_t)i * p.tab_nu + j;
  cell = (int64_t)i * (p.tab_nu - 1) + j;
  if (!table_bilinear(p.tab_lnP, o, p.tab_nu, a, b, lp) || !table_bilinear(p.tab_lncs2, o, p.tab_nu, a, b, lc))
    return 1;
  return 0;
}

// ---- static isotropic background ------------------------------------------------------------
struct Metric {
  double alpha, dalpha, psi, dpsi, n[3];
};

__device__ __forceinline__ Metric metric_at(const sph_params& p, double x, double y, double z) {
  Metric g;
  double rb = sqrt(x * x + y * y + z * z);
  if (rb > 0.0) {
    double ir = 1.0 / rb;
    g.n[0] = x * ir; g.n[1] = y * ir; g.n[2] = z * ir;
  } else {
    g.n[0] = g.n[1] = g.n[2] = 0.0;
  }
  double Rbar = p.bg_dr * (double)(p.bg_n - 1);
  if (rb <= Rbar) {
    double t = rb / p.bg_dr;
    int i = (int)floor(t);
    if (i > p.bg_n - 2) i = p.bg_n - 2;
    double f = t - (double)i;
    const double* T = p.bg;
    int nb = p.bg_n;
    g.alpha = (1.0 - f) * T[i] + f * T[i + 1];
    g.dalpha = (1.0 - f) * T[nb + i] + f * T[nb + i + 1];
    g.psi = (1.0 - f) * T[2 * nb + i] + f * T[2 * nb + i + 1];
    g.dpsi = (1.0 - f) * T[3 * nb + i] + f * T[3 * nb + i + 1];
  } else {
    double a = p.bg_M / (2.0 * rb);
    g.psi = 1.0 + a;
    g.alpha = (1.0 - a) / (1.0 + a);
    g.dpsi = -a / rb;
    g.dalpha = 2.0 / ((1.0 + a) * (1.0 + a)) * a / rb;
  }
  return g;
}

// ---- symmetric 3x3 helpers (6 comps xx,yy,zz,xy,xz,yz) ----------------------------------------
__device__ __forceinline__ double lambda_max_sym(double xx, double yy, double zz, double xy, double xz,
                                                 double yz) {
  double q = (xx + yy + zz) * (1.0 / 3.0);
  double off2 = xy * xy + xz * xz + yz * yz;
  double a = xx - q, b = yy - q, c = zz - q;
  double p2 = a * a + b * b + c * c + 2.0 * off2;
  if (!(p2 > 0.0)) return q;
  double p = sqrt(p2 / 6.0);
  double ip = 1.0 / p;
  a *= ip; b *= ip; c *= ip;
  double e = xy * ip, f = xz * ip, g = yz * ip;
  double det = a * (b * c - g * g) - e * (e * c - g * f) + f * (e * g - b * f);
  double r = 0.5 * det;
  r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
  return q + 2.0 * p * cos(acos(r) * (1.0 / 3.0));
}

// von Mises scaling: f = min(Y0^2/sigma_v^2, 1) (PAPER) or min(Y0/sigma_v, 1) (RADIAL)
__device__ __forceinline__ void yield_scale(int mode, double Y0, double* s) {
  double J = s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
  double sv2 = 1.5 * J;
  if (!(sv2 > 0.0)) return;
  double f = (mode == SPH_YIELD_RADIAL) ? Y0 / sqrt(sv2) : Y0 * Y0 / sv2;
  if (f < 1.0)
    for (int k = 0; k < 6; ++k) s[k] *= f;
}

// ---- context ----------------------------------------------------------------------------------
struct SortScratch {
  uint32_t *keys_alt, *vals_alt;
  uint32_t* hist;        // 256 * max_blocks
  uint32_t* rowtot;      // 256 digit totals / offsets
  unsigned long long* partial;  // per-block reduction partials of the grid set-up (8 per block)
  uint32_t* scan_bsum;   // generic scan: per-block sums
  int64_t scan_cap;      // blocks of 1024 the generic scan can take
  int max_blocks;
};

struct StageTimer {
  std::vector<hipEvent_t> ev;   // pairs (start, stop)
  size_t used = 0;
};

struct sph_ctx {
  sph_params p;
  hipStream_t stream;
  int64_t capacity;
  int64_t n;            // particles at the last build
  int device;
  int32_t gen;          // stage order: 1 cells, 2 density, 3 stress, 4 forces
  bool lists_valid;     // candidate lists match the current n, order and parameters
  uint32_t graph_epoch; // bumped whenever a pointer or parameter that kernels capture changes
  hipGraphExec_t g_eval;   // captured density, epilogue, stress rate, forces
  hipGraphExec_t g_drift;  // captured flag clear, kick-drift with skin test, flag copy
  hipGraphExec_t g_chain;  // the same with the previous step's final kick fused in
  const double* g_x;       // key of the captured graphs: state, size, dt, epoch
  int64_t g_n;
  double g_dt;
  uint32_t g_epoch;
  uint32_t check_id;    // value a failed drift test writes when no step number applies (1)
  uint32_t* drift_flag; // device word: largest check id (step number) that saw a skin violation
  uint32_t* drift_host; // pinned host copy
  uint32_t eval_seq;    // step number of a run-ahead evaluation being queued (0: none)
  bool pos_deferred;    // st->x, y, z, h lag behind pos4 (kicks inside a multi-step call)
  hipEvent_t step_ev[2];   // run-ahead steps: the skin-test word of a step has reached the host
  int64_t rebuilds;
  double4* pos_build;   // x, y, z, h at the last candidate-list build
  // grid and sort
  GridInfo* grid;       // device
  uint32_t *keys, *vals;  // cell-sorted keys and permutation (sorted position -> particle index)
  int2* cell_se;        // per cell [start, end) in the cell-sorted order; cleared at every build
  int64_t max_cells;
  double4* pos_sorted;  // x, y, z, h in the cell-sorted order (candidate gathers of the build)
  SortScratch sort;
  // tile neighbour lists: tile t = particles [tile_start[t], tile_start[t] + tile_cnt[t]) of the
  // array order (at most 64; the array is kept along the global Morton curve); U_t = tile_u +
  // tile_uoff[t] holds the union of the tile's candidates (particle indices).  Candidate entry k
  // of particle p is the local index into U_t stored at nbr16s[((k/8)*capw + p)*8 + k%8] (groups
  // of 8 entries per lane, so a lane fetches 8 entries with one 16-byte load and a wave's load is
  // one contiguous 1 KB); the exact lists that the density pass extracts use the same layout in
  // nbr16 with nbr_count.
  int32_t* tile_start;
  int32_t* tile_cnt;
  uint32_t* tile_uoff;  // tile t owns tile_u[tile_uoff[t], + min(ucap, cnt * cap_s))
  int32_t* tile_u;
  int64_t upool;        // entries of tile_u
  int64_t cap_tiles;
  int32_t* tile_usize;
  int32_t* stress_tiles;  // tiles with a type-1 particle, in tile order (nstress of them)
  uint32_t* tile_st;      // per tile: 1 if a particle or a union member is of type 1
  uint16_t* nbr16;      // exact lists, one per slot (particle * lanes + sub-index)
  int32_t* nbr_count;   // exact neighbours per particle
  int32_t* nbr_count_sl;  // entries per slot list
  uint16_t* nbr16s;
  int32_t* nbr_count_s;
  int64_t capw;         // capacity rounded up to 64
  int32_t cap;          // exact-list capacity
  int32_t cap_s;        // candidate-list capacity
  int32_t ucap;
  // packed gather records (FP64 and FP32 variants)
  double4* pos4;        // x, y, z, h
  double4* fv;          // vx, vy, vz, alpha cs (alpha: viscosity coefficient)
  double2* fa;          // P/D^2, D (negative D marks a particle that carries deviatoric stress)
  double* sig;          // S/D^2, 6*cap
  float4* pos4f;        // x, y, z (relative to the star centre), h/2
  float4* fvf;          // vx, vy, vz, alpha cs/2
  float2* faf;          // P/D^2, D/2 (negative: carries deviatoric stress)
  float* sigf;
  // internal per-particle fields
  double *mu, *Y0, *B, *sdot;
  double4* tovf;        // per particle: fixed-background force coefficients (k_P, B_x, B_y, B_z)
  // half-step copies for kick-drift-kick
  double* half;         // 10*cap: vx, vy, vz, u, S[6]
  double* tmp;          // permutation staging, 8 bytes * cap
  // ensemble
  StarInfo* stars;      // device, may be null
  int32_t nstars;
  // status
  DevStatus* status;    // device
  int32_t err_particle = -1;   // particle of the error returned by the last failing sph_sync
  // timing
  int32_t timing;
  StageTimer timers[6];
  // EoS surrogate network (allocated on first use)
  struct MlpState* mlp;
  // EoS table owned by the context (sph_eos_table_create): lnP then lncs2, nr * nu each
  double* tab_own;
  int32_t tab_own_nr, tab_own_nu;
  double tab_own_g[4];   // lnr0, dlnr, lnu0, dlnu
  // reason for the last failing call (sph_last_error_detail)
  char detail[256];
  // device address of the statistics scratch array on this context's device
  unsigned long long* stats_scratch;
  // per-block partial sums of sph_diagnostics (allocated on first use)
  double* diag_part;
  // method variants
  double* dsum;         // summation density while D is integrated (continuity density)
  double* dDdt;         // sum m (v_a - v_b) . grad_a W of the last evaluation
  double* xcoef;        // per particle, SoA 5 x capacity: first-law energy e0, e1, e2; dP/dt row q, k
  // time-step words (device): [0..2] Courant steps committed by evaluations (slot = step % 3),
  // [3] simulated time, [5] dt of the step in progress
  double* dtw;
  double* dtpart;       // per-block minima of h / (c_L + |v|) of the last density epilogue
  int32_t* eos_list;    // particles the EoS network serves in the current evaluation (split epilogue)
  int32_t* eos_list_n;
  int eos_blocks;       // blocks of that epilogue that wrote dtpart (0: none)
  bool stress_heavy;    // more than half of the tiles hold a type-1 particle (last list build)
  int64_t steps_done;   // steps completed since sph_create (slot bookkeeping of the Courant steps)
  bool adaptive;        // inside an sph_step call with Courant steps
  bool eval_in_step;    // an evaluation queued by sph_step (the lagged dP/dt reads that step's dt)
};

// Records a human-readable reason for a failing return (sph_last_error_detail; c may be NULL for
// calls without a context) and returns e.
sph_status note(sph_ctx* c, sph_status e, const char* fmt, ...);

// ---- host launchers (one per kernel file) ------------------------------------------------------
sph_status sph_sort_pairs(sph_ctx* c, uint32_t* keys, uint32_t* vals, int64_t n);
// outputs_recomputed: the outputs (D, rho, P, c_s, accelerations, du/dt, dS/dt) are recomputed
// before they are next read, so they are not reordered
sph_status sph_rebin(sph_ctx* c, sph_state* st, bool outputs_recomputed);
sph_status launch_drift_check(sph_ctx* c, sph_state* st);
sph_status launch_flag_clear(sph_ctx* c);
sph_status launch_density(sph_ctx* c, sph_state* st);   // pair loop
sph_status launch_exact_lists(sph_ctx* c);               // exact lists of the last evaluation (export)
bool exact_lists_written(const sph_ctx* c);              // whether the density pass writes them
sph_status launch_eos(sph_ctx* c, sph_state* st);       // per-particle epilogue
sph_status launch_stress(sph_ctx* c, sph_state* st);
sph_status launch_forces(sph_ctx* c, sph_state* st);
// check: 0 no skin test, else the step's number since drift_flag was cleared (a smaller non-zero
// value already in the flag, left by an earlier step's failed test, cancels the kick)
// deferred: positions and h are read from and written to pos4 only (st->x, y, z, h lag behind
// until launch_unpack_pos)
// slot: the Courant-step word the kick reads (adaptive steps), or -1 for the fixed dt
sph_status launch_kick_drift(sph_ctx* c, sph_state* st, double dt, uint32_t check, bool deferred = false,
                             int slot = -1);
sph_status launch_kick_final(sph_ctx* c, sph_state* st, double dt, int slot = -1);
// the final kick of one step fused with the kick-drift of the next (inside a multi-step call)
sph_status launch_kick_final_drift(sph_ctx* c, sph_state* st, double dt, uint32_t check, bool deferred = false,
                                   int slot_fin = -1, int slot_drift = -1);
// st->x, y, z, h from pos4 (after deferred kicks)
sph_status launch_unpack_pos(sph_ctx* c, sph_state* st);
sph_status launch_pack(sph_ctx* c, sph_state* st);
sph_status launch_modify_energy(sph_ctx* c, sph_state* st, const double* u_of_r, int32_t nr, double dr);
// after an evaluation's epilogue: dtw[slot] = cfl * the minimum over its per-block partials
sph_status launch_dt_commit(sph_ctx* c, int slot);
sph_status launch_dt_init(sph_ctx* c);
// half-step copies per particle: vx, vy, vz, u, S[6], D (continuity density)
#define SPH_HALF_FIELDS 11
sph_status sph_count_stats(sph_ctx* c, sph_list_stats* out);
// looks up (once per device, with that device current) the device address of the statistics
// scratch array and stores it in the context
sph_status stats_scratch_init(sph_ctx* c);
sph_status sph_scan_u32(sph_ctx* c, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total);
struct MlpView;
bool mlp_view(const sph_ctx* c, MlpView* v);   // false if no trained network is loaded
void mlp_free(sph_ctx* c);
int64_t mlp_trusted_cells(const sph_ctx* c);   // EoS-table cells the network may serve

enum { TIMER_CELLS = 0, TIMER_DENSITY = 1, TIMER_STRESS = 2, TIMER_FORCES = 3, TIMER_KDK = 4, TIMER_EOS = 5 };
void timer_begin(sph_ctx* c, int which);
void timer_end(sph_ctx* c, int which);

__host__ __device__ __forceinline__ int64_t nbr_index(int64_t k, int64_t p, int64_t capw) {
  return (((k >> 3) * capw + p) << 3) + (k & 7);
}

// Lanes per target of the pair passes, and the entries of one slot list: lanes L share a
// particle's at most 2 cap candidates in turn, so a slot receives at most ceil(2 cap / L) exact
// hits (and the particle's list at most cap).  Slot s of the exact lists is entry k at
// nbr_index(k, s, capw * L).
__host__ __device__ __forceinline__ int pass_lanes(const sph_params& p) { return p.lanes > 0 ? p.lanes : 4; }
// Tile cut in smoothing lengths (the measured best with 4 lanes per target on the 2M star)
__host__ __device__ __forceinline__ double tile_cut_of(const sph_params& p) { return p.tile_cut > 0.0 ? p.tile_cut : 10.0; }
__host__ __device__ __forceinline__ int slot_capacity(int cap, int L) {
  const int c = (2 * cap + L - 1) / L;
  return ((c < cap ? c : cap) + 7) / 8 * 8;
}
// Candidate lists use the same slots: candidate k of a particle is entry k / L of slot k % L.
__host__ __device__ __forceinline__ int cand_slot_capacity(int cap_s, int L) { return ((cap_s + L - 1) / L + 7) / 8 * 8; }
__host__ __device__ __forceinline__ int64_t slot_entries_max(int cap) {   // per particle, over L
  int64_t m = 0;
  for (int L = 1; L <= 4; L *= 2) m = m > (int64_t)L * slot_capacity(cap, L) ? m : (int64_t)L * slot_capacity(cap, L);
  return m;
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return SPH_E_HIP;             \
  } while (0)

static inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

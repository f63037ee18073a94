// Pair passes of the particle loop: density (+ EoS epilogue and the exact neighbour decision),
// velocity gradient / stress rate, and momentum/energy forces (+ fixed-background epilogue).
//
// One workgroup = one wavefront = one tile of at most 64 consecutive particles (one lane per
// target).  The tile's neighbour union U is streamed through LDS in chunks of CH packed records
// (loaded by the whole wave); each lane walks its ascending 16-bit local list and reads its
// neighbours' records from LDS.  The walk is software-pipelined: list entries arrive 8 per
// 16-byte load one group ahead of use, and the next neighbour's LDS record is read before the
// current pair's arithmetic.  Kernel type and periodicity are compile-time parameters so the
// inner loops are straight-line code.  The pair arithmetic is templated on the pair precision
// R: double in the FP64 path, float in the mixed-precision path; epilogues (metric, EoS, GR
// terms) are FP64.
#include <type_traits>

#include "sph_internal.h"
#include "sph_mlp.h"

namespace {

constexpr int kB = 256;

// minimum image with selects (same result as min_image, no branches)
template <bool PER, typename T>
__device__ __forceinline__ T wrap_sel(T d, T box, T half) {
  if constexpr (PER) {
    const T lo = d - box, hi = d + box;
    return d > half ? lo : (d < -half ? hi : d);
  } else {
    return d;
  }
}

// Wendland kernels with q = r / h_ab (1/h_ab = ih) and t = max(1 - q/2, 0), in the pair loops
// without their constant factor, which the passes apply once to the sums:
//   C4: W = kW h^-3 t^6 (1 + 3q + 35/12 q^2),  F = kF h^-5 t^5 (1 + 5q/2);
//   C2: W = kW h^-3 t^4 (1 + 2q),              F = kF h^-5 t^3,
// with grad_a W = F (x_a - x_b); t^k / h^k is formed as (t / h)^k.  Outside the support t = 0,
// so both vanish there without a test.
template <int KER>
constexpr double kern_W_const() { return KER == SPH_WC4 ? 495.0 / (256.0 * SPH_PI) : 21.0 / (16.0 * SPH_PI); }
template <int KER>
constexpr double kern_F_const() { return KER == SPH_WC4 ? -1155.0 / (128.0 * SPH_PI) : -105.0 / (16.0 * SPH_PI); }
template <typename R, int KER>
__device__ __forceinline__ R kern_W_unit(R r, R ih) {
  const R q = r * ih;
  const R t = fmax(fma((R)-0.5, q, (R)1), (R)0);
  if constexpr (KER == SPH_WC4) {
    const R w = t * t * ih;   // t^6 / h^3 = w^3
    return w * w * w * fma(fma((R)(35.0 / 12.0), q, (R)3), q, (R)1);
  } else {
    const R w = t * ih;       // t^4 / h^3 = w^3 t
    return w * w * w * t * fma((R)2, q, (R)1);
  }
}
// One eighth of it from iH = 1 / (h_a + h_b) = ih / 2, which needs no halving of h_a + h_b:
// p = r iH = q / 2, and each factor ih of the unit form becomes iH (a power-of-2 scaling, so the
// value is exactly kern_W_unit / 8).
template <typename R, int KER>
__device__ __forceinline__ R kern_W_unit_eighth(R r, R iH) {
  const R p = r * iH;
  const R t = fmax((R)1 - p, (R)0);
  if constexpr (KER == SPH_WC4) {
    const R w = t * t * iH;
    return w * w * w * fma(fma((R)(35.0 / 3.0), p, (R)6), p, (R)1);
  } else {
    const R w = t * iH;
    return w * w * w * t * fma((R)4, p, (R)1);
  }
}
template <typename R, int KER>
__device__ __forceinline__ R kern_F_unit(R r, R ih) {
  const R q = r * ih;
  const R t = fmax(fma((R)-0.5, q, (R)1), (R)0);
  const R w = t * ih;
  if constexpr (KER == SPH_WC4) {
    const R w2 = w * w;       // t^5 / h^5 = w^5
    return w2 * w2 * w * fma((R)2.5, q, (R)1);
  } else {
    return w * w * w * (ih * ih); // t^3 / h^5
  }
}
// |d| from r^2 in FP32: the hardware square root (about 1 ulp; 0 at 0)
__device__ __forceinline__ float sqrt_hw(float x) { return __builtin_amdgcn_sqrtf(x); }

template <typename R> struct Rec;
// Record scale: the FP64 records hold h, alpha c_s and D; the FP32 ones hold h/2, alpha c_s/2 and
// D/2 (exact halvings), so the pair means 0.5 (h_a + h_b), 0.5 alpha (c_a + c_b), 0.5 (D_a + D_b)
// are HS times the sum of the two record values and HS = 1 saves the multiply in FP32 (alpha: the
// viscosity coefficient, which multiplies the mean sound speed wherever it is used).
template <> struct Rec<double> {
  static constexpr double HS = 0.5;
  using P4 = double4;
  using V4 = double4;
  using A2 = double2;
  static constexpr int CH_D = 256;   // LDS records per chunk and wave: density 8 KB
  static constexpr int CHMAX_D = 1024;  // per workgroup: 32 KB + 8 KB of list staging, 4 workgroups per CU
  static constexpr int CH_S = 128;   // stress 8 KB
  static constexpr int CH_F = 128;   // forces 10 KB
};
template <> struct Rec<float> {
  static constexpr float HS = 1.0f;
  using P4 = float4;
  using V4 = float4;
  using A2 = float2;
  static constexpr int CH_D = 384;   // density records: FP32 tile-relative (x, y, z, h), 6 KB
  static constexpr int CHMAX_D = 1280;   // per workgroup: 20 KB + 8 KB of list staging, 5 workgroups per CU
  static constexpr int CH_S = 256;
  static constexpr int CH_F = 256;
  static constexpr int CH_FS = 128;   // forces with S/D^2 in LDS too (64 bytes a record): 32 KB
};

struct PassArgs {
  sph_params p;
  int64_t n;
  int cap, ucap;
  int64_t capw;
  const GridInfo* __restrict__ grid;
  const int32_t* __restrict__ tile_start;
  const int32_t* __restrict__ tile_cnt;
  const uint32_t* __restrict__ tile_uoff;
  const int32_t* __restrict__ tile_u;
  const int32_t* __restrict__ tile_usize;
  const int32_t* __restrict__ stress_tiles;
  const uint16_t* __restrict__ nbr16;    // exact lists (written by the density pass), one per slot
  const int32_t* __restrict__ cnt_sl;   // entries per slot; slot = particle * lanes + sub-index
  int cap_sl;                           // entries a slot holds
  const uint16_t* __restrict__ nbr16s;   // candidate lists of the last build
  const int32_t* __restrict__ cnt_s;
  // the stress and force passes walk the candidate lists instead of the exact ones (the pair
  // terms vanish beyond the support, so the sums are the same; the density pass then writes no
  // exact lists)
  int cand_walk;
  const uint32_t* __restrict__ tile_st;   // per tile: a particle or union member of type 1 (or null)
  const int32_t* __restrict__ star;
  const StarInfo* __restrict__ stars;
  DevStatus* status;
  MlpView mlp;          // EoS surrogate (eos = MLP with a loaded network)
  int has_mlp;
  // run-ahead evaluation of step number seq: cancelled when the skin-test word `stop` holds a
  // step number in [1, seq] (that step's drift broke the skin bound); stop == nullptr: never
  const uint32_t* stop;
  uint32_t seq;
};

constexpr int kNone = 0x7fffffff;

// Per-lane walk over a slot list stored as 16-byte groups of 8 16-bit local indices (group g at
// base + g * gstride).  The group after the current one is always in flight (8 entries ahead);
// the current group is consumed by funnel shifts.
struct TileWalk {
  int64_t p, a;
  bool valid;
  int usize, cnt, k, next;
  const uint4* gnext;      // the group after nxt
  int64_t gstride;
  uint4 cur, nxt;
  const int32_t* U;
  // target t of the tile (a = p for a valid target, 0 otherwise)
  __device__ __forceinline__ void begin(const PassArgs& A, int64_t tile, int t) {
    p = (int64_t)A.tile_start[tile] + t;
    valid = t < A.tile_cnt[tile];
    a = valid ? p : 0;
    usize = A.tile_usize[tile];
    U = A.tile_u + A.tile_uoff[tile];
  }
  __device__ __forceinline__ void start(const uint4* base, int64_t stride, int count) {
    gstride = stride;
    cnt = count;
    k = 0;
    cur = make_uint4(0u, 0u, 0u, 0u);
    nxt = cur;
    if (cnt > 0) cur = base[0];
    if (cnt > 8) nxt = base[gstride];
    gnext = base + 2 * gstride;
    next = cnt > 0 ? (int)(cur.x & 0xffffu) : kNone;
  }
  __device__ __forceinline__ void advance() {
    ++k;
    if ((k & 7) == 0) {
      cur = nxt;
      if (k + 8 < cnt) {
        nxt = *gnext;
        gnext += gstride;
      }
    } else {
      cur.x = __builtin_amdgcn_alignbit(cur.y, cur.x, 16u);
      cur.y = __builtin_amdgcn_alignbit(cur.z, cur.y, 16u);
      cur.z = __builtin_amdgcn_alignbit(cur.w, cur.z, 16u);
      cur.w >>= 16;
    }
    next = k < cnt ? (int)(cur.x & 0xffffu) : kNone;
  }
};

// Walk of a whole slot list when the tile's union fits one LDS chunk: f(local index) for every
// entry, a 16-byte group (8 entries) per round with the entries taken at fixed positions (no
// shifts or per-entry boundary tests), the next group in flight during the current one's 8 pairs.
template <typename F>
__device__ __forceinline__ void walk_groups(const uint4* base, int64_t gstride, int cnt, F&& f) {
  uint4 g = make_uint4(0u, 0u, 0u, 0u);
  if (cnt > 0) g = base[0];
  const uint4* gp = base + gstride;
  for (int k0 = 0; k0 < cnt; k0 += 8) {
    uint4 nx = g;
    if (k0 + 8 < cnt) nx = *gp;
    gp += gstride;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t w = i < 2 ? g.x : (i < 4 ? g.y : (i < 6 ? g.z : g.w));
      if (k0 + i < cnt) f((int)((i & 1) ? (w >> 16) : (w & 0xffffu)));
    }
    g = nx;
  }
}

// Software-pipelined walk of a whole slot list when the tile's union sits in LDS as one chunk.
// Every lane of the wave runs the wave's longest list (cmax, wave-uniform), so the body is
// straight-line code with no per-entry branch: entries past the lane's own count read the records
// of LDS slot `pad`, a sentinel particle far from every target (its pair terms are exactly zero,
// with no overflow), and pass no list entry on.  The records of the next entry are read from LDS
// (load(j)) before the current entry's arithmetic (f(loc, rec)); the next 16-byte group of 8
// entries is read from memory one group ahead; group_end() runs after every group of 8.
template <typename Ld, typename F, typename G>
__device__ __forceinline__ void walk_groups_pf(const uint4* base, int64_t gstride, int cnt, int cmax, int pad,
                                               Ld&& load, F&& f, G&& group_end) {
  auto ent = [](const uint4& q, int i) -> int {
    const uint32_t w = i < 2 ? q.x : (i < 4 ? q.y : (i < 6 ? q.z : q.w));
    return (int)((i & 1) ? (w >> 16) : (w & 0xffffu));
  };
  uint4 g = make_uint4(0u, 0u, 0u, 0u);
  if (cnt > 0) g = base[0];
  const uint4* gp = base + gstride;
  auto rec = load(cnt > 0 ? ent(g, 0) : pad);
  for (int k0 = 0; k0 < cmax; k0 += 8) {
    uint4 nx = g;
    if (k0 + 8 < cnt) nx = *gp;
    gp += gstride;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (k0 + i >= cmax) break;   // wave-uniform
      const int k1 = k0 + i + 1;
      const auto nrec = load(k1 < cnt ? (i < 7 ? ent(g, i + 1) : ent(nx, 0)) : pad);
      f(ent(g, i), rec);
      rec = nrec;
    }
    group_end();
    g = nx;
  }
}

// Largest value of v over the wave, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return __builtin_amdgcn_readfirstlane(v);
}

// Sum over the L adjacent lanes that share a target (every one of them receives the sum).
template <int L, typename T>
__device__ __forceinline__ T lane_group_sum(T v) {
#pragma unroll
  for (int off = 1; off < L; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ bool cancelled(const PassArgs& A) {
  if (!A.stop) return false;
  const uint32_t f = *A.stop;
  return f != 0u && f <= A.seq;
}
// work-item counts of the passes (zero for a cancelled evaluation)
// Stages union members [c0, c0 + CH) of a tile into LDS with NT threads: each thread loads the
// indices of its (at most ceil(CH / NT)) members first and then all their records, so staging
// waits for two memory latencies instead of two per member.  load(b) returns the records of
// particle b, put(j, r) stores them to LDS slot j.
template <int NT, int CH, typename Load, typename Put>
__device__ __forceinline__ void stage_union(const int32_t* __restrict__ U, int c0, int usize, Load&& load,
                                            Put&& put) {
  constexpr int NJ = (CH + NT - 1) / NT;
  using Recs = decltype(load(0));
  int32_t b[NJ];
#pragma unroll
  for (int k = 0; k < NJ; ++k) {
    const int j = (int)threadIdx.x + k * NT;
    b[k] = (j < CH && c0 + j < usize) ? U[c0 + j] : -1;
  }
  Recs r[NJ];
#pragma unroll
  for (int k = 0; k < NJ; ++k)
    if (b[k] >= 0) r[k] = load(b[k]);
#pragma unroll
  for (int k = 0; k < NJ; ++k)
    if (b[k] >= 0) put((int)threadIdx.x + k * NT, r[k]);
}

// The list a stress or force lane walks (slot = particle * L + sub-index) and its length: the exact
// list written by the density pass, or the candidate list of the last build (candidate k of a
// particle is entry k / L of slot k % L).
template <int L>
__device__ __forceinline__ const uint4* pass_list(const PassArgs& A, int64_t slot) {
  return reinterpret_cast<const uint4*>(A.cand_walk ? A.nbr16s : A.nbr16) + slot;
}
template <int L>
__device__ __forceinline__ int pass_count(const PassArgs& A, int64_t p, int sub, int64_t slot) {
  if (!A.cand_walk) return A.cnt_sl[slot];
  const int total = A.cnt_s[p];
  return total > sub ? (total - sub + L - 1) / L : 0;
}

__device__ __forceinline__ int64_t num_tiles(const PassArgs& A) {
  const int64_t nt = (int64_t)A.grid->ntiles;
  return cancelled(A) ? 0 : nt;
}

__device__ __forceinline__ double particle_mass(const PassArgs& A, int64_t a) {
  return (A.star && A.stars) ? A.stars[A.star[a]].m : A.p.m;
}
__device__ __forceinline__ void star_centre(const PassArgs& A, int64_t a, double& cx, double& cy, double& cz) {
  cx = cy = cz = 0.0;
  if (A.star && A.stars) {
    StarInfo s = A.stars[A.star[a]];
    cx = s.cx; cy = s.cy; cz = s.cz;
  }
}

// ---- equation of state -------------------------------------------------------------------------
// Table (and, where the surrogate is not trusted, the MLP mode): bilinear ln P, ln c_s^2.
__device__ __forceinline__ int eos_eval(const sph_params& p, double rho, double u, double& P, double& cs2) {
  if (p.eos == SPH_EOS_TABLE || p.eos == SPH_EOS_MLP) {
    if (!(rho > 0.0) || !(u > 0.0)) return SPH_E_EOS_DOMAIN;
    double lp, lc;
    int64_t cell;
    if (eos_table_ln(p, log(rho), log(u), lp, lc, cell)) return SPH_E_EOS_DOMAIN;
    P = exp(lp);
    cs2 = exp(lc);
    return 0;
  }
  P = (p.gamma - 1.0) * rho * u;
  cs2 = (p.background == SPH_TOV) ? p.gamma * P / (rho * (1.0 + u + P / rho)) : p.gamma * P / rho;
  return 0;
}

// Whether (rho, u) lies in a table cell the network's trust mask accepts.
__device__ __forceinline__ bool mlp_trusted_at(const MlpView& M, const sph_params& p, double rho, double u) {
  if (!M.trust || !(rho > 0.0) || !(u > 0.0)) return false;
  const double fr = (log(rho) - p.tab_lnr0) / p.tab_dlnr, fu = (log(u) - p.tab_lnu0) / p.tab_dlnu;
  if (!(fr >= 0.0 && fu >= 0.0 && fr <= (double)(p.tab_nr - 1) && fu <= (double)(p.tab_nu - 1))) return false;
  int i = (int)floor(fr), j = (int)floor(fu);
  i = i > p.tab_nr - 2 ? p.tab_nr - 2 : i;
  j = j > p.tab_nu - 2 ? p.tab_nu - 2 : j;
  return M.trust[(int64_t)i * (p.tab_nu - 1) + j] != 0;
}

// ---- density --------------------------------------------------------------------------------
struct DensOut {
  double *D, *rho, *P, *cs, *mu, *Y0, *B;   // D: where the pair loop writes the summation density
  const double* Dread;   // the D the epilogue uses: the summed one, or the integrated one (continuity)
  double* xcoef;         // SoA 5 x xs: first-law energy e0, e1, e2; dP/dt row q, k
  int64_t xs;
  double* dtpart;        // per-block minimum of h / (c_L + |v|) (Courant step), or nullptr
  const double* dtw;     // time-step words (dtw[5]: dt of the step in progress)
  int in_step;           // the evaluation belongs to a step (the lagged dP/dt applies)
  double4* tov;     // fixed-background force coefficients (TOV background only)
  double4* fv;
  double2* fa;
  double* sig;
  float4* fvf;
  float2* faf;
  float* sigf;
};

// Appends 16-bit local indices to a lane's exact list (the layout TileWalk reads).  Entries go to
// a ring of RB 16-byte rows of the lane's own in LDS (written at every candidate, kept only on a
// hit); the rows are stored as 16-byte groups only when the ring is full or at the end.  Stores
// in the pair loop would make each wait for a list load also wait for them (one counter tracks
// both), so a lane with at most 8 RB hits stores nothing until the loop is over.  No other lane
// touches the ring, so no barrier is needed.
template <int RB>
struct ListWriter {
  uint4* gp;          // where the lane's next unstored group goes
  int64_t gstride;    // uint4 between consecutive groups
  uint16_t* ring;     // RB rows of 8 entries (16-byte aligned)
  int cap;
  int n;              // entries appended
  int stored;         // groups stored
  __device__ __forceinline__ void init(uint4* base, int64_t stride, uint16_t* r, int cap_) {
    gp = base;
    gstride = stride;
    ring = r;
    cap = cap_;
    n = 0;
    stored = 0;
  }
  __device__ __forceinline__ void store_rows(int upto) {   // groups [stored, upto)
    for (; stored < upto; ++stored) {
      if (stored * 8 < cap) {   // groups past the slot's capacity are not stored (error latched)
        uint4 g;
        __builtin_memcpy(&g, ring + 8 * (stored & (RB - 1)), sizeof(g));
        *gp = g;
      }
      gp += gstride;
    }
  }
  __device__ __forceinline__ void put(int loc, bool hit) {
    const uint16_t v = (uint16_t)loc;
    __builtin_memcpy(ring + (n & (8 * RB - 1)), &v, sizeof(v));
    n += hit ? 1 : 0;
    if (hit && (n & (8 * RB - 1)) == 0) store_rows(n >> 3);   // ring full
  }
  __device__ __forceinline__ void flush() { store_rows((n + 7) >> 3); }
  // append without the ring-full test: the caller stores the complete groups (store_complete) at
  // least once every 8 appends, so at most 15 entries wait in the ring
  __device__ __forceinline__ void put_unchecked(int loc, bool hit) {
    const uint16_t v = (uint16_t)loc;
    __builtin_memcpy(ring + (n & (8 * RB - 1)), &v, sizeof(v));
    n += hit ? 1 : 0;
  }
  __device__ __forceinline__ void store_complete() { store_rows(n >> 3); }
};

// Density-stage epilogue in FP64 for particle a with computational density D: rest-mass density
// from D = rho psi^6 W_L, EoS, shear modulus, yield stress and the packed records of the stress
// and force passes (lanes with valid = false store nothing).  With GIVEN the EoS values are the
// network's (lnpc = ln P, ln c_s^2), otherwise the table's or the Gamma law's.  With net !=
// nullptr (the table pass of a split epilogue) a particle in a cell the network serves is left
// to the network pass: *net is set and only rho is stored.
template <typename R, bool GIVEN>
__device__ __forceinline__ void density_epilogue(const PassArgs& A, int64_t a, bool valid, double D,
                                                 const double4* __restrict__ pos64, const double* __restrict__ vx,
                                                 const double* __restrict__ vy, const double* __restrict__ vz,
                                                 const double* __restrict__ u, const double* __restrict__ S,
                                                 const int8_t* __restrict__ type, const uint8_t* __restrict__ broken,
                                                 DensOut O, bool* net = nullptr, double2 lnpc = double2{}) {
  const sph_params& p = A.p;
  const double va[3] = {vx[a], vy[a], vz[a]};
  const bool tov = p.background == SPH_TOV;
  double rho = D, hfac = 1.0;
  Metric g{};
  double v2 = 0.0, psi2 = 1.0, psi4 = 1.0, WL = 1.0;
  if (tov) {
    double cx, cy, cz;
    star_centre(A, a, cx, cy, cz);
    const double4 p64 = pos64[a];   // the background is always evaluated in FP64
    g = metric_at(p, p64.x - cx, p64.y - cy, p64.z - cz);
    v2 = va[0] * va[0] + va[1] * va[1] + va[2] * va[2];
    psi2 = g.psi * g.psi;
    psi4 = psi2 * psi2;
    WL = 1.0 / sqrt(1.0 - psi4 * v2 / (g.alpha * g.alpha));
    rho = D / (psi4 * psi2 * WL);
  }
  if (net && mlp_trusted_at(A.mlp, p, rho, u[a])) {
    if (valid) O.rho[a] = rho;   // the network pass's input
    *net = true;
    return;
  }
  double P, cs2;
  int e = 0;
  if constexpr (GIVEN) {
    P = exp(lnpc.x);
    cs2 = exp(lnpc.y);
  } else {
    e = eos_eval(p, rho, u[a], P, cs2);
  }
  if (!valid) return;
  if (e) latch_error(A.status, e, (int)a);
  if (tov) {
    hfac = 1.0 + u[a] + P / rho;
    // coefficients of the trajectory equation (zero shift, gamma_ij = psi^4 delta_ij) for the
    // force pass, acc = -k_P m A^P + B + m A^S with A^P, A^S its pair sums: the pressure
    // coefficient k_P = alpha^2 psi^6 / (W_L h psi^4) (1/(W_L rho h) per unit D, so that a TOV
    // star is static with grad P ~= D A^P) and
    // B_i = -(alpha dalpha n_i + 4 psi^3 dpsi ((n.v) v_i - v^2 n_i / 2)) / psi^4 + 2 (dalpha / alpha) (n.v) v_i
    const double ipsi4 = 1.0 / psi4;
    const double kP = g.alpha * g.alpha * psi2 / (WL * hfac);
    const double nv = g.n[0] * va[0] + g.n[1] * va[1] + g.n[2] * va[2];
    const double c0 = 2.0 * g.dalpha / g.alpha * nv;
    const double cg = 4.0 * psi2 * g.psi * g.dpsi;
    double Bv[3];
    for (int i = 0; i < 3; ++i)
      Bv[i] = -(g.alpha * g.dalpha * g.n[i] + cg * (nv * va[i] - 0.5 * v2 * g.n[i])) * ipsi4 + c0 * va[i];
    O.tov[a] = make_double4(kP, Bv[0], Bv[1], Bv[2]);
  }
  const double cs = sqrt(cs2);
  const double Bm = rho * hfac * cs2;
  const bool solid = type[a] == 1 && !(broken[a] && p.break_mode == SPH_BREAK_FLUIDIZE);
  double mu = 0.0;
  if (solid) {
    double fac = p.mu_pfactor;
    if (A.star && A.stars) fac = A.stars[A.star[a]].mu_pfactor;
    mu = (p.mu_mode == SPH_MU_PFACTOR) ? fac * P : p.mu_const;
  }
  const double E = mu > 0.0 ? 9.0 * Bm * mu / (3.0 * Bm + mu) : 0.0;
  if (p.energy_mode == SPH_ENERGY_FIRST_LAW) {
    // du/dt = (P / rho^2) drho/dt along the path with rho = D / (psi^6 W_L):
    //   (P / (rho D)) dD/dt - (P / rho) [6 (psi'/psi)(n.v) + dln W_L/dt],
    //   dln W_L/dt = W_L^2 / 2 [(4 psi^3 psi' (n.v) v^2 + 2 psi^4 v.a) / alpha^2 - 2 psi^4 v^2 alpha' (n.v) / alpha^3];
    // the force pass adds e0 dD/dt + e1 + e2 v.a to the viscous heating and the stress work
    double e0 = P / (rho * D), e1 = 0.0, e2 = 0.0;
    if (tov) {
      const double nv = g.n[0] * va[0] + g.n[1] * va[1] + g.n[2] * va[2];
      const double ia2 = 1.0 / (g.alpha * g.alpha);
      const double Pr = P / rho;
      e1 = -Pr * (6.0 * g.dpsi / g.psi * nv +
                  0.5 * WL * WL * (4.0 * psi2 * g.psi * g.dpsi * nv * v2 * ia2 - 2.0 * psi4 * v2 * g.dalpha * nv * ia2 / g.alpha));
      e2 = -Pr * WL * WL * psi4 * ia2;
    }
    O.xcoef[a] = e0;
    O.xcoef[O.xs + a] = e1;
    O.xcoef[2 * O.xs + a] = e2;
  }
  if (p.dtP_mode == SPH_DTP_LAGGED && tov) {
    // the dP/dt entry of the trajectory equation, -v^i dP/dt / (W_L^2 rho h), with dP/dt at fixed
    // position = (P - P_prev) / dt_step - v . grad P; the force pass supplies v . grad P
    const double dtp = O.in_step ? O.dtw[5] : 0.0;
    const double kt = dtp > 0.0 ? 1.0 / (WL * WL * rho * hfac) : 0.0;
    O.xcoef[3 * O.xs + a] = dtp > 0.0 ? kt * (P - O.P[a]) / dtp : 0.0;   // O.P still holds P_prev
    O.xcoef[4 * O.xs + a] = kt;
  }
  O.rho[a] = rho;   // D stays as the pair loop wrote it
  O.P[a] = P;
  O.cs[a] = cs;
  if (type[a] == 1) {   // the moduli and the yield stress are read for crust particles only
    O.mu[a] = mu;
    O.B[a] = Bm;
    O.Y0[a] = (p.y0_mode == SPH_Y0_EFACTOR) ? p.y0_over_E * E : p.y0_const;
  }
  const double iD2 = 1.0 / (D * D);
  const double pi = P * iD2;
  const bool stressed = solid;
  const int64_t n = A.n;
  if (sizeof(R) == 8) {
    O.fv[a] = make_double4(va[0], va[1], va[2], p.visc_alpha * cs);   // alpha c_s for the viscosity
    O.fa[a] = make_double2(pi, stressed ? -D : D);
    if (stressed)   // S/D^2 is read only for stressed particles (the sign of D in fa marks them)
      for (int c = 0; c < 6; ++c) O.sig[c * n + a] = S[c * n + a] * iD2;
  } else {
    O.fvf[a] = make_float4((float)va[0], (float)va[1], (float)va[2], (float)(0.5 * p.visc_alpha * cs));
    O.faf[a] = make_float2((float)pi, stressed ? -(float)(0.5 * D) : (float)(0.5 * D));
    if (stressed)
      for (int c = 0; c < 6; ++c) O.sigf[c * n + a] = (float)(S[c * n + a] * iD2);
  }
  if (!isfinite(D) || !isfinite(P) || !isfinite(cs)) latch_error(A.status, SPH_E_NONFINITE, (int)a);
}

// Width of the FP32 guard band of the neighbour decision, relative to M_a H + H^2 (M_a the
// largest coordinate magnitude of the target relative to the tile's reference particle,
// H = h_a + h_b): 64 u with u = 2^-24.  With coordinates and smoothing lengths rounded to FP32 and
// r^2, H^2 evaluated in FP32, |r2_f - r^2| <= 4 sqrt(3) u M |d| + 5 u r^2 and
// |H2_f - H^2| <= 7 u H^2 (to first order), M the larger coordinate magnitude of the pair.  The
// FP32 decision can differ from the exact one only if r^2 lies within that error of H^2, i.e.
// |d| = H (1 + O(u)); then M <= M_a + |d| and the error is at most
// 4 sqrt(3) u M_a H + (4 sqrt(3) + 12) u H^2 < 64 u (M_a H + H^2).  Outside the band the FP32
// decision therefore equals the FP64 one.  The pass takes the decision from r2_f - H_f^2 formed
// with one FMA (its sign is that of r2_f - H_f^2, and H_f^2 is closer to H^2 than the rounded
// H2_f) and the band as H (kBand H + kBand M_a).
constexpr float kBand = 3.814697265625e-06f;   // 2^-18

// Density pass.  Walks the candidate lists, takes the exact neighbour decision r^2 < (h_a + h_b)^2
// of the FP64 positions on every candidate, sums the kernel over the neighbours in R and counts
// them; with XL it also writes the exact lists (for the stress and force passes when they walk
// exact lists, and for the neighbour export).  A workgroup of L waves takes one tile: lane g
// serves target g / L as sub-lane g % L, walks the candidate slot list (particle * L + sub-lane)
// and writes the exact hits to the exact slot list of the same index; the L partial sums are
// added across the lanes.  The per-particle epilogue runs in k_density_epilogue, one lane per
// particle.
//   FP64 (R = double): union records staged in LDS as FP64 (x, y, z, h), FP64 test.
//   FP32 (R = float): union records staged as FP32 coordinates relative to the tile's first
//   particle (16 bytes), the decision taken in FP32 and, inside the guard band kBand, again
//   exactly from the FP64 positions; the lists are the same as in FP64.
template <typename R, int KER, bool PER, int L, bool XL>
__global__ __launch_bounds__(64 * L)
__attribute__((amdgpu_waves_per_eu(std::is_same<R, float>::value ? 5 : 4)))
void k_density(PassArgs A, const double4* __restrict__ pos64, DensOut O,
                                                    uint16_t* __restrict__ xlist, int32_t* __restrict__ xcount,
                                                    int32_t* __restrict__ xcount_sl) {
  constexpr bool F32 = std::is_same<R, float>::value;
  using SR = typename std::conditional<F32, float4, double4>::type;
  constexpr int CH = Rec<R>::CH_D * L < Rec<R>::CHMAX_D ? Rec<R>::CH_D * L : Rec<R>::CHMAX_D;
  constexpr int CHU = CH - 1;   // union records per chunk; slot CHU holds the walk's sentinel
  __shared__ SR sp[CH];
  constexpr int RB = 2;
  __shared__ __align__(16) uint16_t lring[XL ? 64 * L : 1][8 * RB];   // per-lane staging of the exact lists
  const double box = A.p.box, half = 0.5 * box;
  const float boxf = (float)box, halff = (float)half;
  const int tl = threadIdx.x / L, sub = threadIdx.x % L;
  if (threadIdx.x == 0) {   // the sentinel: far from every target, h = 0 (no neighbour, W = 0)
    if constexpr (F32) sp[CHU] = make_float4(1e10f, 1e10f, 1e10f, 0.0f);
    else sp[CHU] = make_double4(1e10, 1e10, 1e10, 0.0);
  }
  const int64_t ntl = num_tiles(A);
  for (int64_t k_ = blockIdx.x / SPH_XCD, chunk_ = xcd_chunk(ntl); k_ < chunk_; k_ += gridDim.x / SPH_XCD) {
    const int64_t tile = (int64_t)(blockIdx.x % SPH_XCD) * chunk_ + k_;
    if (tile >= ntl) break;
  TileWalk tw;
  tw.begin(A, tile, tl);
  const int total = tw.valid ? A.cnt_s[tw.p] : 0;
  const int64_t a = tw.a;
  const int64_t slot = a * L + sub;
  const uint4* lst = reinterpret_cast<const uint4*>(A.nbr16s) + slot;
  const int cnt = total > sub ? (total - sub + L - 1) / L : 0;
  const double4 pa = tw.valid ? pos64[a] : make_double4(0.0, 0.0, 0.0, 1.0);
  const double4 ref = pos64[A.tile_start[tile]];
  float4 paf = make_float4(0.f, 0.f, 0.f, 1.f);
  float kMa = 0.f;   // kBand times the target's largest coordinate magnitude
  if constexpr (F32) {
    paf = make_float4((float)wrap_sel<PER>(pa.x - ref.x, box, half), (float)wrap_sel<PER>(pa.y - ref.y, box, half),
                      (float)wrap_sel<PER>(pa.z - ref.z, box, half), (float)pa.w);
    kMa = kBand * fmaxf(fabsf(paf.x), fmaxf(fabsf(paf.y), fabsf(paf.z)));
  }
  R sum = 0;
  ListWriter<RB> wr;
  wr.init(reinterpret_cast<uint4*>(xlist) + slot, A.capw * L, lring[XL ? threadIdx.x : 0], A.cap_sl);
  // candidate union member loc with record pb (the sentinel: a miss with W = 0)
  auto cand = [&](int loc, const SR& pb, auto&& put) {
    bool hit;
    R W;
    if constexpr (F32) {
      const float dx = wrap_sel<PER>(paf.x - pb.x, boxf, halff);
      const float dy = wrap_sel<PER>(paf.y - pb.y, boxf, halff);
      const float dz = wrap_sel<PER>(paf.z - pb.z, boxf, halff);
      const float r2 = dx * dx + dy * dy + dz * dz;
      const float H = paf.w + pb.w;
      const float diff = fmaf(-H, H, r2);   // one rounding: the sign of r2 - H^2
      hit = diff < 0.f;
      if (fabsf(diff) <= H * fmaf(kBand, H, kMa)) {   // near the support edge: decide in FP64
        const double4 q = pos64[tw.U[loc]];
        const double r2d = pair_r2(wrap_sel<PER>(pa.x - q.x, box, half), wrap_sel<PER>(pa.y - q.y, box, half),
                                   wrap_sel<PER>(pa.z - q.z, box, half));
        const double Hd = pa.w + q.w;
        hit = r2d < Hd * Hd;
      }
      W = kern_W_unit_eighth<float, KER>(sqrt_hw(r2), rcp_fast(H));   // zero for misses
    } else {
      const double dx = wrap_sel<PER>(pa.x - pb.x, box, half);
      const double dy = wrap_sel<PER>(pa.y - pb.y, box, half);
      const double dz = wrap_sel<PER>(pa.z - pb.z, box, half);
      const double r2 = pair_r2(dx, dy, dz);
      const double H = pa.w + pb.w;
      hit = r2 < H * H;
      W = kern_W_unit<R, KER>(sqrt_fast((R)r2), rcp_fast((R)(0.5 * H)));
      W = hit ? W : (R)0;   // the exact decision also at the support edge
    }
    sum += W;
    put(loc, hit);
  };
  auto stage = [&](int c0) {
    stage_union<64 * L, CHU>(tw.U, c0, tw.usize, [&](int32_t b) { return pos64[b]; }, [&](int j, const double4& q) {
      if constexpr (F32)
        sp[j] = make_float4((float)wrap_sel<PER>(q.x - ref.x, box, half), (float)wrap_sel<PER>(q.y - ref.y, box, half),
                            (float)wrap_sel<PER>(q.z - ref.z, box, half), (float)q.w);
      else
        sp[j] = q;
    });
  };
  if (tw.usize <= CHU) {   // whole union in one chunk: pipelined group walk
    __syncthreads();
    stage(0);
    __syncthreads();
    walk_groups_pf(
        lst, A.capw * L, cnt, wave_max_i(cnt), CHU, [&](int j) { return sp[j]; },
        [&](int loc, const SR& pb) {
          cand(loc, pb, [&](int l, bool h) {
            if constexpr (XL) wr.put_unchecked(l, h);
            else wr.n += h ? 1 : 0;
          });
        },
        [&]() {
          if constexpr (XL) wr.store_complete();
        });
  } else {
    tw.start(lst, A.capw * L, cnt);
    for (int c0 = 0; c0 < tw.usize; c0 += CHU) {
      __syncthreads();
      stage(c0);
      __syncthreads();
      const int cend = c0 + CHU;
      while (tw.next < cend) {
        const int loc = tw.next;
        tw.advance();
        cand(loc, sp[loc - c0], [&](int l, bool h) {
          if constexpr (XL) wr.put(l, h);
          else wr.n += h ? 1 : 0;
        });
      }
    }
  }
  if constexpr (XL) wr.flush();
  sum = lane_group_sum<L>(sum);
  const int nexact = lane_group_sum<L>(wr.n);
  if (tw.valid) {
    xcount_sl[slot] = wr.n < A.cap_sl ? wr.n : A.cap_sl;
    if (sub == 0) xcount[a] = nexact < A.cap ? nexact : A.cap;
    if (nexact > A.cap || wr.n > A.cap_sl) latch_error(A.status, SPH_E_NGB_CAPACITY, (int)a);
  }
  if (tw.valid && sub == 0) {
    const double W0 = wendland_self<double>(KER, pa.w);   // the particle's own term
    // the FP32 sum holds kernel values / 8 (kern_W_unit_eighth); the factor 8 is exact
    O.D[a] = particle_mass(A, a) * fma((F32 ? 8.0 : 1.0) * kern_W_const<KER>(), (double)sum, W0);
  }
  }
}

// Per-particle epilogue of the density stage (EoS, moduli, packed records), one lane per particle,
// D from the pair loop.  Kept out of the pair-loop kernel, where only one lane of a target's L
// would work on it and its registers would lower the loop's occupancy.  With the EoS network the
// epilogue is split in two passes: this one (SPLIT) takes the table EoS and appends the particles
// in cells the network serves to a list (nlist, nlist_n), which k_density_epilogue_net then
// finishes with the network in full waves; the network's registers would otherwise lower the
// occupancy of the whole epilogue, and its work would run for every wave with one served lane.
__device__ __forceinline__ void courant_min(const DensOut& O, const double4* __restrict__ pos64,
                                            const double* __restrict__ vx, const double* __restrict__ vy,
                                            const double* __restrict__ vz, const int8_t* __restrict__ type,
                                            int64_t a, double& qmin) {
  // Courant step: h / (c_L + |v|), c_L^2 = c_s^2 + 4 mu / (3 rho)
  const double cs = O.cs[a], rh = O.rho[a];
  const double mu = type[a] == 1 ? O.mu[a] : 0.0;
  const double cl = sqrt(cs * cs + 4.0 * mu / (3.0 * rh));
  const double vm = sqrt(vx[a] * vx[a] + vy[a] * vy[a] + vz[a] * vz[a]);
  const double q = pos64[a].w / (cl + vm);
  qmin = q < qmin ? q : qmin;
}
// The Courant minimum of a wave (WAVE) or of a whole workgroup of NT threads, stored to
// dtpart[slot] (every thread of the wave or workgroup calls).
template <int NT, bool WAVE>
__device__ __forceinline__ void courant_store(const DensOut& O, double qmin, int slot) {
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(qmin, off, 64);
    qmin = o < qmin ? o : qmin;
  }
  if constexpr (WAVE || NT == 64) {
    if ((threadIdx.x & 63) == 0) O.dtpart[slot] = qmin;
  } else {
    __shared__ double s_q[NT / 64];
    if ((threadIdx.x & 63) == 0) s_q[threadIdx.x >> 6] = qmin;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < NT / 64; ++w) qmin = s_q[w] < qmin ? s_q[w] : qmin;
      O.dtpart[slot] = qmin;
    }
  }
}
// Threads per workgroup of the table pass: 64, or 256 when it hands particles to the network
// pass (the list is appended to once per workgroup).
template <bool SPLIT>
constexpr int epilogue_threads() { return SPLIT ? 256 : 64; }

template <typename R, bool SPLIT>
__global__ __launch_bounds__(epilogue_threads<SPLIT>()) void k_density_epilogue(
    PassArgs A, const double4* __restrict__ pos64, const double* __restrict__ vx, const double* __restrict__ vy,
    const double* __restrict__ vz, const double* __restrict__ u, const double* __restrict__ S,
    const int8_t* __restrict__ type, const uint8_t* __restrict__ broken, DensOut O, int32_t* __restrict__ nlist,
    int32_t* __restrict__ nlist_n) {
  constexpr int NT = epilogue_threads<SPLIT>(), NW = NT / 64;
  const int64_t n = cancelled(A) ? 0 : A.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int s_cnt[NW + 1];
  double qmin = __builtin_inf();
  for (int64_t base = (int64_t)blockIdx.x * NT; base < n; base += (int64_t)gridDim.x * NT) {
    const int64_t a = base + tid;
    const bool valid = a < n;
    const int64_t ae = valid ? a : base;   // lanes past the end work on a valid particle, store nothing
    bool net = false;
    density_epilogue<R, false>(A, ae, valid, O.Dread[ae], pos64, vx, vy, vz, u, S, type, broken, O,
                               SPLIT ? &net : nullptr);
    if constexpr (SPLIT) {
      // the workgroup's served particles join the list in particle order, with one atomic
      const unsigned long long m = __ballot(valid && net);
      if (lane == 0) s_cnt[wave] = __popcll(m);
      __syncthreads();
      if (tid == 0) {
        int t = 0;
        for (int w = 0; w < NW; ++w) t += s_cnt[w];
        s_cnt[NW] = t ? atomicAdd(nlist_n, t) : 0;
      }
      __syncthreads();
      if (valid && net) {
        int off = s_cnt[NW];
        for (int w = 0; w < wave; ++w) off += s_cnt[w];
        nlist[off + __popcll(m & (lane ? (~0ull >> (64 - lane)) : 0ull))] = (int32_t)a;
      }
      __syncthreads();   // s_cnt is reused by the next round
    }
    if (O.dtpart && valid && !net) courant_min(O, pos64, vx, vy, vz, type, a, qmin);
  }
  if (O.dtpart) courant_store<NT, false>(O, qmin, blockIdx.x);
}

// The network pass of a split epilogue: the particles of nlist[0, *nlist_n), 64 per wave.  A wave
// evaluates the network for its 64 particles (ln rho from the rho the table pass stored, the
// parameters staged in LDS once per workgroup of 4 waves) and then runs the epilogue with the
// network's ln P, ln c_s^2; wave k of block b writes its Courant minimum to dtpart[dt_off + 4 b + k].
template <typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_density_epilogue_net(PassArgs A, const double4* __restrict__ pos64,
                                                              const double* __restrict__ vx,
                                                              const double* __restrict__ vy,
                                                              const double* __restrict__ vz,
                                                              const double* __restrict__ u,
                                                              const double* __restrict__ S,
                                                              const int8_t* __restrict__ type,
                                                              const uint8_t* __restrict__ broken, DensOut O,
                                                              const int32_t* __restrict__ nlist,
                                                              const int32_t* __restrict__ nlist_n, int dt_off) {
  const int64_t cnt = cancelled(A) ? 0 : *nlist_n;
  if ((int64_t)blockIdx.x * 256 >= cnt && !O.dtpart) return;   // no particle for this block
  mlp_stage_lds(A.mlp);
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const MlpNorm nm = A.mlp.norm;
  double qmin = __builtin_inf();
  for (int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64; base < cnt; base += (int64_t)gridDim.x * 256) {
    const int64_t i = base + (threadIdx.x & 63);
    const bool valid = i < cnt;
    const int64_t a = nlist[valid ? i : base];
    const double lnr = log(O.rho[a]), lnu = log(u[a]);
    float y0 = 0.f, y1 = 0.f;
    mlp_wave<true>(A.mlp, (float)((lnr - nm.in_lo[0]) * nm.in_sc[0] - 1.0),
                   (float)((lnu - nm.in_lo[1]) * nm.in_sc[1] - 1.0), y0, y1);
    const double2 lnpc = make_double2((double)y0 * nm.out_sc[0] + nm.out_c[0], (double)y1 * nm.out_sc[1] + nm.out_c[1]);
    density_epilogue<R, true>(A, a, valid, O.Dread[a], pos64, vx, vy, vz, u, S, type, broken, O, nullptr, lnpc);
    if (O.dtpart && valid) courant_min(O, pos64, vx, vy, vz, type, a, qmin);
  }
  if (O.dtpart) courant_store<256, true>(O, qmin, dt_off + blockIdx.x * 4 + wave);
}

__global__ void k_word_clear(int32_t* w) { *w = 0; }   // a kernel, not a memset: graph-safe

// ---- velocity gradient and stress rate ---------------------------------------------------------
// Lane g of the L-wave workgroup walks the exact slot list (g / L, g % L) written by the density
// pass; the partial velocity gradients of a target's L lanes are added before the epilogue.
template <typename R, int KER, bool PER, int L>
__global__ __launch_bounds__(64 * L) void k_stress(PassArgs A, const typename Rec<R>::P4* __restrict__ pos,
                                                   const typename Rec<R>::V4* __restrict__ fv,
                                                   const typename Rec<R>::A2* __restrict__ fa,
                                                   const double* __restrict__ S, const double* __restrict__ mu,
                                                   double* __restrict__ dSdt, double* __restrict__ sdot) {
  using P4 = typename Rec<R>::P4;
  using V4 = typename Rec<R>::V4;
  constexpr int CH = Rec<R>::CH_S * L;
  const int tl = threadIdx.x / L, sub = threadIdx.x % L;
  __shared__ P4 sp[CH];
  __shared__ V4 sv[CH];
  const R box = (R)A.p.box, half = (R)0.5 * box;
  // only the tiles of the work list (tiles with a type-1 particle); every other particle's rates
  // are zero since the last build
  const int64_t nst = cancelled(A) ? 0 : (int64_t)A.grid->nstress;
  for (int64_t w = blockIdx.x; w < nst; w += gridDim.x) {
    const int64_t tile = A.stress_tiles[w];
  TileWalk tw;
  tw.begin(A, tile, tl);
  const int64_t a = tw.a;
  const int64_t slot = a * L + sub;
  const int64_t n = A.n;
  const typename Rec<R>::A2 faa = tw.valid ? fa[a] : typename Rec<R>::A2{0, 1};
  const bool stressed = tw.valid && faa.y < 0;
  if (tw.valid && !stressed && sub == 0) {  // fluid particle (or fluidized): no deviatoric stress evolution
    for (int c = 0; c < 6; ++c) dSdt[c * n + a] = 0.0;
    sdot[a] = 0.0;
  }
  if (!__syncthreads_or(stressed)) continue;   // whole tile fluid
  const sph_params& p = A.p;
  const P4 pa = tw.valid ? pos[a] : P4{0, 0, 0, 1};
  const V4 va = tw.valid ? fv[a] : V4{0, 0, 0, 0};
  R G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  struct Recs { P4 p; V4 v; };
  auto pair = [&](const Recs& r) {
    const P4& pb = r.p;
    const V4& vb = r.v;
    const R d[3] = {wrap_sel<PER>(pa.x - pb.x, box, half), wrap_sel<PER>(pa.y - pb.y, box, half),
                    wrap_sel<PER>(pa.z - pb.z, box, half)};
    const R r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const R ih = rcp_fast(Rec<R>::HS * (pa.w + pb.w));
    R F;   // without the kernel's constant, applied in the epilogue
    if constexpr (std::is_same<R, float>::value) F = kern_F_unit<float, KER>(sqrt_hw(r2), ih);
    else F = kern_F_unit<R, KER>(sqrt_fast(r2), ih);
    const R g[3] = {F * d[0], F * d[1], F * d[2]};
    const R v[3] = {vb.x - va.x, vb.y - va.y, vb.z - va.z};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) G[i][jj] += v[i] * g[jj];
  };
  auto stage = [&](int c0, int ch) {
    stage_union<64 * L, CH>(tw.U, c0, c0 + ch < tw.usize ? c0 + ch : tw.usize,
                            [&](int32_t b) { return Recs{pos[b], fv[b]}; },
                            [&](int j, const Recs& r) { sp[j] = r.p; sv[j] = r.v; });
  };
  if (std::is_same<R, float>::value && tw.usize < CH) {
    // FP32 with the whole union in one chunk: pipelined group walk, LDS slot CH - 1 the sentinel
    // (far away, h = 0: F = 0)
    __syncthreads();
    stage(0, CH - 1);
    if (threadIdx.x == 0) {
      sp[CH - 1] = P4{(R)1e10, (R)1e10, (R)1e10, (R)0};
      sv[CH - 1] = V4{(R)0, (R)0, (R)0, (R)0};
    }
    __syncthreads();
    const int cnt = stressed ? pass_count<L>(A, tw.p, sub, slot) : 0;
    walk_groups_pf(
        pass_list<L>(A, slot), A.capw * L, cnt, wave_max_i(cnt), CH - 1,
        [&](int j) { return Recs{sp[j], sv[j]}; }, [&](int, const Recs& r) { pair(r); }, [] {});
  } else {
    tw.start(pass_list<L>(A, slot), A.capw * L, stressed ? pass_count<L>(A, tw.p, sub, slot) : 0);
    for (int c0 = 0; c0 < tw.usize; c0 += CH) {
      __syncthreads();
      stage(c0, CH);
      __syncthreads();
      const int cend = c0 + CH;
      while (tw.next < cend) {
        const int j = tw.next - c0;
        tw.advance();
        pair(Recs{sp[j], sv[j]});
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) G[i][jj] = lane_group_sum<L>(G[i][jj]);
  if (!stressed || sub != 0) continue;
  const double m = particle_mass(A, a) * kern_F_const<KER>();
  const double D = -(double)faa.y * (2.0 * (double)Rec<R>::HS);  // stressed particles store -D (FP32: -D/2)
  const double iD2 = m / (2.0 * D);
  double ed[3][3], Rd[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      ed[i][j] = ((double)G[i][j] + (double)G[j][i]) * iD2;   // strain rate, eq. solid5
      Rd[i][j] = ((double)G[i][j] - (double)G[j][i]) * iD2;   // rotation rate, eq. solid6
    }
  double Sm[3][3];
  Sm[0][0] = S[a]; Sm[1][1] = S[n + a]; Sm[2][2] = S[2 * n + a];
  Sm[0][1] = Sm[1][0] = S[3 * n + a];
  Sm[0][2] = Sm[2][0] = S[4 * n + a];
  Sm[1][2] = Sm[2][1] = S[5 * n + a];
  const double tr3 = (ed[0][0] + ed[1][1] + ed[2][2]) * (1.0 / 3.0);
  const double tmu = 2.0 * mu[a];
  const double sgn = (p.rotation == SPH_ROT_LITERAL) ? -1.0 : 1.0;
  double dS[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double RS = Rd[i][0] * Sm[0][j] + Rd[i][1] * Sm[1][j] + Rd[i][2] * Sm[2][j];
      double SR = Sm[i][0] * Rd[0][j] + Sm[i][1] * Rd[1][j] + Sm[i][2] * Rd[2][j];
      dS[i][j] = tmu * (ed[i][j] - (i == j ? tr3 : 0.0)) + sgn * (RS - SR);   // eq. solid4
    }
  dSdt[a] = dS[0][0];
  dSdt[n + a] = dS[1][1];
  dSdt[2 * n + a] = dS[2][2];
  dSdt[3 * n + a] = dS[0][1];
  dSdt[4 * n + a] = dS[0][2];
  dSdt[5 * n + a] = dS[1][2];
  double se = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) se += Sm[i][j] * ed[i][j];
  sdot[a] = se / D;   // stress work S^ij epsdot^ij / rho of eq. solid3
  }
}

// ---- forces -----------------------------------------------------------------------------------
struct ForceOut {
  double *ax, *ay, *az, *dudt;
  const double4* pos64;                  // FP64 positions (external potential)
  const double *vx, *vy, *vz;            // velocities of the evaluation (drag, variants)
  double* dDdt;                          // sum m (v_a - v_b) . grad_a W (continuity density)
  const double* xcoef;                   // first-law and dP/dt coefficients of the epilogue
  int64_t xs;
  const double* D;                       // FP64 computational density
};

// External effective potential (g_eff = -grad phi_eff along the radius from the star centre,
// linear in the table, 0 beyond its last entry), harmonic potential walls and the relaxation drag,
// added to the acceleration of particle a.
__device__ __forceinline__ void ext_accel(const PassArgs& A, const ForceOut& O, int64_t a, double acc[3]) {
  const sph_params& p = A.p;
  double cx, cy, cz;
  star_centre(A, a, cx, cy, cz);
  const double4 q = O.pos64[a];
  const double X[3] = {q.x - cx, q.y - cy, q.z - cz};
  const double r = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
  if (r > 0.0) {
    double g = 0.0;
    const double t = p.ext == SPH_EXT_RADIAL ? r / p.ext_dr : 1e300;
    if (t <= (double)(p.ext_n - 1)) {
      int i = (int)floor(t);
      i = i > p.ext_n - 2 ? p.ext_n - 2 : i;
      const double f = t - (double)i;
      g = (1.0 - f) * p.ext_g[i] + f * p.ext_g[i + 1];
    }
    if (p.wall_in > 0.0 && r < p.wall_in) g += p.wall_k * (p.wall_in - r);
    if (p.wall_out > 0.0 && r > p.wall_out) g -= p.wall_k * (r - p.wall_out);
    const double gr = g / r;
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k] += gr * X[k];
  }
  if (p.damping > 0.0) {
    acc[0] -= p.damping * O.vx[a];
    acc[1] -= p.damping * O.vy[a];
    acc[2] -= p.damping * O.vz[a];
  }
}

// Lane g of the L-wave workgroup walks the exact slot list (g / L, g % L); the partial sums of a
// target's L lanes are added before the fixed-background epilogue.
// XS selects the optional sums (compile-time, so that the default mode keeps its registers):
//   kXDD: sum m v_ab . grad_a W (continuity density and first-law energy);
//   kXGP: that and v_a . (P_a/D_a^2 + P_b/D_b^2) grad_a W (the advection of P in the lagged dP/dt row);
// and kXSL (FP32, with neither sum): the neighbours' S/D^2 staged in LDS with the other records,
// for workloads where most tiles hold stressed particles (otherwise each stressed pair reads the
// neighbour's union index and six S/D^2 values from memory).
constexpr int kXDD = 1, kXGP = 2, kXSL = 4;
template <typename R, int KER, bool PER, int L, int XS>
__global__ __launch_bounds__(64 * L) __attribute__((amdgpu_waves_per_eu(4))) void k_forces(PassArgs A, const typename Rec<R>::P4* __restrict__ pos,
                                                   const typename Rec<R>::V4* __restrict__ fv,
                                                   const typename Rec<R>::A2* __restrict__ fa,
                                                   const R* __restrict__ sig, const double4* __restrict__ tov,
                                                   const double* __restrict__ sdot, ForceOut O) {
  using P4 = typename Rec<R>::P4;
  using V4 = typename Rec<R>::V4;
  using A2 = typename Rec<R>::A2;
  constexpr bool DD = (XS & 3) != 0, GP = (XS & 3) == kXGP, SL = (XS & kXSL) != 0;
  static_assert(!SL || std::is_same<R, float>::value, "S/D^2 in LDS: FP32 records only");
  constexpr int CH = (SL ? Rec<float>::CH_FS : Rec<R>::CH_F) * L;
  constexpr int CHU = CH - 1;   // union records per chunk; slot CHU holds the walk's sentinel
  const int tl = threadIdx.x / L, sub = threadIdx.x % L;
  __shared__ P4 sp[CH];
  __shared__ V4 sv[CH];
  __shared__ A2 sa2[CH];
  __shared__ R ssg[SL ? 6 : 1][SL ? CH : 1];   // kXSL: S/D^2 of the staged members (0 if unstressed)
  const R box = (R)A.p.box, half = (R)0.5 * box;
  if (threadIdx.x == 0) {   // the sentinel: far from every target, at rest, h = 0, unstressed (F = 0)
    sp[CHU] = P4{(R)1e10, (R)1e10, (R)1e10, (R)0};
    sv[CHU] = V4{(R)0, (R)0, (R)0, (R)0};
    sa2[CHU] = A2{(R)0, (R)1};
  }
  const int64_t ntl = num_tiles(A);
  for (int64_t k_ = blockIdx.x / SPH_XCD, chunk_ = xcd_chunk(ntl); k_ < chunk_; k_ += gridDim.x / SPH_XCD) {
    const int64_t tile = (int64_t)(blockIdx.x % SPH_XCD) * chunk_ + k_;
    if (tile >= ntl) break;
  TileWalk tw;
  tw.begin(A, tile, tl);
  const int64_t a = tw.a;
  const int64_t slot = a * L + sub;
  const uint4* lst = pass_list<L>(A, slot);
  const int cnt = tw.valid ? pass_count<L>(A, tw.p, sub, slot) : 0;
  const int64_t n = A.n;
  const sph_params& p = A.p;
  const P4 pa = tw.valid ? pos[a] : P4{0, 0, 0, 1};
  const V4 va = tw.valid ? fv[a] : V4{0, 0, 0, 0};
  const A2 faa = tw.valid ? fa[a] : A2{0, 1};
  const bool a_st = faa.y < 0;
  const R Da = a_st ? -faa.y : faa.y;
  const R pia = faa.x;
  R sa[6] = {0, 0, 0, 0, 0, 0};
  if (a_st)
#pragma unroll
    for (int c = 0; c < 6; ++c) sa[c] = sig[c * n + a];
  const R alpha_v = (R)p.visc_alpha, beta_v = (R)p.visc_beta, eps_v = (R)p.visc_eps;
  R AP[3] = {0, 0, 0}, AS[3] = {0, 0, 0}, ud = 0, dd = 0, gp = 0;
  struct Recs { P4 p; V4 v; A2 f; };
  int cbase = 0;   // union index of LDS slot 0 (the chunk's first member)
  // pair with union member loc, records r (the sentinel: F = 0, which zeroes every term)
  // ST: the stress term is compiled in (a stressed target or union member can occur)
  auto pair_st = [&](int loc, const Recs& r, auto ST) {
    const P4& pb = r.p;
    const V4& vb = r.v;
    const A2& fab = r.f;
    const R d[3] = {wrap_sel<PER>(pa.x - pb.x, box, half), wrap_sel<PER>(pa.y - pb.y, box, half),
                    wrap_sel<PER>(pa.z - pb.z, box, half)};
    const R r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const R hab = Rec<R>::HS * (pa.w + pb.w);
    R F;   // grad_a W = kF F d (the constant kF is applied to the sums)
    if constexpr (std::is_same<R, float>::value) F = kern_F_unit<float, KER>(sqrt_hw(r2), rcp_fast(hab));
    else F = kern_F_unit<R, KER>(sqrt_fast(r2), rcp_fast(hab));
    const R v[3] = {va.x - vb.x, va.y - vb.y, va.z - vb.z};
    const R vr = v[0] * d[0] + v[1] * d[1] + v[2] * d[2];
    const bool b_st = fab.y < 0;
    const R Db = fabs(fab.y);
    // Monaghan viscosity on approaching pairs, Pi = mu (beta mu - alpha c_bar) / Dbar with
    // mu = hab vr / X: with tv = mu / Dbar (one reciprocal), Pi = tv (beta tv Dbar - alpha c_bar)
    const R X = r2 + eps_v * hab * hab;
    const R Dbar = Rec<R>::HS * (Da + Db);
    const R tv = hab * vr * rcp_fast(X * Dbar);
    const R acbar = Rec<R>::HS * (va.w + vb.w);   // alpha c_bar (the records hold alpha c_s)
    const R Pi = vr < (R)0 ? tv * fma(beta_v * tv, Dbar, -acbar) : (R)0;
    const R cPF = (pia + fab.x + Pi) * F;
    AP[0] += cPF * d[0];
    AP[1] += cPF * d[1];
    AP[2] += cPF * d[2];
    const R Fvr = F * vr;                   // v_ab . grad_a W = F (v_ab . d)
    ud += (pia + (R)0.5 * Pi) * Fvr;
    if constexpr (DD) dd += Fvr;
    if constexpr (GP) gp += (pia + fab.x) * F * (va.x * d[0] + va.y * d[1] + va.z * d[2]);
    if (decltype(ST)::value && (a_st || b_st)) {
      const R g[3] = {F * d[0], F * d[1], F * d[2]};
      R s6[6];
      if constexpr (SL) {
        // only a stressed member's slot: padding entries of the walk pass a stale loc with the
        // sentinel's records
#pragma unroll
        for (int c = 0; c < 6; ++c) s6[c] = sa[c] + (b_st ? ssg[c][loc - cbase] : (R)0);
      } else {
        const int32_t b = b_st ? tw.U[loc] : 0;
#pragma unroll
        for (int c = 0; c < 6; ++c) s6[c] = sa[c] + (b_st ? sig[c * n + b] : (R)0);
      }
      AS[0] += s6[0] * g[0] + s6[3] * g[1] + s6[4] * g[2];
      AS[1] += s6[3] * g[0] + s6[1] * g[1] + s6[5] * g[2];
      AS[2] += s6[4] * g[0] + s6[5] * g[1] + s6[2] * g[2];
    }
  };
  auto stage = [&](int c0) {
    if constexpr (SL) {
      struct RecsS { P4 p; V4 v; A2 f; R s[6]; };
      stage_union<64 * L, CHU>(
          tw.U, c0, tw.usize,
          [&](int32_t b) {
            RecsS r{pos[b], fv[b], fa[b], {0, 0, 0, 0, 0, 0}};
            if (r.f.y < 0)
#pragma unroll
              for (int c = 0; c < 6; ++c) r.s[c] = sig[c * n + b];
            return r;
          },
          [&](int j, const RecsS& r) {
            sp[j] = r.p;
            sv[j] = r.v;
            sa2[j] = r.f;
#pragma unroll
            for (int c = 0; c < 6; ++c) ssg[c][j] = r.s[c];
          });
    } else {
      stage_union<64 * L, CHU>(tw.U, c0, tw.usize, [&](int32_t b) { return Recs{pos[b], fv[b], fa[b]}; },
                              [&](int j, const Recs& r) { sp[j] = r.p; sv[j] = r.v; sa2[j] = r.f; });
    }
  };
  auto pair = [&](int loc, const Recs& r) { pair_st(loc, r, std::true_type{}); };
  // a tile whose particles and union members are all of type 0 (the list build's flag) walks
  // without the stress term
  auto stress_tile = [&] { return SL || !A.tile_st || A.tile_st[tile] != 0u; };
  // FP32 with the whole union in one chunk (the usual case): pipelined group walk.  (In FP64 the 8
  // inlined copies of the longer pair body run slower than the shifting walk, measured.)
  if (std::is_same<R, float>::value && tw.usize <= CHU) {
    __syncthreads();
    stage(0);
    __syncthreads();
    const bool any_st = stress_tile();
    auto ld = [&](int j) { return Recs{sp[j], sv[j], sa2[j]}; };
    if (any_st)
      walk_groups_pf(lst, A.capw * L, cnt, wave_max_i(cnt), CHU, ld, pair, [] {});
    else
      walk_groups_pf(
          lst, A.capw * L, cnt, wave_max_i(cnt), CHU, ld,
          [&](int loc, const Recs& r) { pair_st(loc, r, std::false_type{}); }, [] {});
  } else {
    const bool any_st = sizeof(R) == 4 || XS != 0 || stress_tile();
    tw.start(lst, A.capw * L, cnt);
    for (int c0 = 0; c0 < tw.usize; c0 += CHU) {
      __syncthreads();
      stage(c0);
      __syncthreads();
      cbase = c0;
      const int cend = c0 + CHU;
      auto walk = [&](auto ST) {
        while (tw.next < cend) {
          const int loc = tw.next;
          tw.advance();
          const int j = loc - c0;
          pair_st(loc, Recs{sp[j], sv[j], sa2[j]}, ST);
        }
      };
      // (FP64 only: in FP32 this walk serves the rare large unions, and a second copy slowed the
      // pass; the FP64 variant with the extra sums keeps one walk too, a second one spills)
      if (any_st)
        walk(std::true_type{});
      else
        walk(std::false_type{});
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    AP[i] = lane_group_sum<L>(AP[i]);
    AS[i] = lane_group_sum<L>(AS[i]);
  }
  ud = lane_group_sum<L>(ud);
  if constexpr (DD) dd = lane_group_sum<L>(dd);
  if constexpr (GP) gp = lane_group_sum<L>(gp);
  if (!tw.valid || sub != 0) continue;
  const double m = particle_mass(A, a) * kern_F_const<KER>();
  double APd[3] = {m * (double)AP[0], m * (double)AP[1], m * (double)AP[2]};
  double ASd[3] = {m * (double)AS[0], m * (double)AS[1], m * (double)AS[2]};
  double acc[3];
  if (p.background == SPH_TOV) {
    // trajectory equation with the coefficients of the density-stage epilogue
    const double4 tc = tov[a];
    acc[0] = -tc.x * APd[0] + tc.y + ASd[0];
    acc[1] = -tc.x * APd[1] + tc.z + ASd[1];
    acc[2] = -tc.x * APd[2] + tc.w + ASd[2];
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] = -APd[i] + ASd[i];   // eq. solid2
  }
  const double md = m * (double)dd;                            // sum m v_ab . grad_a W
  if constexpr (DD) O.dDdt[a] = md;
  if constexpr (GP) {   // dP/dt row: -v^i k (P - P_prev) / dt + v^i k v . grad P, grad P ~ D A^P
    const double kt = O.xcoef[4 * O.xs + a];
    if (kt != 0.0) {
      const double q = O.xcoef[3 * O.xs + a] - kt * O.D[a] * m * (double)gp;
      acc[0] -= O.vx[a] * q;
      acc[1] -= O.vy[a] * q;
      acc[2] -= O.vz[a] * q;
    }
  }
  double du;
  if (DD && p.energy_mode == SPH_ENERGY_FIRST_LAW) {   // first law: e0 dD/dt + e1 + e2 v.a + heating + work
    const double va_dot = O.vx[a] * acc[0] + O.vy[a] * acc[1] + O.vz[a] * acc[2];
    du = O.xcoef[a] * md + m * ((double)ud - (double)pia * (double)dd) + O.xcoef[O.xs + a] +
         O.xcoef[2 * O.xs + a] * va_dot + sdot[a];
  } else {
    du = m * (double)ud + sdot[a];                             // eq. solid3
  }
  O.ax[a] = acc[0];
  O.ay[a] = acc[1];
  O.az[a] = acc[2];
  O.dudt[a] = du;
  if (!isfinite(acc[0]) || !isfinite(acc[1]) || !isfinite(acc[2]) || !isfinite(du))
    latch_error(A.status, SPH_E_NONFINITE, (int)a);
  }
}

// External effective potential, walls and drag (relaxation set-up, crust shell), added after the
// force pass by one lane per particle: kept out of k_forces, whose registers (and so its
// occupancy) the FP64 evaluation would otherwise raise.  With the first-law energy the
// e2 v . a term takes the added acceleration too.
__global__ __launch_bounds__(256) void k_ext_accel(PassArgs A, ForceOut O) {
  const int64_t n = cancelled(A) ? 0 : A.n;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
    double acc[3] = {0.0, 0.0, 0.0};
    ext_accel(A, O, a, acc);
    O.ax[a] += acc[0];
    O.ay[a] += acc[1];
    O.az[a] += acc[2];
    if (A.p.energy_mode == SPH_ENERGY_FIRST_LAW) {
      const double va = O.vx[a] * acc[0] + O.vy[a] * acc[1] + O.vz[a] * acc[2];
      O.dudt[a] += O.xcoef[2 * O.xs + a] * va;
    }
    if (!isfinite(O.ax[a]) || !isfinite(O.ay[a]) || !isfinite(O.az[a]) || !isfinite(O.dudt[a]))
      latch_error(A.status, SPH_E_NONFINITE, (int)a);
  }
}

PassArgs make_args(sph_ctx* c, sph_state* st) {
  PassArgs A;
  A.p = c->p;
  A.n = st->n;
  A.cap = c->cap;
  A.ucap = c->ucap;
  A.capw = c->capw;
  A.grid = c->grid;
  A.tile_start = c->tile_start;
  A.tile_cnt = c->tile_cnt;
  A.tile_uoff = c->tile_uoff;
  A.tile_u = c->tile_u;
  A.tile_usize = c->tile_usize;
  A.stress_tiles = c->stress_tiles;
  A.nbr16 = c->nbr16;
  A.cnt_sl = c->nbr_count_sl;
  A.cap_sl = slot_capacity(c->cap, pass_lanes(c->p));
  A.nbr16s = c->nbr16s;
  A.cnt_s = c->nbr_count_s;
  A.cand_walk = exact_lists_written(c) ? 0 : 1;
  A.tile_st = c->tile_st;
  A.star = c->stars ? st->star : nullptr;
  A.stars = c->stars;
  A.status = c->status;
  A.has_mlp = mlp_view(c, &A.mlp) ? 1 : 0;
  A.stop = c->eval_seq ? c->drift_flag : nullptr;
  A.seq = c->eval_seq;
  return A;
}

}  // namespace

// Calls f(kernel, periodic) with both as compile-time constants.
template <typename Fn>
static void dispatch_cfg(int kernel, int periodic, Fn&& f) {
  if (kernel == SPH_WC4) {
    if (periodic) f(std::integral_constant<int, SPH_WC4>{}, std::true_type{});
    else f(std::integral_constant<int, SPH_WC4>{}, std::false_type{});
  } else {
    if (periodic) f(std::integral_constant<int, SPH_WC2>{}, std::true_type{});
    else f(std::integral_constant<int, SPH_WC2>{}, std::false_type{});
  }
}

// one workgroup per tile (up to 65536), or a persistent grid of pass_blocks (a multiple of the
// XCD count) that loops over the tiles
static dim3 pass_grid(const sph_ctx* c) {
  if (c->p.pass_blocks > 0) {
    const int64_t b = ((int64_t)c->p.pass_blocks + SPH_XCD - 1) / SPH_XCD * SPH_XCD;
    return dim3((unsigned)(b < 65536 ? b : 65536));
  }
  return dim3((unsigned)(c->cap_tiles < 65536 ? c->cap_tiles : 65536));
}

// Calls f(L) with the pair passes' lanes per target as a compile-time constant.
template <typename Fn>
static void dispatch_lanes(int lanes, Fn&& f) {
  if (lanes == 4) f(std::integral_constant<int, 4>{});
  else if (lanes == 2) f(std::integral_constant<int, 2>{});
  else f(std::integral_constant<int, 1>{});
}

static DensOut dens_out(sph_ctx* c, sph_state* st) {
  DensOut O{};
  // the pair loop writes the summation density; with the continuity density D is state and the
  // sum goes to scratch
  O.D = c->p.density_mode == SPH_DENS_CONTINUITY ? c->dsum : st->D;
  O.rho = st->rho; O.P = st->P; O.cs = st->cs; O.mu = c->mu; O.Y0 = c->Y0; O.B = c->B; O.tov = c->tovf;
  O.fv = c->fv; O.fa = c->fa; O.sig = c->sig; O.fvf = c->fvf; O.faf = c->faf; O.sigf = c->sigf;
  O.Dread = st->D;
  O.xcoef = c->xcoef;
  O.xs = c->capacity;
  // Courant minima: stage calls (sph_density) and steps with the adaptive dt
  O.dtpart = (!c->eval_in_step || c->adaptive) ? c->dtpart : nullptr;
  O.dtw = c->dtw;
  O.in_step = c->eval_in_step ? 1 : 0;
  return O;
}

// The density pass; it writes the exact lists when the stress and force passes walk them.
sph_status launch_density(sph_ctx* c, sph_state* st) {
  PassArgs A = make_args(c, st);
  DensOut O = dens_out(c, st);
  const dim3 g = pass_grid(c);
  const bool f32 = c->p.precision == SPH_FP32;
  const bool xl = !A.cand_walk;
  dispatch_cfg(c->p.kernel, c->p.periodic, [&](auto K, auto P) {
    dispatch_lanes(pass_lanes(c->p), [&](auto LL) {
      constexpr int KER = decltype(K)::value;
      constexpr bool PER = decltype(P)::value;
      constexpr int L = decltype(LL)::value;
      const dim3 b(64 * L);
      auto launch = [&](auto XX) {
        constexpr bool XL = decltype(XX)::value;
        if (f32)
          hipLaunchKernelGGL(HIP_KERNEL_NAME(k_density<float, KER, PER, L, XL>), g, b, 0, c->stream, A, c->pos4, O,
                             c->nbr16, c->nbr_count, c->nbr_count_sl);
        else
          hipLaunchKernelGGL(HIP_KERNEL_NAME(k_density<double, KER, PER, L, XL>), g, b, 0, c->stream, A, c->pos4, O,
                             c->nbr16, c->nbr_count, c->nbr_count_sl);
      };
      if (xl) launch(std::true_type{});
      else launch(std::false_type{});
    });
  });
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

bool exact_lists_written(const sph_ctx* c) { return c->p.precision != SPH_FP32; }

// Exact lists of the last evaluation (positions and h of its packed records) when the density
// pass did not write them: the density pass once more with XL, its sums dropped into scratch.
sph_status launch_exact_lists(sph_ctx* c) {
  sph_state st{};
  st.n = c->n;
  PassArgs A = make_args(c, &st);
  A.stop = nullptr;
  DensOut O{};
  O.D = c->tmp;
  const dim3 g = pass_grid(c);
  const bool f32 = c->p.precision == SPH_FP32;
  dispatch_cfg(c->p.kernel, c->p.periodic, [&](auto K, auto P) {
    dispatch_lanes(pass_lanes(c->p), [&](auto LL) {
      constexpr int KER = decltype(K)::value;
      constexpr bool PER = decltype(P)::value;
      constexpr int L = decltype(LL)::value;
      const dim3 b(64 * L);
      if (f32)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_density<float, KER, PER, L, true>), g, b, 0, c->stream, A, c->pos4, O,
                           c->nbr16, c->nbr_count, c->nbr_count_sl);
      else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_density<double, KER, PER, L, true>), g, b, 0, c->stream, A, c->pos4,
                           O, c->nbr16, c->nbr_count, c->nbr_count_sl);
    });
  });
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

sph_status launch_eos(sph_ctx* c, sph_state* st) {
  PassArgs A = make_args(c, st);
  DensOut O = dens_out(c, st);
  const bool f32 = c->p.precision == SPH_FP32;
  // the network passes only where some table cell is trusted; with none, every particle takes the
  // table (the same values), so the table pass runs alone
  const bool mlp = c->p.eos == SPH_EOS_MLP && A.has_mlp && mlp_trusted_cells(c) > 0;
  const int64_t nt = mlp ? epilogue_threads<true>() : epilogue_threads<false>();
  const unsigned nb = (unsigned)((st->n + nt - 1) / nt < 65536 ? (st->n + nt - 1) / nt : 65536);
  constexpr unsigned kNetBlocks = 1024;   // 4 waves each, 4 workgroups per CU (128 VGPRs)
  c->eos_blocks = O.dtpart ? (int)nb + (mlp ? 4 * (int)kNetBlocks : 0) : 0;
  if (mlp) hipLaunchKernelGGL(k_word_clear, dim3(1), dim3(1), 0, c->stream, c->eos_list_n);
  auto epi = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(nb), dim3((unsigned)nt), 0, c->stream, A, c->pos4, st->vx, st->vy, st->vz, st->u,
                       st->S, st->type, st->broken, O, c->eos_list, c->eos_list_n);
  };
  auto net = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(kNetBlocks), dim3(256), 0, c->stream, A, c->pos4, st->vx, st->vy, st->vz, st->u, st->S,
                       st->type, st->broken, O, c->eos_list, c->eos_list_n, (int)nb);
  };
  if (f32 && mlp) {
    epi(k_density_epilogue<float, true>);
    net(k_density_epilogue_net<float>);
  } else if (f32) {
    epi(k_density_epilogue<float, false>);
  } else if (mlp) {
    epi(k_density_epilogue<double, true>);
    net(k_density_epilogue_net<double>);
  } else {
    epi(k_density_epilogue<double, false>);
  }
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

sph_status launch_stress(sph_ctx* c, sph_state* st) {
  PassArgs A = make_args(c, st);
  const dim3 g((unsigned)(c->cap_tiles < 4096 ? c->cap_tiles : 4096));   // loops over the work list
  dispatch_cfg(c->p.kernel, c->p.periodic, [&](auto K, auto P) {
    dispatch_lanes(pass_lanes(c->p), [&](auto LL) {
      constexpr int KER = decltype(K)::value;
      constexpr bool PER = decltype(P)::value;
      constexpr int L = decltype(LL)::value;
      const dim3 b(64 * L);
      if (c->p.precision == SPH_FP32)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_stress<float, KER, PER, L>), g, b, 0, c->stream, A, c->pos4f, c->fvf,
                           c->faf, st->S, c->mu, st->dSdt, c->sdot);
      else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_stress<double, KER, PER, L>), g, b, 0, c->stream, A, c->pos4, c->fv,
                           c->fa, st->S, c->mu, st->dSdt, c->sdot);
    });
  });
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

sph_status launch_forces(sph_ctx* c, sph_state* st) {
  PassArgs A = make_args(c, st);
  ForceOut O{st->ax, st->ay, st->az, st->dudt, c->pos4, st->vx, st->vy, st->vz, c->dDdt, c->xcoef, c->capacity, st->D};
  const int xs = (c->p.dtP_mode == SPH_DTP_LAGGED && c->p.background == SPH_TOV) ? kXGP
                 : (c->p.density_mode == SPH_DENS_CONTINUITY || c->p.energy_mode == SPH_ENERGY_FIRST_LAW) ? kXDD
                                                                                                        : 0;
  const dim3 g = pass_grid(c);
  dispatch_cfg(c->p.kernel, c->p.periodic, [&](auto K, auto P) {
    dispatch_lanes(pass_lanes(c->p), [&](auto LL) {
      constexpr int KER = decltype(K)::value;
      constexpr bool PER = decltype(P)::value;
      constexpr int L = decltype(LL)::value;
      const dim3 b(64 * L);
      auto launch = [&](auto XX) {
        constexpr int X = decltype(XX)::value;
        if (c->p.precision == SPH_FP32)
          hipLaunchKernelGGL(HIP_KERNEL_NAME(k_forces<float, KER, PER, L, X>), g, b, 0, c->stream, A, c->pos4f,
                             c->fvf, c->faf, c->sigf, c->tovf, c->sdot, O);
        else
          hipLaunchKernelGGL(HIP_KERNEL_NAME(k_forces<double, KER, PER, L, X>), g, b, 0, c->stream, A, c->pos4,
                             c->fv, c->fa, c->sig, c->tovf, c->sdot, O);
      };
      if (xs == kXGP) launch(std::integral_constant<int, kXGP>{});
      else if (xs == kXDD) launch(std::integral_constant<int, kXDD>{});
      else if (c->stress_heavy && c->p.precision == SPH_FP32)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_forces<float, KER, PER, L, kXSL>), g, b, 0, c->stream, A, c->pos4f,
                           c->fvf, c->faf, c->sigf, c->tovf, c->sdot, O);
      else launch(std::integral_constant<int, 0>{});
    });
  });
  const sph_params& p = c->p;
  if (p.ext == SPH_EXT_RADIAL || p.wall_in > 0.0 || p.wall_out > 0.0 || p.damping > 0.0) {
    const int64_t nb = (A.n + 255) / 256;
    hipLaunchKernelGGL(k_ext_accel, dim3((unsigned)(nb < 4096 ? (nb > 0 ? nb : 1) : 4096)), dim3(256), 0, c->stream, A, O);
  }
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

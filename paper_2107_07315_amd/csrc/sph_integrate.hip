// Kick-drift-kick time integration with the solid-model updates of section "Solid SPH
// Equations": von Mises yield scaling after every stress update and the maximum-strain breaking
// test eps = lambda_max(S) / E, E = 9 B mu / (3 B + mu).  Memory-bound elementwise kernels.
#include "sph_internal.h"

namespace {

constexpr int kB = 256;

struct KdkArgs {
  sph_params p;
  int64_t n;
  int64_t hstride;  // stride of the half-step arrays (capacity)
  double dt;
  double* x; double* y; double* z;
  double* vx; double* vy; double* vz;
  double* u; double* h; double* S;
  const double* ax; const double* ay; const double* az;
  const double* dudt; double* dSdt;
  uint8_t* broken; const int8_t* type;
  const double* D; const double* mu; const double* B; const double* Y0;
  double* half;
  const int32_t* star; const StarInfo* stars;
  DevStatus* status;
  // drift: packed position records for the next evaluation and the skin test
  double4* pos4; float4* pos4f;
  const double4* pos_build; const GridInfo* grid;
  // skin test: a violating particle raises *flag to check_id, this step's number since the flag
  // was cleared; a step finds a smaller non-zero value there when an earlier step (run ahead of
  // the host's test) broke the bound, and then leaves the state alone.  flag == nullptr: no test
  uint32_t check_id; uint32_t* flag;
  // positions and h read from and written to pos4 only (inside a multi-step call the public
  // x, y, z, h are brought up to date once, before a list build and at the end of the call)
  bool deferred;
  // continuity density: D is integrated with the rate of the last evaluation
  bool cont;
  double* Dst;
  const double* dDdt;
  // time step: fixed dt, or (adaptive) the Courant steps committed in dtw[slot]; the kick-drift
  // adds its dt to the simulated time dtw[3] and records it in dtw[5]
  double* dtw;
  int slot_fin, slot_drift;   // < 0: fixed dt
};

__device__ __forceinline__ double dt_of(const KdkArgs& K, int slot) { return slot >= 0 ? K.dtw[slot] : K.dt; }

// a kick of a step that runs ahead of a failed skin test does nothing
__device__ __forceinline__ bool kick_cancelled(const KdkArgs& K) {
  if (!K.flag) return false;
  const uint32_t f = *K.flag;
  return f != 0u && f < K.check_id;
}

__device__ __forceinline__ double wrap(double q, int periodic, double box) {
  if (periodic) {
    if (q >= box) q -= box;
    else if (q < 0.0) q += box;
  }
  return q;
}

// First half kick, drift and predictors of particle a from its start-of-step v, u, S and h:
// stores the half-step copies, x, the predicted v, u and (yielded) S, the packed position records,
// and runs the skin test.  Type-0 particles carry no deviatoric stress (S and its rate are zero,
// set at every list build), so their stress arrays are neither read nor written.
__device__ __forceinline__ void kick_drift_from(const KdkArgs& K, int64_t a, const double x0[3], const double v0[3],
                                                double u0, const double S0[6], double h, bool solid, double D0) {
  const double dt = dt_of(K, K.slot_drift);
  const double hdt = 0.5 * dt;
  const int64_t n = K.n, hs = K.hstride;
  double* H = K.half;
  const double ax = K.ax[a], ay = K.ay[a], az = K.az[a], du = K.dudt[a];
  double vh[3] = {v0[0] + hdt * ax, v0[1] + hdt * ay, v0[2] + hdt * az};
  double uh = u0 + hdt * du;
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (solid)
    for (int c = 0; c < 6; ++c) {
      const double ds = K.dSdt[c * n + a];
      double sh = S0[c] + hdt * ds;
      H[(4 + c) * hs + a] = sh;
      s[c] = sh + hdt * ds;
    }
  H[0 * hs + a] = vh[0];
  H[1 * hs + a] = vh[1];
  H[2 * hs + a] = vh[2];
  H[3 * hs + a] = uh;
  if (K.cont) {   // eq. solid1: half kick and predictor of the computational density
    const double dd = K.dDdt[a];
    const double Dh = D0 + hdt * dd;
    H[10 * hs + a] = Dh;
    K.Dst[a] = Dh + hdt * dd;
  }
  if (a == 0) {   // one lane records the step's dt and advances the simulated time
    K.dtw[5] = dt;
    K.dtw[3] += dt;
  }
  const double xn = wrap(x0[0] + dt * vh[0], K.p.periodic, K.p.box);
  const double yn = wrap(x0[1] + dt * vh[1], K.p.periodic, K.p.box);
  const double zn = wrap(x0[2] + dt * vh[2], K.p.periodic, K.p.box);
  if (!K.deferred) {
    K.x[a] = xn;
    K.y[a] = yn;
    K.z[a] = zn;
  }
  K.pos4[a] = make_double4(xn, yn, zn, h);
  if (K.pos4f) {
    double cx = 0.0, cy = 0.0, cz = 0.0;
    if (K.star && K.stars) {
      const StarInfo si = K.stars[K.star[a]];
      cx = si.cx; cy = si.cy; cz = si.cz;
    }
    K.pos4f[a] = make_float4((float)(xn - cx), (float)(yn - cy), (float)(zn - cz), (float)(0.5 * h));   // h/2
  }
  if (K.flag) {
    const double4 b = K.pos_build[a];
    const int per = K.p.periodic;
    const double box = K.p.box;
    if (skin_exceeded(min_image(xn - b.x, per, box), min_image(yn - b.y, per, box), min_image(zn - b.z, per, box),
                      h, b, K.grid->skin))
      atomicMax(K.flag, K.check_id);
  }
  K.vx[a] = vh[0] + hdt * ax;
  K.vy[a] = vh[1] + hdt * ay;
  K.vz[a] = vh[2] + hdt * az;
  K.u[a] = uh + hdt * du;
  if (solid) {
    yield_scale(K.p.yield_mode, K.Y0[a], s);
    for (int c = 0; c < 6; ++c) K.S[c * n + a] = s[c];
  }
}

// Second half kick of particle a from the half-step copies: end-of-step v, u and S (yield scaling
// and the breaking test applied; breaking is recorded), and the adaptive h of the step's density.
__device__ __forceinline__ void final_kick_of(const KdkArgs& K, int64_t a, double v[3], double& u, double s[6],
                                              double& h, bool solid, double& D) {
  const double hdt = 0.5 * dt_of(K, K.slot_fin);
  const int64_t n = K.n, hs = K.hstride;
  const double* H = K.half;
  v[0] = H[0 * hs + a] + hdt * K.ax[a];
  v[1] = H[1 * hs + a] + hdt * K.ay[a];
  v[2] = H[2 * hs + a] + hdt * K.az[a];
  u = H[3 * hs + a] + hdt * K.dudt[a];
  for (int c = 0; c < 6; ++c) s[c] = 0.0;
  if (solid) {
    for (int c = 0; c < 6; ++c) s[c] = H[(4 + c) * hs + a] + hdt * K.dSdt[c * n + a];
    yield_scale(K.p.yield_mode, K.Y0[a], s);
  }
  if (solid && K.p.break_mode != SPH_BREAK_OFF && !K.broken[a]) {
    const double mu = K.mu[a], Bm = K.B[a];
    if (mu > 0.0) {
      const double E = 9.0 * Bm * mu / (3.0 * Bm + mu);
      const double lm = lambda_max_sym(s[0], s[1], s[2], s[3], s[4], s[5]);
      if (lm / E >= K.p.eps_break) {
        K.broken[a] = 1;
        // FLUIDIZE: no deviatoric stress from here on; the stress rate of the last evaluation
        // goes with it, so that the next half kick does not rebuild a stress
        if (K.p.break_mode == SPH_BREAK_FLUIDIZE)
          for (int c = 0; c < 6; ++c) {
            s[c] = 0.0;
            K.dSdt[c * n + a] = 0.0;
          }
      }
    }
  }
  D = K.cont ? H[10 * hs + a] + hdt * K.dDdt[a] : K.D[a];   // the end-of-step density
  if (K.p.h_mode == SPH_H_ADAPTIVE) {
    double m = (K.star && K.stars) ? K.stars[K.star[a]].m : K.p.m;
    h = K.p.eta * cbrt(m / D);
  } else {
    h = K.h[a];   // constant h: the state's value is always current
  }
}

// half kick, drift, and predictors (velocity, energy, yielded stress) for the evaluation; also
// packs the position records of the evaluation and runs the skin test against the last build
__global__ __launch_bounds__(kB) void k_kick_drift(KdkArgs K) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= K.n || kick_cancelled(K)) return;
  const int64_t n = K.n;
  const bool solid = K.type[a] == 1;
  const double x0[3] = {K.x[a], K.y[a], K.z[a]};
  const double v0[3] = {K.vx[a], K.vy[a], K.vz[a]};
  double S0[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (solid)
    for (int c = 0; c < 6; ++c) S0[c] = K.S[c * n + a];
  kick_drift_from(K, a, x0, v0, K.u[a], S0, K.h[a], solid, K.cont ? K.Dst[a] : 0.0);
}

// second half kick: end-of-step state
__global__ __launch_bounds__(kB) void k_kick_final(KdkArgs K) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= K.n) return;
  const int64_t n = K.n;
  const bool solid = K.type[a] == 1;
  double v[3], u, s[6], h, D;
  final_kick_of(K, a, v, u, s, h, solid, D);
  if (K.cont) K.Dst[a] = D;
  K.vx[a] = v[0];
  K.vy[a] = v[1];
  K.vz[a] = v[2];
  K.u[a] = u;
  if (solid)
    for (int c = 0; c < 6; ++c) K.S[c * n + a] = s[c];
  K.h[a] = h;
}

// The second half kick of one step and the first half kick and drift of the next in one pass:
// the end-of-step v, u, S and h stay in registers (the same arithmetic as the two kernels).
__global__ __launch_bounds__(kB) void k_kick_final_drift(KdkArgs K) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= K.n || kick_cancelled(K)) return;
  const bool solid = K.type[a] == 1;
  double x0[3];
  if (K.deferred) {
    const double4 q = K.pos4[a];
    x0[0] = q.x; x0[1] = q.y; x0[2] = q.z;
  } else {
    x0[0] = K.x[a]; x0[1] = K.y[a]; x0[2] = K.z[a];
  }
  double v[3], u, s[6], h, D;
  final_kick_of(K, a, v, u, s, h, solid, D);
  if (!K.deferred) K.h[a] = h;
  kick_drift_from(K, a, x0, v, u, s, h, solid, D);
}

KdkArgs make_kdk(sph_ctx* c, sph_state* st, double dt) {
  KdkArgs K;
  K.p = c->p;
  K.n = st->n;
  K.hstride = c->capacity;
  K.dt = dt;
  K.x = st->x; K.y = st->y; K.z = st->z;
  K.vx = st->vx; K.vy = st->vy; K.vz = st->vz;
  K.u = st->u; K.h = st->h; K.S = st->S;
  K.ax = st->ax; K.ay = st->ay; K.az = st->az;
  K.dudt = st->dudt; K.dSdt = st->dSdt;
  K.broken = st->broken; K.type = st->type;
  K.D = st->D; K.mu = c->mu; K.B = c->B; K.Y0 = c->Y0;
  K.half = c->half;
  K.star = c->stars ? st->star : nullptr;
  K.stars = c->stars;
  K.status = c->status;
  K.pos4 = c->pos4;
  K.pos4f = c->p.precision == SPH_FP32 ? c->pos4f : nullptr;
  K.pos_build = c->pos_build;
  K.grid = c->grid;
  K.check_id = c->check_id;
  K.flag = nullptr;
  K.deferred = false;
  K.cont = c->p.density_mode == SPH_DENS_CONTINUITY;
  K.Dst = st->D;
  K.dDdt = c->dDdt;
  K.dtw = c->dtw;
  K.slot_fin = K.slot_drift = -1;
  return K;
}

// x, y, z, h of the state from the packed position records
__global__ __launch_bounds__(kB) void k_unpack_pos(const double4* __restrict__ pos4, int64_t n, double* __restrict__ x,
                                                   double* __restrict__ y, double* __restrict__ z,
                                                   double* __restrict__ h) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const double4 q = pos4[a];
  x[a] = q.x;
  y[a] = q.y;
  z[a] = q.z;
  h[a] = q.w;
}

__global__ void k_flag_clear(uint32_t* f) { *f = 0u; }   // a kernel, not a memset: graph-safe

// Courant step of an evaluation: dtw[slot] = cfl * min_a h_a / (c_L,a + |v_a|) from the per-block
// minima of the density epilogue (one workgroup, a fixed reduction order).
__global__ __launch_bounds__(256) void k_dt_commit(double* __restrict__ dtw, int slot, double cfl,
                                                   const double* __restrict__ part, int nb) {
  __shared__ double red[256];
  double m = __builtin_inf();
  for (int b = threadIdx.x; b < nb; b += 256) m = part[b] < m ? part[b] : m;
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x + s] < red[threadIdx.x] ? red[threadIdx.x + s] : red[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) dtw[slot] = cfl * red[0];
}

__global__ void k_dt_init(double* dtw) {
  if (threadIdx.x < 8) dtw[threadIdx.x] = 0.0;
}

// Modification step: u from the profile u(r) of the real EoS at the particle's distance from its
// star centre (linear in the table, its last entry beyond it), velocity zeroed.
__global__ __launch_bounds__(kB) void k_modify_energy(const double* __restrict__ x, const double* __restrict__ y,
                                                      const double* __restrict__ z, int64_t n,
                                                      const int32_t* __restrict__ star,
                                                      const StarInfo* __restrict__ stars,
                                                      const double* __restrict__ u_of_r, int32_t nr, double dr,
                                                      double* __restrict__ u, double* __restrict__ vx,
                                                      double* __restrict__ vy, double* __restrict__ vz) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double cx = 0.0, cy = 0.0, cz = 0.0;
  if (star && stars) {
    const StarInfo si = stars[star[a]];
    cx = si.cx; cy = si.cy; cz = si.cz;
  }
  const double X = x[a] - cx, Y = y[a] - cy, Z = z[a] - cz;
  const double r = sqrt(X * X + Y * Y + Z * Z);
  const double t = r / dr;
  double v;
  if (t >= (double)(nr - 1)) {
    v = u_of_r[nr - 1];
  } else {
    const int i = (int)floor(t);
    const double f = t - (double)i;
    v = (1.0 - f) * u_of_r[i] + f * u_of_r[i + 1];
  }
  u[a] = v;
  vx[a] = 0.0;
  vy[a] = 0.0;
  vz[a] = 0.0;
}
}  // namespace

sph_status launch_modify_energy(sph_ctx* c, sph_state* st, const double* u_of_r, int32_t nr, double dr) {
  hipLaunchKernelGGL(k_modify_energy, dim3(grid_for(st->n, kB)), dim3(kB), 0, c->stream, st->x, st->y, st->z, st->n,
                     c->stars ? st->star : nullptr, c->stars, u_of_r, nr, dr, st->u, st->vx, st->vy, st->vz);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

sph_status launch_dt_commit(sph_ctx* c, int slot) {
  if (c->eos_blocks <= 0) return SPH_OK;
  hipLaunchKernelGGL(k_dt_commit, dim3(1), dim3(256), 0, c->stream, c->dtw, slot, c->p.cfl > 0.0 ? c->p.cfl : 0.3,
                     c->dtpart, c->eos_blocks);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

sph_status launch_dt_init(sph_ctx* c) {
  hipLaunchKernelGGL(k_dt_init, dim3(1), dim3(64), 0, c->stream, c->dtw);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

sph_status launch_flag_clear(sph_ctx* c) {
  hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(1), 0, c->stream, c->drift_flag);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

sph_status launch_kick_drift(sph_ctx* c, sph_state* st, double dt, uint32_t check, bool deferred, int slot) {
  KdkArgs K = make_kdk(c, st, dt);
  K.slot_drift = slot;
  if (check) { K.flag = c->drift_flag; K.check_id = check; }
  K.deferred = deferred;
  hipLaunchKernelGGL(k_kick_drift, dim3(grid_for(st->n, kB)), dim3(kB), 0, c->stream, K);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

sph_status launch_kick_final_drift(sph_ctx* c, sph_state* st, double dt, uint32_t check, bool deferred, int slot_fin,
                                   int slot_drift) {
  KdkArgs K = make_kdk(c, st, dt);
  K.slot_fin = slot_fin;
  K.slot_drift = slot_drift;
  if (check) { K.flag = c->drift_flag; K.check_id = check; }
  K.deferred = deferred;
  hipLaunchKernelGGL(k_kick_final_drift, dim3(grid_for(st->n, kB)), dim3(kB), 0, c->stream, K);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

sph_status launch_unpack_pos(sph_ctx* c, sph_state* st) {
  hipLaunchKernelGGL(k_unpack_pos, dim3(grid_for(st->n, kB)), dim3(kB), 0, c->stream, c->pos4, st->n, st->x, st->y,
                     st->z, st->h);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

sph_status launch_kick_final(sph_ctx* c, sph_state* st, double dt, int slot) {
  KdkArgs K = make_kdk(c, st, dt);
  K.slot_fin = slot;
  hipLaunchKernelGGL(k_kick_final, dim3(grid_for(st->n, kB)), dim3(kB), 0, c->stream, K);
  HIP_TRY(hipGetLastError());
  return SPH_OK;
}

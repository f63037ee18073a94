// Oscillation diagnostics of sections "Spherically symmetric and static neutron star tests" and
// "Neutron Star Oscillations with a solid crust": kinetic energy and its toroidal part, internal
// energy, the mean u of a radial band (radial modes are read from u) and the linear least-squares
// fit of v_theta over a slab in (r, theta) (non-radial modes).  One pass over the particles with
// per-block partial sums in FP64, then one block that adds the partials in a fixed order and
// solves the 3x3 normal equations, so a result does not depend on scheduling.  HBM-bound: 80 B per
// particle read.
#include "sph_internal.h"

namespace {

constexpr int kB = 256;
constexpr int kMaxBlocks = 1024;
constexpr int kSums = 18;   // ke, tor, ein, u_band, n_band, n_slab, M00 M01 M02 M11 M12 M22, r0 r1 r2, pvf, pff, pad

__global__ __launch_bounds__(kB) void k_diag_partials(const double* __restrict__ x, const double* __restrict__ y,
                                                      const double* __restrict__ z, const double* __restrict__ vx,
                                                      const double* __restrict__ vy, const double* __restrict__ vz,
                                                      const double* __restrict__ u, int64_t n, double m,
                                                      const int32_t* __restrict__ star,
                                                      const StarInfo* __restrict__ stars, sph_diag_params dp,
                                                      double* __restrict__ part) {
  double s[kSums];
#pragma unroll
  for (int k = 0; k < kSums; ++k) s[k] = 0.0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
    const double ma = (star && stars) ? stars[star[a]].m : m;
    const double X = x[a], Y = y[a], Z = z[a];
    const double VX = vx[a], VY = vy[a], VZ = vz[a];
    const double r = sqrt(X * X + Y * Y + Z * Z);
    const double rc = sqrt(X * X + Y * Y);
    s[0] += 0.5 * ma * (VX * VX + VY * VY + VZ * VZ);
    s[2] += ma * u[a];
    if (rc > 0.0) {
      const double vphi = (-Y * VX + X * VY) / rc;   // e_phi = (-sin phi, cos phi, 0)
      s[1] += 0.5 * ma * vphi * vphi;
      const double f = 3.0 * (rc / r) * (Z / r);     // l = 2 toroidal profile 3 sin(theta) cos(theta)
      s[15] += ma * vphi * f;
      s[16] += ma * f * f;
    }
    if (r >= dp.r_lo && r < dp.r_hi) {
      s[3] += u[a];
      s[4] += 1.0;
    }
    if (r > 0.0 && rc > 0.0) {
      const double th = acos(Z / r);
      if (fabs(r - dp.slab_r) <= dp.slab_dr && fabs(th - dp.slab_th) <= dp.slab_dth) {
        const double ct = Z / r, st = rc / r;
        const double vth = ct * (X * VX + Y * VY) / rc - st * VZ;   // e_theta = (ct cp, ct sp, -st)
        const double f1 = r - dp.slab_r, f2 = th - dp.slab_th;
        s[5] += 1.0;
        s[6] += 1.0;
        s[7] += f1;
        s[8] += f2;
        s[9] += f1 * f1;
        s[10] += f1 * f2;
        s[11] += f2 * f2;
        s[12] += vth;
        s[13] += f1 * vth;
        s[14] += f2 * vth;
      }
    }
  }
  // block sum: wave shuffles, then the four waves through LDS in a fixed order
  __shared__ double red[kB / 64][kSums];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kSums; ++k) {
    double v = s[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kSums) {
    double v = 0.0;
    for (int w = 0; w < kB / 64; ++w) v += red[w][threadIdx.x];
    part[(int64_t)blockIdx.x * kSums + threadIdx.x] = v;
  }
}

__device__ __forceinline__ double det3(double a00, double a01, double a02, double a10, double a11, double a12,
                                       double a20, double a21, double a22) {
  return a00 * (a11 * a22 - a12 * a21) - a01 * (a10 * a22 - a12 * a20) + a02 * (a10 * a21 - a11 * a20);
}

__global__ __launch_bounds__(64) void k_diag_final(const double* __restrict__ part, int nblocks,
                                                   sph_diag* __restrict__ out) {
  __shared__ double tot[kSums];
  if (threadIdx.x < kSums) {
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += part[(int64_t)b * kSums + threadIdx.x];
    tot[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  sph_diag d;
  d.kinetic = tot[0];
  d.toroidal = tot[1];
  d.internal = tot[2];
  d.n_band = (int64_t)tot[4];
  d.u_band = tot[4] > 0.0 ? tot[3] / tot[4] : 0.0;
  d.n_slab = (int64_t)tot[5];
  d.tor_l2 = tot[16] > 0.0 ? tot[15] / tot[16] : 0.0;
  const double M00 = tot[6], M01 = tot[7], M02 = tot[8], M11 = tot[9], M12 = tot[10], M22 = tot[11];
  const double r0 = tot[12], r1 = tot[13], r2 = tot[14];
  const double det = det3(M00, M01, M02, M01, M11, M12, M02, M12, M22);
  d.slab_c0 = d.slab_cr = d.slab_cth = 0.0;
  if (d.n_slab >= 3 && det != 0.0) {   // Cramer's rule on the normal equations
    d.slab_c0 = det3(r0, M01, M02, r1, M11, M12, r2, M12, M22) / det;
    d.slab_cr = det3(M00, r0, M02, M01, r1, M12, M02, r2, M22) / det;
    d.slab_cth = det3(M00, M01, r0, M01, M11, r1, M02, M12, r2) / det;
  }
  *out = d;
}

}  // namespace

extern "C" sph_status sph_diagnostics(sph_ctx* c, const sph_state* st, const sph_diag_params* dp, sph_diag* out) {
  if (!c) return note(nullptr, SPH_E_ARG, "context is NULL");
  if (!st || !dp || !out) return note(c, SPH_E_ARG, "state, params and out must not be NULL");
  if (st->n < 0 || st->n > c->capacity) return note(c, SPH_E_ARG, "n = %lld outside [0, capacity]", (long long)st->n);
  if (st->n > 0 && (!st->x || !st->y || !st->z || !st->vx || !st->vy || !st->vz || !st->u))
    return note(c, SPH_E_ARG, "diagnostics need x, y, z, vx, vy, vz and u");
  if (!c->diag_part) {
    if (hipMalloc((void**)&c->diag_part, sizeof(double) * kSums * kMaxBlocks) != hipSuccess) {
      c->diag_part = nullptr;
      return note(c, SPH_E_OOM, "diagnostics partial sums");
    }
  }
  int nb = (int)grid_for(st->n > 0 ? st->n : 1, kB);
  nb = nb < kMaxBlocks ? nb : kMaxBlocks;
  hipLaunchKernelGGL(k_diag_partials, dim3(nb), dim3(kB), 0, c->stream, st->x, st->y, st->z, st->vx, st->vy, st->vz,
                     st->u, st->n, c->p.m, c->stars ? st->star : nullptr, c->stars, *dp, c->diag_part);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, c->stream, c->diag_part, nb, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return note(c, SPH_E_HIP, "diagnostics launch: %s", hipGetErrorString(e));
  return SPH_OK;
}

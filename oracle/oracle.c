/*
 * CPU FP64 oracle for the SPH particle loop of Tsao et al., "Modeling Neutron Star
 * Oscillations in a Fixed General Relativistic Background Including Solid Crust Dynamics".
 *
 * TEST INFRASTRUCTURE ONLY: the slow, plain reference the GPU path is checked against.
 * Built with -O2 -ffp-contract=off (no FMA contraction, no fast-math), OpenMP over
 * particles.  Each per-particle sum runs over the neighbour list in increasing index order.
 *
 * Section/equation references are to the paper:
 *   eq. solid1..solid6  conservation equations, stress rate, strain/rotation rates
 *   "von Mises"         yield scaling S -> f S, f = min(Y0^2/sigma_v^2, 1)
 *   "maximum-strain"    eps = sigma_max / E, E = 9 B mu / (3 B + mu)
 *   "3+1"               ds^2 = -alpha^2 dt^2 + gamma_ij dx^i dx^j (zero shift)
 *   "trajectory"        the fluid trajectory equation of the fixed-background section
 *   "computational density"  D = rho sqrt(gamma) W
 *
 * Readings where the paper is silent or inconsistent (each listed in the design notes):
 *  - pressure coefficient of the trajectory equation taken as 1/(W~^2 rho h), the form that
 *    holds a TOV star static (the printed 1/(W~ rho h) does not);
 *  - rotation term of eq. solid4 taken with the objective (Jaumann) sign R S - S R; the
 *    printed sign is available as ORC_ROT_LITERAL;
 *  - computational density D used for rho in every pair sum; proper rho only in the EoS;
 *  - Monaghan (1992) form of the unspecified artificial viscosity Pi_ab;
 *  - Wendland C2/C4 kernels with support h_a + h_b;
 *  - principal stresses of the deviatoric S for the breaking test; B = rho h c_s^2.
 * The fixed-background acceleration and the energy equation in that background are
 * "parity unpinned" beyond the continuum static-equilibrium check: no closed form exists
 * for them on a particle star.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------------------ */
/* geometry                                                                              */

static inline double min_image(double d, int periodic, double L) {
  if (periodic) {
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
  }
  return d;
}

/* b is a neighbour of a iff r^2 < (h_a + h_b)^2, each operation rounded in this order. */
static inline int is_neighbour(const orc_params* p, double xa, double ya, double za, double ha,
                               double xb, double yb, double zb, double hb) {
  double dx = min_image(xa - xb, p->periodic, p->box);
  double dy = min_image(ya - yb, p->periodic, p->box);
  double dz = min_image(za - zb, p->periodic, p->box);
  double r2 = (dx * dx + dy * dy) + dz * dz;
  double H = ha + hb;
  return r2 < H * H;
}

/* ------------------------------------------------------------------------------------ */
/* kernel                                                                                */

void orc_kernel(int32_t kernel, double r, double hab, double* W, double* F) {
  double q = r / hab;
  if (q >= 2.0) { *W = 0.0; *F = 0.0; return; }
  double t = 1.0 - 0.5 * q;
  double h3 = hab * hab * hab, h5 = h3 * hab * hab;
  if (kernel == ORC_WC4) {
    /* Wendland C4 with support 2h: 495/(256 pi h^3) t^6 (1 + 3q + 35 q^2/12) */
    double t5 = t * t * t * t * t;
    *W = 495.0 / (256.0 * PI * h3) * t5 * t * (1.0 + 3.0 * q + 35.0 / 12.0 * q * q);
    *F = -1155.0 / (128.0 * PI * h5) * t5 * (1.0 + 2.5 * q);
  } else {
    /* Wendland C2 with support 2h: 21/(16 pi h^3) t^4 (1 + 2q) */
    double t3 = t * t * t;
    *W = 21.0 / (16.0 * PI * h3) * t3 * t * (1.0 + 2.0 * q);
    *F = -105.0 / (16.0 * PI * h5) * t3;
  }
}

/* Condition number of the kernel-gradient factor F with respect to q = r/h_ab:
 * 1 + q |d ln F / d q|.  Near the support edge F ~ t^k with t = 1 - q/2 small, so a relative
 * perturbation of q (from rounding r or h_ab) is amplified; the parity bound kappa carries it. */
static double kernel_cond(int32_t kernel, double r, double hab) {
  double q = r / hab;
  if (q >= 2.0) return 1.0;
  double t = 1.0 - 0.5 * q;
  if (!(t > 0.0)) return 1.0;
  double dl = (kernel == ORC_WC4) ? (-2.5 / t + 2.5 / (1.0 + 2.5 * q)) : (-1.5 / t);
  return 1.0 + q * fabs(dl);
}

/* ------------------------------------------------------------------------------------ */
/* neighbour sets                                                                        */

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

static int neighbours_brute(const orc_params* p, int64_t n, const double* x, const double* y,
                            const double* z, const double* h, int64_t* off, int32_t* ids,
                            int64_t cap) {
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return ORC_E_OOM;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t a = 0; a < n; ++a) {
    int64_t c = 0;
    for (int64_t b = 0; b < n; ++b)
      if (b != a && is_neighbour(p, x[a], y[a], z[a], h[a], x[b], y[b], z[b], h[b])) ++c;
    cnt[a] = c;
  }
  off[0] = 0;
  for (int64_t a = 0; a < n; ++a) off[a + 1] = off[a] + cnt[a];
  free(cnt);
  if (off[n] > cap) return ORC_E_NGB_CAPACITY;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t a = 0; a < n; ++a) {
    int64_t k = off[a];
    for (int64_t b = 0; b < n; ++b)
      if (b != a && is_neighbour(p, x[a], y[a], z[a], h[a], x[b], y[b], z[b], h[b]))
        ids[k++] = (int32_t)b;
  }
  return ORC_OK;
}

/* Uniform grid with cell size about 2 h_min.  Each unordered pair {a, b} is found once, by
 * the member with the larger (h, index): r < h_a + h_b <= 2 max(h_a, h_b), so scanning the
 * cells within 2 h_a of particle a is enough.  Lists are then symmetrised and sorted. */
static int neighbours_grid(const orc_params* p, int64_t n, const double* x, const double* y,
                           const double* z, const double* h, int64_t* off, int32_t* ids,
                           int64_t cap) {
  double hmin = h[0], lo[3], hi[3];
  lo[0] = hi[0] = x[0]; lo[1] = hi[1] = y[0]; lo[2] = hi[2] = z[0];
  for (int64_t a = 0; a < n; ++a) {
    if (h[a] < hmin) hmin = h[a];
    double q[3] = {x[a], y[a], z[a]};
    for (int d = 0; d < 3; ++d) { if (q[d] < lo[d]) lo[d] = q[d]; if (q[d] > hi[d]) hi[d] = q[d]; }
  }
  if (!(hmin > 0.0)) return ORC_E_ARG;
  double c = 2.0 * hmin;
  int64_t dims[3];
  for (;;) {
    int64_t tot = 1;
    for (int d = 0; d < 3; ++d) {
      if (p->periodic) {
        dims[d] = (int64_t)floor(p->box / c);
        if (dims[d] < 1) dims[d] = 1;
      } else {
        dims[d] = (int64_t)floor((hi[d] - lo[d]) / c) + 1;
      }
      tot *= dims[d];
    }
    if (tot <= ((int64_t)1 << 25)) break;
    c *= 1.25;
  }
  double cs[3];
  for (int d = 0; d < 3; ++d) {
    if (p->periodic) { lo[d] = 0.0; cs[d] = p->box / (double)dims[d]; }
    else cs[d] = c;
  }
  int64_t ncell = dims[0] * dims[1] * dims[2];
  int64_t* cstart = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
  int64_t* cellof = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* items = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t* lo_cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cstart || !cellof || !items || !lo_cnt) {
    free(cstart); free(cellof); free(items); free(lo_cnt); return ORC_E_OOM;
  }
  for (int64_t a = 0; a < n; ++a) {
    double q[3] = {x[a], y[a], z[a]};
    int64_t ci[3];
    for (int d = 0; d < 3; ++d) {
      int64_t k = (int64_t)floor((q[d] - lo[d]) / cs[d]);
      if (k < 0) k = 0;
      if (k > dims[d] - 1) k = dims[d] - 1;
      ci[d] = k;
    }
    cellof[a] = (ci[2] * dims[1] + ci[1]) * dims[0] + ci[0];
    cstart[cellof[a] + 1]++;
  }
  for (int64_t k = 0; k < ncell; ++k) cstart[k + 1] += cstart[k];
  {
    int64_t* cur = (int64_t*)malloc((size_t)ncell * sizeof(int64_t));
    if (!cur) { free(cstart); free(cellof); free(items); free(lo_cnt); return ORC_E_OOM; }
    memcpy(cur, cstart, (size_t)ncell * sizeof(int64_t));
    for (int64_t a = 0; a < n; ++a) items[cur[cellof[a]]++] = (int32_t)a;  /* ascending */
    free(cur);
  }

  int64_t* lo_off = NULL;
  int32_t* lo_ids = NULL;
  for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < n; ++a) {
      int64_t ca[3] = {cellof[a] % dims[0], (cellof[a] / dims[0]) % dims[1],
                       cellof[a] / (dims[0] * dims[1])};
      int64_t rlo[3], rhi[3];
      int wrap[3];
      for (int d = 0; d < 3; ++d) {
        int64_t k = (int64_t)ceil(2.0 * h[a] / cs[d]);
        wrap[d] = 0;
        if (p->periodic) {
          if (2 * k + 1 >= dims[d]) { rlo[d] = 0; rhi[d] = dims[d] - 1; }
          else { rlo[d] = ca[d] - k; rhi[d] = ca[d] + k; wrap[d] = 1; }
        } else {
          rlo[d] = ca[d] - k < 0 ? 0 : ca[d] - k;
          rhi[d] = ca[d] + k > dims[d] - 1 ? dims[d] - 1 : ca[d] + k;
        }
      }
      int64_t c_found = 0, w = pass ? lo_off[a] : 0;
      for (int64_t kz = rlo[2]; kz <= rhi[2]; ++kz)
        for (int64_t ky = rlo[1]; ky <= rhi[1]; ++ky)
          for (int64_t kx = rlo[0]; kx <= rhi[0]; ++kx) {
            int64_t k3[3] = {kx, ky, kz};
            for (int d = 0; d < 3; ++d)
              if (wrap[d]) k3[d] = ((k3[d] % dims[d]) + dims[d]) % dims[d];
            int64_t cell = (k3[2] * dims[1] + k3[1]) * dims[0] + k3[0];
            for (int64_t s = cstart[cell]; s < cstart[cell + 1]; ++s) {
              int64_t b = items[s];
              int precedes = (h[b] < h[a]) || (h[b] == h[a] && b < a);
              if (!precedes) continue;
              if (!is_neighbour(p, x[a], y[a], z[a], h[a], x[b], y[b], z[b], h[b])) continue;
              if (pass) lo_ids[w++] = (int32_t)b;
              else ++c_found;
            }
          }
      if (!pass) lo_cnt[a] = c_found;
    }
    if (!pass) {
      lo_off = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
      if (!lo_off) { free(cstart); free(cellof); free(items); free(lo_cnt); return ORC_E_OOM; }
      lo_off[0] = 0;
      for (int64_t a = 0; a < n; ++a) lo_off[a + 1] = lo_off[a] + lo_cnt[a];
      lo_ids = (int32_t*)malloc(((size_t)lo_off[n] + 1) * sizeof(int32_t));
      if (!lo_ids) { free(cstart); free(cellof); free(items); free(lo_cnt); free(lo_off); return ORC_E_OOM; }
    }
  }
  free(cstart); free(cellof); free(items);
  /* degrees of the symmetric relation */
  int64_t* deg = lo_cnt;
  for (int64_t a = 0; a < n; ++a)
    for (int64_t s = lo_off[a]; s < lo_off[a + 1]; ++s) deg[lo_ids[s]]++;
  off[0] = 0;
  for (int64_t a = 0; a < n; ++a) off[a + 1] = off[a] + deg[a];
  if (off[n] > cap) { free(lo_off); free(lo_ids); free(lo_cnt); return ORC_E_NGB_CAPACITY; }
  int64_t* cur = deg;  /* reuse as cursors */
  for (int64_t a = 0; a < n; ++a) cur[a] = off[a];
  for (int64_t a = 0; a < n; ++a)
    for (int64_t s = lo_off[a]; s < lo_off[a + 1]; ++s) {
      int32_t b = lo_ids[s];
      ids[cur[a]++] = b;
      ids[cur[b]++] = (int32_t)a;
    }
  free(lo_off); free(lo_ids); free(lo_cnt);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t a = 0; a < n; ++a)
    qsort(ids + off[a], (size_t)(off[a + 1] - off[a]), sizeof(int32_t), cmp_i32);
  return ORC_OK;
}

int orc_neighbours(const orc_params* p, int64_t n, const double* x, const double* y,
                   const double* z, const double* h, int32_t mode, int64_t* offsets,
                   int32_t* ids, int64_t cap) {
  if (n < 0 || !offsets) return ORC_E_ARG;
  offsets[0] = 0;
  if (n == 0) return ORC_OK;
  if (p->periodic) {
    for (int64_t a = 0; a < n; ++a)
      if (!(2.0 * h[a] < 0.5 * p->box)) return ORC_E_ARG;  /* one image per pair */
  }
  if (mode == ORC_NGB_BRUTE) return neighbours_brute(p, n, x, y, z, h, offsets, ids, cap);
  return neighbours_grid(p, n, x, y, z, h, offsets, ids, cap);
}

/* ------------------------------------------------------------------------------------ */
/* background metric (isotropic coordinates, zero shift)                                 */

typedef struct { double alpha, dalpha, psi, dpsi, n[3], rbar; } metric_t;

/* particle mass, shear factor and background centre of particle a (its star's in an ensemble) */
static inline int has_stars(const orc_params* p, const orc_state* st) { return p->nstars > 0 && p->star_info && st->star; }
static inline double pmass(const orc_params* p, const orc_state* st, int64_t a) {
  return has_stars(p, st) ? p->star_info[5 * st->star[a] + 3] : p->m;
}
static inline double pmufac(const orc_params* p, const orc_state* st, int64_t a) {
  return has_stars(p, st) ? p->star_info[5 * st->star[a] + 4] : p->mu_pfactor;
}
static inline void pcentre(const orc_params* p, const orc_state* st, int64_t a, double c[3]) {
  c[0] = c[1] = c[2] = 0.0;
  if (has_stars(p, st))
    for (int k = 0; k < 3; ++k) c[k] = p->star_info[5 * st->star[a] + k];
}

static metric_t metric_at(const orc_params* p, double x, double y, double z) {
  metric_t g;
  double rb = sqrt(x * x + y * y + z * z);
  g.rbar = rb;
  if (rb > 0.0) { g.n[0] = x / rb; g.n[1] = y / rb; g.n[2] = z / rb; }
  else { g.n[0] = g.n[1] = g.n[2] = 0.0; }
  double Rbar = p->bg_dr * (double)(p->bg_n - 1);
  if (rb <= Rbar) {
    double t = rb / p->bg_dr;
    int64_t i = (int64_t)floor(t);
    if (i > p->bg_n - 2) i = p->bg_n - 2;
    double f = t - (double)i;
    const double* T = p->bg;
    int64_t nb = p->bg_n;
    g.alpha = (1.0 - f) * T[i] + f * T[i + 1];
    g.dalpha = (1.0 - f) * T[nb + i] + f * T[nb + i + 1];
    g.psi = (1.0 - f) * T[2 * nb + i] + f * T[2 * nb + i + 1];
    g.dpsi = (1.0 - f) * T[3 * nb + i] + f * T[3 * nb + i + 1];
  } else {
    /* exterior Schwarzschild in isotropic radius */
    double a = p->bg_M / (2.0 * rb);
    g.psi = 1.0 + a;
    g.alpha = (1.0 - a) / (1.0 + a);
    g.dpsi = -a / rb;
    g.dalpha = 2.0 / ((1.0 + a) * (1.0 + a)) * a / rb;
  }
  return g;
}

/* ------------------------------------------------------------------------------------ */
/* equation of state                                                                     */

/* Returns 0 on success; fills P and the sound speed squared. */
static int eos_eval(const orc_params* p, double rho, double u, double* P, double* cs2) {
  if (p->eos == ORC_EOS_TABLE) {
    if (!(rho > 0.0) || !(u > 0.0)) return ORC_E_EOS_DOMAIN;
    double fr = (log(rho) - p->tab_lnr0) / p->tab_dlnr;
    double fu = (log(u) - p->tab_lnu0) / p->tab_dlnu;
    if (!(fr >= 0.0) || !(fu >= 0.0) || fr > (double)(p->tab_nr - 1) || fu > (double)(p->tab_nu - 1))
      return ORC_E_EOS_DOMAIN;
    int64_t i = (int64_t)floor(fr), j = (int64_t)floor(fu);
    if (i > p->tab_nr - 2) i = p->tab_nr - 2;
    if (j > p->tab_nu - 2) j = p->tab_nu - 2;
    double a = fr - (double)i, b = fu - (double)j;
    int64_t nu = p->tab_nu;
    const double* T[2] = {p->tab_lnP, p->tab_lncs2};
    double v[2];
    for (int k = 0; k < 2; ++k) {
      double f00 = T[k][i * nu + j], f01 = T[k][i * nu + j + 1];
      double f10 = T[k][(i + 1) * nu + j], f11 = T[k][(i + 1) * nu + j + 1];
      if (!isfinite(f00) || !isfinite(f01) || !isfinite(f10) || !isfinite(f11)) return ORC_E_EOS_DOMAIN;
      v[k] = (1.0 - a) * ((1.0 - b) * f00 + b * f01) + a * ((1.0 - b) * f10 + b * f11);
    }
    *P = exp(v[0]);
    *cs2 = exp(v[1]);
    return 0;
  }
  /* Gamma law P = (Gamma - 1) rho u */
  *P = (p->gamma - 1.0) * rho * u;
  if (p->background == ORC_TOV) {
    double hen = 1.0 + u + *P / rho;       /* specific enthalpy */
    *cs2 = p->gamma * *P / (rho * hen);    /* relativistic sound speed */
  } else {
    *cs2 = p->gamma * *P / rho;            /* Newtonian sound speed */
  }
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* density                                                                               */

int orc_density(const orc_params* p, orc_state* st, const int64_t* off, const int32_t* ids) {
  int64_t n = st->n;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(max : err)
  for (int64_t a = 0; a < n; ++a) {
    double Wself, Fself;
    orc_kernel(p->kernel, 0.0, st->h[a], &Wself, &Fself);
    /* D_a = sum over b in N(a) and b = a of m W(r_ab, h_ab), ascending b */
    double D = 0.0;
    int self_done = 0;
    for (int64_t s = off[a]; s < off[a + 1]; ++s) {
      int64_t b = ids[s];
      if (!self_done && b > a) { D += pmass(p, st, a) * Wself; self_done = 1; }
      double dx = min_image(st->x[a] - st->x[b], p->periodic, p->box);
      double dy = min_image(st->y[a] - st->y[b], p->periodic, p->box);
      double dz = min_image(st->z[a] - st->z[b], p->periodic, p->box);
      double r = sqrt((dx * dx + dy * dy) + dz * dz);
      double W, F;
      orc_kernel(p->kernel, r, 0.5 * (st->h[a] + st->h[b]), &W, &F);
      D += pmass(p, st, b) * W;
    }
    if (!self_done) D += pmass(p, st, a) * Wself;
    if (p->density_mode == ORC_DENS_CONTINUITY) D = st->D[a];   /* eq. solid1: D is integrated */
    else st->D[a] = D;

    /* rest-mass density from the computational density D = rho psi^6 W_L */
    double rho = D, hen_fac = 1.0;
    if (p->background == ORC_TOV) {
      double c[3];
      pcentre(p, st, a, c);
      metric_t g = metric_at(p, st->x[a] - c[0], st->y[a] - c[1], st->z[a] - c[2]);
      double v2 = st->vx[a] * st->vx[a] + st->vy[a] * st->vy[a] + st->vz[a] * st->vz[a];
      double psi2 = g.psi * g.psi, psi4 = psi2 * psi2, psi6 = psi4 * psi2;
      double vv = psi4 * v2 / (g.alpha * g.alpha);   /* v^i v_i with v^i = xdot^i / alpha */
      double WL = 1.0 / sqrt(1.0 - vv);
      rho = D / (psi6 * WL);
    }
    double P, cs2;
    int e = eos_eval(p, rho, st->u[a], &P, &cs2);
    if (e) { err = e > err ? e : err; P = NAN; cs2 = NAN; }
    if (p->background == ORC_TOV) hen_fac = 1.0 + st->u[a] + P / rho;
    st->rho[a] = rho;
    st->P[a] = P;
    st->cs[a] = sqrt(cs2);
    /* bulk modulus B = n dP/dn = rho h c_s^2 (= Gamma P for the Gamma law) */
    double B = rho * hen_fac * cs2;
    st->B[a] = B;
    double mu = 0.0;
    int solid = st->type[a] == 1 && !(st->broken[a] && p->break_mode == ORC_BREAK_FLUIDIZE);
    if (solid) mu = (p->mu_mode == ORC_MU_PFACTOR) ? pmufac(p, st, a) * P : p->mu_const;
    st->mu[a] = mu;
    double E = (mu > 0.0) ? 9.0 * B * mu / (3.0 * B + mu) : 0.0;
    st->Y0[a] = (p->y0_mode == ORC_Y0_EFACTOR) ? p->y0_over_E * E : p->y0_const;
    if (!isfinite(D) || !isfinite(rho) || !isfinite(P) || !isfinite(cs2))
      err = err > ORC_E_NONFINITE ? err : ORC_E_NONFINITE;
  }
  return err;
}

/* ------------------------------------------------------------------------------------ */
/* stress rate                                                                           */

static inline void s6_to_m(const double* S, int64_t n, int64_t a, double M[3][3]) {
  M[0][0] = S[0 * n + a]; M[1][1] = S[1 * n + a]; M[2][2] = S[2 * n + a];
  M[0][1] = M[1][0] = S[3 * n + a];
  M[0][2] = M[2][0] = S[4 * n + a];
  M[1][2] = M[2][1] = S[5 * n + a];
}

int orc_stress_rate(const orc_params* p, orc_state* st, const int64_t* off, const int32_t* ids,
                    double* kappa_G) {
  int64_t n = st->n;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t a = 0; a < n; ++a) {
    int solid = st->type[a] == 1 && !(st->broken[a] && p->break_mode == ORC_BREAK_FLUIDIZE);
    if (!solid) {
      for (int k = 0; k < 6; ++k) st->dSdt[k * n + a] = 0.0;
      st->sdot[a] = 0.0;
      if (kappa_G) kappa_G[a] = 0.0;
      continue;
    }
    /* G^ij = sum_b m (v_b - v_a)^i d_j W_ab   (eqs. solid5, solid6 before the 1/(2 rho) factor) */
    double G[3][3] = {{0}}, kap = 0.0;
    double va[3] = {st->vx[a], st->vy[a], st->vz[a]};
    for (int64_t s = off[a]; s < off[a + 1]; ++s) {
      int64_t b = ids[s];
      double d[3];
      d[0] = min_image(st->x[a] - st->x[b], p->periodic, p->box);
      d[1] = min_image(st->y[a] - st->y[b], p->periodic, p->box);
      d[2] = min_image(st->z[a] - st->z[b], p->periodic, p->box);
      double r = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
      double W, F;
      orc_kernel(p->kernel, r, 0.5 * (st->h[a] + st->h[b]), &W, &F);
      double g[3] = {F * d[0], F * d[1], F * d[2]};
      double kc = kernel_cond(p->kernel, r, 0.5 * (st->h[a] + st->h[b]));
      double vba[3] = {st->vx[b] - va[0], st->vy[b] - va[1], st->vz[b] - va[2]};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          G[i][j] += pmass(p, st, b) * vba[i] * g[j];
          kap += fabs(pmass(p, st, b) * vba[i] * g[j]) * kc;
        }
    }
    if (kappa_G) kappa_G[a] = kap;
    double D = st->D[a];
    double ed[3][3], Rd[3][3], S[3][3], dS[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        ed[i][j] = (G[i][j] + G[j][i]) / (2.0 * D);   /* strain rate, eq. solid5 */
        Rd[i][j] = (G[i][j] - G[j][i]) / (2.0 * D);   /* rotation rate, eq. solid6 */
      }
    s6_to_m(st->S, n, a, S);
    double tr = ed[0][0] + ed[1][1] + ed[2][2];
    double mu = st->mu[a];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double RS = 0.0, SR = 0.0;
        for (int l = 0; l < 3; ++l) { RS += Rd[i][l] * S[l][j]; SR += S[i][l] * Rd[l][j]; }
        double rot = (p->rotation == ORC_ROT_LITERAL) ? (SR - RS) : (RS - SR);
        dS[i][j] = 2.0 * mu * (ed[i][j] - (i == j ? tr / 3.0 : 0.0)) + rot;   /* eq. solid4 */
      }
    st->dSdt[0 * n + a] = dS[0][0];
    st->dSdt[1 * n + a] = dS[1][1];
    st->dSdt[2 * n + a] = dS[2][2];
    st->dSdt[3 * n + a] = dS[0][1];
    st->dSdt[4 * n + a] = dS[0][2];
    st->dSdt[5 * n + a] = dS[1][2];
    double se = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) se += S[i][j] * ed[i][j];
    st->sdot[a] = se / D;                               /* S^ij epsdot^ij / rho, eq. solid3 */
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------ */
/* forces                                                                                */

typedef struct { double AP[3], AS[3], udot, kP, kS, kU, dd, uvisc, gp, kD, kgp; } pairsum_t;

/* Momentum and energy pair sums of eqs. solid2 and solid3 for particle a (D in place of rho). */
static pairsum_t pair_sums(const orc_params* p, const orc_state* st, int64_t a, const int32_t* list,
                           int64_t cnt) {
  pairsum_t o;
  memset(&o, 0, sizeof(o));
  int64_t n = st->n;
  double Da = st->D[a];
  double pia = st->P[a] / (Da * Da);
  double Sa[3][3], Sb[3][3];
  s6_to_m(st->S, n, a, Sa);
  for (int64_t s = 0; s < cnt; ++s) {
    int64_t b = list[s];
    double d[3];
    d[0] = min_image(st->x[a] - st->x[b], p->periodic, p->box);
    d[1] = min_image(st->y[a] - st->y[b], p->periodic, p->box);
    d[2] = min_image(st->z[a] - st->z[b], p->periodic, p->box);
    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    double r = sqrt(r2);
    double hab = 0.5 * (st->h[a] + st->h[b]);
    double W, F;
    orc_kernel(p->kernel, r, hab, &W, &F);
    double g[3] = {F * d[0], F * d[1], F * d[2]};
    double kc = kernel_cond(p->kernel, r, hab);
    double v[3] = {st->vx[a] - st->vx[b], st->vy[a] - st->vy[b], st->vz[a] - st->vz[b]};
    double vr = v[0] * d[0] + v[1] * d[1] + v[2] * d[2];
    double Db = st->D[b];
    double pib = st->P[b] / (Db * Db);
    /* artificial viscosity, Monaghan (1992) form, on approaching pairs */
    double Pi = 0.0;
    if (vr < 0.0) {
      double muab = hab * vr / (r2 + p->visc_eps * hab * hab);
      double cbar = 0.5 * (st->cs[a] + st->cs[b]);
      double Dbar = 0.5 * (Da + Db);
      Pi = (-p->visc_alpha * cbar * muab + p->visc_beta * muab * muab) / Dbar;
    }
    const double mb = pmass(p, st, b);
    double cP = mb * (pia + pib + Pi);
    double gn = fabs(g[0]) + fabs(g[1]) + fabs(g[2]);
    for (int i = 0; i < 3; ++i) o.AP[i] += cP * g[i];
    /* kappa: sum of the magnitudes of every elementary product (summation condition bound) */
    o.kP += mb * (fabs(pia) + fabs(pib) + fabs(Pi)) * gn * kc;
    s6_to_m(st->S, n, b, Sb);
    double Da2 = Da * Da, Db2 = Db * Db;
    for (int i = 0; i < 3; ++i) {
      double t = 0.0;
      for (int j = 0; j < 3; ++j) {
        t += (Sa[i][j] / Da2 + Sb[i][j] / Db2) * g[j];
        o.kS += mb * (fabs(Sa[i][j]) / Da2 + fabs(Sb[i][j]) / Db2) * fabs(g[j]) * kc;
      }
      o.AS[i] += mb * t;
    }
    double vg = v[0] * g[0] + v[1] * g[1] + v[2] * g[2];
    double cu = mb * (pia + 0.5 * Pi) * vg;
    o.udot += cu;
    o.dd += mb * vg;                               /* sum m v_ab . grad_a W (continuity rate) */
    o.uvisc += mb * 0.5 * Pi * vg;                 /* viscous heating alone */
    o.kD += mb * (fabs(v[0] * g[0]) + fabs(v[1] * g[1]) + fabs(v[2] * g[2])) * kc;
    {                                              /* v_a . grad P / D_a, pressure terms only */
      double vag = st->vx[a] * g[0] + st->vy[a] * g[1] + st->vz[a] * g[2];
      o.gp += mb * (pia + pib) * vag;
      o.kgp += mb * (fabs(pia) + fabs(pib)) * (fabs(st->vx[a] * g[0]) + fabs(st->vy[a] * g[1]) + fabs(st->vz[a] * g[2])) * kc;
    }
    o.kU += mb * (fabs(pia) + 0.5 * fabs(Pi)) * (fabs(v[0] * g[0]) + fabs(v[1] * g[1]) + fabs(v[2] * g[2])) * kc;
  }
  return o;
}

/* External effective potential of the setup section (g_eff = -grad phi_eff, tabulated as g(r)
 * along the radius from the star centre, linear between entries, 0 beyond the last), harmonic
 * potential walls at wall_in / wall_out and a velocity drag; returns the summed magnitudes of the
 * added terms (for the summation bound). */
static double ext_accel(const orc_params* p, const orc_state* st, int64_t a, double acc[3]) {
  double c[3];
  pcentre(p, st, a, c);
  double X[3] = {st->x[a] - c[0], st->y[a] - c[1], st->z[a] - c[2]};
  double r = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
  double kap = 0.0;
  if (r > 0.0) {
    double g = 0.0;
    double t = p->ext == ORC_EXT_RADIAL ? r / p->ext_dr : 1e300;
    if (t <= (double)(p->ext_n - 1)) {
      int64_t i = (int64_t)floor(t);
      if (i > p->ext_n - 2) i = p->ext_n - 2;
      double f = t - (double)i;
      g = (1.0 - f) * p->ext_g[i] + f * p->ext_g[i + 1];
    }
    if (p->wall_in > 0.0 && r < p->wall_in) g += p->wall_k * (p->wall_in - r);
    if (p->wall_out > 0.0 && r > p->wall_out) g -= p->wall_k * (r - p->wall_out);
    for (int k = 0; k < 3; ++k) acc[k] += g * X[k] / r;
    kap += fabs(g);
  }
  if (p->damping > 0.0) {
    double v[3] = {st->vx[a], st->vy[a], st->vz[a]};
    for (int k = 0; k < 3; ++k) {
      acc[k] -= p->damping * v[k];
      kap += p->damping * fabs(v[k]);
    }
  }
  return kap;
}

int orc_forces(const orc_params* p, orc_state* st, const int64_t* off, const int32_t* ids,
               double* kappa_a, double* kappa_u) {
  int64_t n = st->n;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(max : err)
  for (int64_t a = 0; a < n; ++a) {
    pairsum_t o = pair_sums(p, st, a, ids + off[a], off[a + 1] - off[a]);
    double acc[3], kap;
    double v[3] = {st->vx[a], st->vy[a], st->vz[a]};
    if (p->background == ORC_TOV) {
      /* trajectory equation with zero shift, static isotropic metric gamma_ij = psi^4 delta_ij */
      double c[3];
      pcentre(p, st, a, c);
      metric_t g = metric_at(p, st->x[a] - c[0], st->y[a] - c[1], st->z[a] - c[2]);
      double psi2 = g.psi * g.psi, psi4 = psi2 * psi2, psi6 = psi4 * psi2;
      double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
      double WL = 1.0 / sqrt(1.0 - psi4 * v2 / (g.alpha * g.alpha));
      double hen = 1.0 + st->u[a] + st->P[a] / st->rho[a];
      /* grad P / (W~^2 rho h) with grad P ~= D A^P and W~ = W_L / alpha */
      double fP = g.alpha * g.alpha * psi6 / (WL * hen);
      double nv = g.n[0] * v[0] + g.n[1] * v[1] + g.n[2] * v[2];
      double c0 = 2.0 * g.dalpha / g.alpha * nv;          /* lambda = 0 row: 2 (alpha'/alpha)(n.v) v^i */
      double cg = 4.0 * psi2 * g.psi * g.dpsi;             /* d_k gamma_ij = 4 psi^3 psi' n_k delta_ij */
      double kG = 0.0;
      for (int i = 0; i < 3; ++i) {
        double Gi = g.alpha * g.dalpha * g.n[i] + cg * (nv * v[i] - 0.5 * v2 * g.n[i]);
        acc[i] = -(fP * o.AP[i] + Gi) / psi4 + c0 * v[i] + o.AS[i];
        kG += fabs(Gi) / psi4 + fabs(c0 * v[i]);
      }
      kap = fP * o.kP / psi4 + o.kS + kG;
      kap += ext_accel(p, st, a, acc);
      const double rho = st->rho[a], P = st->P[a], Da = st->D[a];
      if (p->dtP_mode == ORC_DTP_LAGGED && st->dtprev > 0.0 && st->Pprev) {
        /* the lambda = 0 row of the trajectory equation, -xdot^i dP/dt / (W~^2 rho h) with
         * W~ = W_L / alpha, times -g^00 = 1/alpha^2: -xdot^i dP/dt / (W_L^2 rho h); the partial
         * time derivative from the change along the path minus the advection, dP/dt|_x =
         * (P - P_prev) / dt - xdot . grad P with grad P ~ D sum m (P_a/D_a^2 + P_b/D_b^2) grad W */
        double dPdt = (P - st->Pprev[a]) / st->dtprev - Da * o.gp;
        double kt = 1.0 / (WL * WL * rho * hen);
        for (int i = 0; i < 3; ++i) acc[i] -= v[i] * kt * dPdt;
        kap += kt * (fabs(P - st->Pprev[a]) / st->dtprev + Da * o.kgp) * (fabs(v[0]) + fabs(v[1]) + fabs(v[2]));
      }
      if (p->energy_mode == ORC_ENERGY_FIRST_LAW) {
        /* du/dt = (P / rho^2) drho/dt along the path, rho = D / (psi^6 W_L):
         * dln rho/dt = dln D/dt - 6 (psi'/psi) (n.v) - dln W_L/dt, with dln D/dt = dd / D and
         * dln W_L/dt = W_L^2 / 2 d(psi^4 v^2 / alpha^2)/dt along the path */
        double va = v[0] * acc[0] + v[1] * acc[1] + v[2] * acc[2];
        double dq = (4.0 * psi2 * g.psi * g.dpsi * nv * v2 + 2.0 * psi4 * va) / (g.alpha * g.alpha) -
                    2.0 * psi4 * v2 * g.dalpha * nv / (g.alpha * g.alpha * g.alpha);
        double dlnrho = o.dd / Da - 6.0 * g.dpsi / g.psi * nv - 0.5 * WL * WL * dq;
        st->dudt[a] = P / rho * dlnrho + o.uvisc + st->sdot[a];
        if (kappa_u) kappa_u[a] = P / rho * (o.kD / Da + fabs(6.0 * g.dpsi / g.psi * nv) + fabs(0.5 * WL * WL * dq)) +
                                  o.kU + fabs(st->sdot[a]);
      }
    } else {
      for (int i = 0; i < 3; ++i) acc[i] = -o.AP[i] + o.AS[i];   /* eq. solid2 */
      kap = o.kP + o.kS;
      kap += ext_accel(p, st, a, acc);
    }
    st->ax[a] = acc[0];
    st->ay[a] = acc[1];
    st->az[a] = acc[2];
    if (st->dDdt) st->dDdt[a] = o.dd;
    if (p->energy_mode == ORC_ENERGY_FIRST_LAW && p->background == ORC_TOV) {
      /* written above */
    } else if (p->energy_mode == ORC_ENERGY_FIRST_LAW) {
      /* Newtonian: rho = D, so (P / D^2) dD/dt: the pressure term of eq. solid3 */
      st->dudt[a] = st->P[a] / (st->D[a] * st->D[a]) * o.dd + o.uvisc + st->sdot[a];
      if (kappa_u) kappa_u[a] = o.kU + fabs(st->sdot[a]);
    } else {
      st->dudt[a] = o.udot + st->sdot[a];                        /* eq. solid3 */
      if (kappa_u) kappa_u[a] = o.kU + fabs(st->sdot[a]);
    }
    if (kappa_a) kappa_a[a] = kap;
    if (!isfinite(acc[0]) || !isfinite(acc[1]) || !isfinite(acc[2]) || !isfinite(st->dudt[a]))
      err = ORC_E_NONFINITE;
  }
  /* Courant step of this evaluation: cfl min_a h_a / (c_L,a + |v_a|), c_L^2 = c_s^2 + 4 mu / (3 rho) */
  double dmin = INFINITY;
  for (int64_t a = 0; a < n; ++a) {
    double cl = sqrt(st->cs[a] * st->cs[a] + 4.0 * st->mu[a] / (3.0 * st->rho[a]));
    double vm = sqrt(st->vx[a] * st->vx[a] + st->vy[a] * st->vy[a] + st->vz[a] * st->vz[a]);
    double q = st->h[a] / (cl + vm);
    if (q < dmin) dmin = q;
  }
  st->dt_next = (p->cfl > 0.0 ? p->cfl : 0.3) * dmin;
  return err;
}

int orc_pair_forces(const orc_params* p, orc_state* st, double* Fout) {
  int64_t n = st->n;
  if (n > 4096) return ORC_E_ARG;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < n; ++a) {
    for (int64_t b = 0; b < n; ++b) {
      double* F = Fout + 3 * (a * n + b);
      F[0] = F[1] = F[2] = 0.0;
      if (b == a) continue;
      if (!is_neighbour(p, st->x[a], st->y[a], st->z[a], st->h[a], st->x[b], st->y[b], st->z[b], st->h[b]))
        continue;
      int32_t id = (int32_t)b;
      pairsum_t o = pair_sums(p, st, a, &id, 1);
      for (int i = 0; i < 3; ++i) F[i] = pmass(p, st, a) * (-o.AP[i] + o.AS[i]);
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------ */
/* yield, principal stress, breaking                                                     */

void orc_yield(const orc_params* p, int64_t n, double* S, const double* Y0) {
  for (int64_t a = 0; a < n; ++a) {
    double xx = S[a], yy = S[n + a], zz = S[2 * n + a];
    double xy = S[3 * n + a], xz = S[4 * n + a], yz = S[5 * n + a];
    double J = xx * xx + yy * yy + zz * zz + 2.0 * (xy * xy + xz * xz + yz * yz);
    double sv2 = 1.5 * J;                                  /* sigma_v^2 = 3/2 S:S */
    if (!(sv2 > 0.0)) continue;
    double Y = Y0[a];
    double f;
    if (p->yield_mode == ORC_YIELD_RADIAL) f = Y / sqrt(sv2);
    else f = Y * Y / sv2;                                  /* f = min(Y0^2 / sigma_v^2, 1) */
    if (f < 1.0)
      for (int k = 0; k < 6; ++k) S[k * n + a] *= f;
  }
}

/* Largest eigenvalue of a symmetric 3x3 matrix by the trigonometric closed form. */
static double lambda_max(double xx, double yy, double zz, double xy, double xz, double yz) {
  double q = (xx + yy + zz) / 3.0;
  double p1 = xy * xy + xz * xz + yz * yz;
  double p2 = (xx - q) * (xx - q) + (yy - q) * (yy - q) + (zz - q) * (zz - q) + 2.0 * p1;
  if (!(p2 > 0.0)) return q;
  double pp = sqrt(p2 / 6.0);
  double b00 = (xx - q) / pp, b11 = (yy - q) / pp, b22 = (zz - q) / pp;
  double b01 = xy / pp, b02 = xz / pp, b12 = yz / pp;
  double det = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) + b02 * (b01 * b12 - b11 * b02);
  double r = 0.5 * det;
  if (r < -1.0) r = -1.0;
  if (r > 1.0) r = 1.0;
  double phi = acos(r) / 3.0;
  return q + 2.0 * pp * cos(phi);
}

void orc_lambda_max(int64_t n, const double* s6, double* out) {
  for (int64_t a = 0; a < n; ++a) {
    const double* s = s6 + 6 * a;
    out[a] = lambda_max(s[0], s[1], s[2], s[3], s[4], s[5]);
  }
}

/* ------------------------------------------------------------------------------------ */
/* evaluation and time integration                                                       */

int32_t orc_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

int orc_evaluate(const orc_params* p, orc_state* st, int32_t ngb_mode) {
  int64_t n = st->n;
  int64_t* off = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!off) return ORC_E_OOM;
  int64_t cap = n * 128 + 1024;
  int32_t* ids = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
  if (!ids) { free(off); return ORC_E_OOM; }
  int e = orc_neighbours(p, n, st->x, st->y, st->z, st->h, ngb_mode, off, ids, cap);
  if (e == ORC_E_NGB_CAPACITY) {
    free(ids);
    cap = off[n] + 1;
    ids = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    if (!ids) { free(off); return ORC_E_OOM; }
    e = orc_neighbours(p, n, st->x, st->y, st->z, st->h, ngb_mode, off, ids, cap);
  }
  if (!e) e = orc_density(p, st, off, ids);
  if (!e) e = orc_stress_rate(p, st, off, ids, NULL);
  if (!e) e = orc_forces(p, st, off, ids, NULL, NULL);
  free(off);
  free(ids);
  return e;
}

static void wrap_box(const orc_params* p, double* q) {
  if (!p->periodic) return;
  if (*q >= p->box) *q -= p->box;
  else if (*q < 0.0) *q += p->box;
}

/* Breaking by maximum strain: eps = lambda_max(S) / E, E = 9 B mu / (3 B + mu). */
static void apply_breaking(const orc_params* p, orc_state* st) {
  if (p->break_mode == ORC_BREAK_OFF) return;
  int64_t n = st->n;
  for (int64_t a = 0; a < n; ++a) {
    if (st->type[a] != 1 || st->broken[a]) continue;
    double mu = st->mu[a], B = st->B[a];
    if (!(mu > 0.0)) continue;
    double E = 9.0 * B * mu / (3.0 * B + mu);
    double lm = lambda_max(st->S[a], st->S[n + a], st->S[2 * n + a], st->S[3 * n + a],
                           st->S[4 * n + a], st->S[5 * n + a]);
    if (lm / E >= p->eps_break) {
      st->broken[a] = 1;
      /* FLUIDIZE: no deviatoric stress from here on; the stress rate of the last evaluation is
       * dropped with it, so that the next step's half kick does not rebuild a stress */
      if (p->break_mode == ORC_BREAK_FLUIDIZE)
        for (int k = 0; k < 6; ++k) {
          st->S[k * n + a] = 0.0;
          st->dSdt[k * n + a] = 0.0;
        }
    }
  }
}

int orc_step(const orc_params* p, orc_state* st, double dt, int32_t nsteps, int32_t ngb_mode) {
  int64_t n = st->n;
  const int cont = p->density_mode == ORC_DENS_CONTINUITY;
  if (cont && !st->dDdt) return ORC_E_ARG;
  if (p->dtP_mode == ORC_DTP_LAGGED && !st->Pprev) return ORC_E_ARG;
  if (p->damping > 0.0 && dt > 0.0 && p->damping * dt >= 1.0) return ORC_E_ARG;   /* explicit drag */
  double* vh = (double*)malloc((size_t)n * 11 * sizeof(double));
  if (!vh) return ORC_E_OOM;
  double *vxh = vh, *vyh = vh + n, *vzh = vh + 2 * n, *uh = vh + 3 * n, *Sh = vh + 4 * n, *Dh = vh + 10 * n;
  int e = 0;
  for (int32_t step = 0; step < nsteps && !e; ++step) {
    /* fixed dt, or (dt <= 0) the Courant step of the last evaluation */
    const double dts = dt > 0.0 ? dt : st->dt_next;
    for (int64_t a = 0; a < n; ++a) {
      /* kick: half-step velocity, energy and stress with the rates of the last evaluation */
      vxh[a] = st->vx[a] + 0.5 * dts * st->ax[a];
      vyh[a] = st->vy[a] + 0.5 * dts * st->ay[a];
      vzh[a] = st->vz[a] + 0.5 * dts * st->az[a];
      uh[a] = st->u[a] + 0.5 * dts * st->dudt[a];
      for (int k = 0; k < 6; ++k) Sh[k * n + a] = st->S[k * n + a] + 0.5 * dts * st->dSdt[k * n + a];
      if (cont) Dh[a] = st->D[a] + 0.5 * dts * st->dDdt[a];
      /* drift */
      st->x[a] += dts * vxh[a];
      st->y[a] += dts * vyh[a];
      st->z[a] += dts * vzh[a];
      wrap_box(p, &st->x[a]);
      wrap_box(p, &st->y[a]);
      wrap_box(p, &st->z[a]);
      /* predictors for the velocity-dependent evaluation */
      st->vx[a] = vxh[a] + 0.5 * dts * st->ax[a];
      st->vy[a] = vyh[a] + 0.5 * dts * st->ay[a];
      st->vz[a] = vzh[a] + 0.5 * dts * st->az[a];
      st->u[a] = uh[a] + 0.5 * dts * st->dudt[a];
      for (int k = 0; k < 6; ++k) st->S[k * n + a] = Sh[k * n + a] + 0.5 * dts * st->dSdt[k * n + a];
      if (cont) st->D[a] = Dh[a] + 0.5 * dts * st->dDdt[a];
    }
    orc_yield(p, n, st->S, st->Y0);
    if (p->dtP_mode == ORC_DTP_LAGGED) {   /* the pressure of this evaluation's predecessor */
      memcpy(st->Pprev, st->P, (size_t)n * sizeof(double));
      st->dtprev = dts;
    }
    e = orc_evaluate(p, st, ngb_mode);
    if (e) break;
    for (int64_t a = 0; a < n; ++a) {
      st->vx[a] = vxh[a] + 0.5 * dts * st->ax[a];
      st->vy[a] = vyh[a] + 0.5 * dts * st->ay[a];
      st->vz[a] = vzh[a] + 0.5 * dts * st->az[a];
      st->u[a] = uh[a] + 0.5 * dts * st->dudt[a];
      for (int k = 0; k < 6; ++k) st->S[k * n + a] = Sh[k * n + a] + 0.5 * dts * st->dSdt[k * n + a];
      if (cont) st->D[a] = Dh[a] + 0.5 * dts * st->dDdt[a];
    }
    orc_yield(p, n, st->S, st->Y0);
    apply_breaking(p, st);
    if (p->h_mode == ORC_H_ADAPTIVE)
      for (int64_t a = 0; a < n; ++a) st->h[a] = p->eta * cbrt(pmass(p, st, a) / st->D[a]);
  }
  free(vh);
  return e;
}

/* ------------------------------------------------------------------------------------ */
/* EoS surrogate network: forward pass and backpropagation in FP64                       */

#define MH ORC_MLP_H
/* offsets of the parameter blocks in the flat array */
#define OW1 0
#define OB1 (OW1 + MH * 2)
#define OW2 (OB1 + MH)
#define OB2 (OW2 + MH * MH)
#define OW3 (OB2 + MH)
#define OB3 (OW3 + MH * MH)
#define OW4 (OB3 + MH)
#define OB4 (OW4 + 2 * MH)

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double dsilu(double z) {
  double s = 1.0 / (1.0 + exp(-z));
  return s * (1.0 + z * (1.0 - s));
}

/* one sample: pre-activations z1..z3 and the output y */
static void mlp_sample(const double* w, const double* x, double* z1, double* z2, double* z3, double* y) {
  double h1[MH], h2[MH], h3[MH];
  for (int f = 0; f < MH; ++f) {
    z1[f] = w[OW1 + 2 * f] * x[0] + w[OW1 + 2 * f + 1] * x[1] + w[OB1 + f];
    h1[f] = silu(z1[f]);
  }
  for (int f = 0; f < MH; ++f) {
    double a = w[OB2 + f];
    for (int g = 0; g < MH; ++g) a += w[OW2 + MH * f + g] * h1[g];
    z2[f] = a;
    h2[f] = silu(a);
  }
  for (int f = 0; f < MH; ++f) {
    double a = w[OB3 + f];
    for (int g = 0; g < MH; ++g) a += w[OW3 + MH * f + g] * h2[g];
    z3[f] = a;
    h3[f] = silu(a);
  }
  for (int o = 0; o < 2; ++o) {
    double a = w[OB4 + o];
    for (int g = 0; g < MH; ++g) a += w[OW4 + MH * o + g] * h3[g];
    y[o] = a;
  }
}

void orc_mlp_forward(const double* w, int64_t n, const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < n; ++s) {
    double z1[MH], z2[MH], z3[MH];
    mlp_sample(w, x + 2 * s, z1, z2, z3, y + 2 * s);
  }
}

void orc_mlp_features(const double* w, int64_t n, const double* x, double* h) {
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < n; ++s) {
    double z1[MH], z2[MH], z3[MH], y[2];
    mlp_sample(w, x + 2 * s, z1, z2, z3, y);
    for (int f = 0; f < MH; ++f) h[MH * s + f] = silu(z3[f]);
  }
}

double orc_mlp_loss_grad(const double* w, int64_t n, const double* x, const double* t, double* grad) {
  memset(grad, 0, sizeof(double) * ORC_MLP_NPARAM);
  double loss = 0.0;
  const double inv_n = n > 0 ? 1.0 / (double)n : 0.0;
  for (int64_t s = 0; s < n; ++s) {   /* serial: a fixed summation order */
    const double* xs = x + 2 * s;
    double z1[MH], z2[MH], z3[MH], y[2];
    mlp_sample(w, xs, z1, z2, z3, y);
    double dy[2];
    for (int o = 0; o < 2; ++o) {
      const double e = y[o] - t[2 * s + o];
      loss += 0.5 * e * e * inv_n;
      dy[o] = e * inv_n;            /* dL/dy */
    }
    /* output layer */
    double g3[MH];
    for (int f = 0; f < MH; ++f) {
      const double h3 = silu(z3[f]);
      double dh = 0.0;
      for (int o = 0; o < 2; ++o) {
        grad[OW4 + MH * o + f] += dy[o] * h3;
        dh += w[OW4 + MH * o + f] * dy[o];
      }
      g3[f] = dh * dsilu(z3[f]);
    }
    for (int o = 0; o < 2; ++o) grad[OB4 + o] += dy[o];
    /* layer 3 */
    double g2[MH];
    for (int g = 0; g < MH; ++g) {
      double dh = 0.0;
      for (int f = 0; f < MH; ++f) dh += w[OW3 + MH * f + g] * g3[f];
      g2[g] = dh * dsilu(z2[g]);
    }
    for (int f = 0; f < MH; ++f) {
      grad[OB3 + f] += g3[f];
      for (int g = 0; g < MH; ++g) grad[OW3 + MH * f + g] += g3[f] * silu(z2[g]);
    }
    /* layer 2 */
    double g1[MH];
    for (int g = 0; g < MH; ++g) {
      double dh = 0.0;
      for (int f = 0; f < MH; ++f) dh += w[OW2 + MH * f + g] * g2[f];
      g1[g] = dh * dsilu(z1[g]);
    }
    for (int f = 0; f < MH; ++f) {
      grad[OB2 + f] += g2[f];
      for (int g = 0; g < MH; ++g) grad[OW2 + MH * f + g] += g2[f] * silu(z1[g]);
    }
    /* layer 1 */
    for (int f = 0; f < MH; ++f) {
      grad[OB1 + f] += g1[f];
      grad[OW1 + 2 * f] += g1[f] * xs[0];
      grad[OW1 + 2 * f + 1] += g1[f] * xs[1];
    }
  }
  return loss;
}

/* ------------------------------------------------------------------------------------ */
/* modification step after relaxation                                                    */

/* u of each particle from the profile u(r) of the real EoS (table on r_i = i dr, linear, the
 * last entry beyond it), r the distance from the particle's star centre; velocities zeroed. */
void orc_modify_energy(const orc_params* p, orc_state* st, const double* u_of_r, int32_t nr, double dr) {
  for (int64_t a = 0; a < st->n; ++a) {
    double c[3];
    pcentre(p, st, a, c);
    double X[3] = {st->x[a] - c[0], st->y[a] - c[1], st->z[a] - c[2]};
    double r = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    double t = r / dr;
    double u;
    if (t >= (double)(nr - 1)) {
      u = u_of_r[nr - 1];
    } else {
      int64_t i = (int64_t)floor(t);
      double f = t - (double)i;
      u = (1.0 - f) * u_of_r[i] + f * u_of_r[i + 1];
    }
    st->u[a] = u;
    st->vx[a] = st->vy[a] = st->vz[a] = 0.0;
  }
}

/* ------------------------------------------------------------------------------------ */
/* oscillation diagnostics                                                               */

/* Sums of one state for the oscillation analyses of the test sections (radial modes from u,
 * non-radial modes from v_theta in a slab at r = slab_r +- slab_dr, theta = slab_th +- slab_dth
 * described by a linear fit in r and theta; the crust shell's kinetic energy).  Radius, theta
 * and phi are taken about the origin with theta from the +z axis. */
void orc_diagnostics(const orc_params* p, const orc_state* st, const orc_diag_params* dp, orc_diag* out) {
  double ke = 0.0, tor = 0.0, ein = 0.0, ub = 0.0, pvf = 0.0, pff = 0.0;
  int64_t nb = 0, ns = 0;
  double M[3][3] = {{0}}, rhs[3] = {0};
  for (int64_t a = 0; a < st->n; ++a) {
    const double m = pmass(p, st, a);
    const double x = st->x[a], y = st->y[a], z = st->z[a];
    const double vx = st->vx[a], vy = st->vy[a], vz = st->vz[a];
    const double r = sqrt(x * x + y * y + z * z);
    const double rc = sqrt(x * x + y * y);
    ke += 0.5 * m * (vx * vx + vy * vy + vz * vz);
    ein += m * st->u[a];
    if (rc > 0.0) {
      const double vphi = (-y * vx + x * vy) / rc;      /* e_phi = (-sin phi, cos phi, 0) */
      tor += 0.5 * m * vphi * vphi;
      const double f = 3.0 * (rc / r) * (z / r);       /* 3 sin(theta) cos(theta) */
      pvf += m * vphi * f;
      pff += m * f * f;
    }
    if (r >= dp->r_lo && r < dp->r_hi) { ub += st->u[a]; ++nb; }
    if (r > 0.0 && rc > 0.0) {
      const double th = acos(z / r);
      if (fabs(r - dp->slab_r) <= dp->slab_dr && fabs(th - dp->slab_th) <= dp->slab_dth) {
        /* e_theta = (cos th cos phi, cos th sin phi, -sin th) */
        const double ct = z / r, sth = rc / r;
        const double vth = ct * (x * vx + y * vy) / rc - sth * vz;
        const double f[3] = {1.0, r - dp->slab_r, th - dp->slab_th};
        for (int i = 0; i < 3; ++i) {
          for (int j = 0; j < 3; ++j) M[i][j] += f[i] * f[j];
          rhs[i] += f[i] * vth;
        }
        ++ns;
      }
    }
  }
  out->kinetic = ke;
  out->toroidal = tor;
  out->internal = ein;
  out->u_band = nb > 0 ? ub / (double)nb : 0.0;
  out->n_band = nb;
  out->n_slab = ns;
  out->tor_l2 = pff > 0.0 ? pvf / pff : 0.0;
  /* normal equations of the least-squares fit, solved by Cramer's rule */
  double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
               M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
  double c[3] = {0.0, 0.0, 0.0};
  if (ns >= 3 && det != 0.0) {
    for (int k = 0; k < 3; ++k) {
      double A[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = (j == k) ? rhs[i] : M[i][j];
      c[k] = (A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
              A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0])) / det;
    }
  }
  out->slab_c0 = c[0];
  out->slab_cr = c[1];
  out->slab_cth = c[2];
}

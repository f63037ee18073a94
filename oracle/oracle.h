/*
 * CPU FP64 oracle for the SPH particle loop of "Modeling Neutron Star Oscillations in a
 * Fixed General Relativistic Background Including Solid Crust Dynamics" (Tsao et al.).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that the GPU
 * path is checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never calls it and shares no code,
 * header or table with it.
 *
 * Every function takes HOST pointers, runs synchronously, and returns an orc_status.
 * Arrays are structure-of-arrays of length n; the deviatoric stress S and its rate dSdt
 * are 6*n, component-major in the order xx, yy, zz, xy, xz, yz.
 * Per-particle sums over neighbours are taken in increasing neighbour index order, so the
 * oracle is deterministic for any thread count.
 *
 * Parity status of each function is stated next to it; "parity unpinned" marks a reading
 * of the paper with no independent check beyond oracle/GPU consistency.
 */
#ifndef SPH_ORACLE_H
#define SPH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ORC_OK = 0, ORC_E_ARG = 1, ORC_E_OOM = 3, ORC_E_NGB_CAPACITY = 5,
  ORC_E_NONFINITE = 6, ORC_E_EOS_DOMAIN = 7
} orc_status;

enum { ORC_WC2 = 0, ORC_WC4 = 1 };
enum { ORC_H_FIXED = 0, ORC_H_ADAPTIVE = 1 };
enum { ORC_NEWTONIAN = 0, ORC_TOV = 1 };
enum { ORC_EOS_GAMMA = 0, ORC_EOS_TABLE = 1 };
enum { ORC_MU_CONST = 0, ORC_MU_PFACTOR = 1 };
enum { ORC_YIELD_PAPER = 0, ORC_YIELD_RADIAL = 1 };
enum { ORC_Y0_CONST = 0, ORC_Y0_EFACTOR = 1 };
enum { ORC_BREAK_OFF = 0, ORC_BREAK_ONSET = 1, ORC_BREAK_FLUIDIZE = 2 };
enum { ORC_ROT_OBJECTIVE = 0, ORC_ROT_LITERAL = 1 };
enum { ORC_NGB_BRUTE = 0, ORC_NGB_GRID = 1 };
enum { ORC_EXT_NONE = 0, ORC_EXT_RADIAL = 1 };
enum { ORC_DENS_SUMMATION = 0, ORC_DENS_CONTINUITY = 1 };
enum { ORC_ENERGY_PAPER = 0, ORC_ENERGY_FIRST_LAW = 1 };
enum { ORC_DTP_OFF = 0, ORC_DTP_LAGGED = 1 };

typedef struct {
  int32_t kernel, h_mode, background, periodic;
  double eta, box;                 /* periodic box [0, box)^3 */
  double m;                        /* equal particle mass */
  /* background: bg[0..3][bg_n] = alpha, dalpha/drbar, psi, dpsi/drbar on rbar_i = i*bg_dr */
  const double* bg; int32_t bg_n; double bg_dr, bg_M;
  /* artificial viscosity */
  double visc_alpha, visc_beta, visc_eps;
  /* equation of state */
  int32_t eos; double gamma;
  const double* tab_lnP; const double* tab_lncs2;  /* [i_rho * tab_nu + i_u] */
  int32_t tab_nr, tab_nu; double tab_lnr0, tab_dlnr, tab_lnu0, tab_dlnu;
  /* solid */
  int32_t mu_mode; double mu_const, mu_pfactor;
  int32_t yield_mode, y0_mode; double y0_const, y0_over_E;
  int32_t break_mode; double eps_break;
  int32_t rotation;
  /* ensembles: nstars > 0 with star_info[5 * s + k] = (centre x, y, z, particle mass, shear
   * factor) of star s replaces m and mu_pfactor per particle (state field star), and the
   * background is evaluated about each particle's star centre */
  int32_t nstars;
  const double* star_info;
  /* external radial acceleration g(r) n (table ext_g on r_i = i ext_dr, linear, 0 beyond), walls
   * and drag: see orc_forces */
  int32_t ext; int32_t ext_n; const double* ext_g;
  double ext_dr, wall_in, wall_out, wall_k, damping;
  /* method variants: density by continuity (eq. solid1), first-law energy equation, the dP/dt
   * row of the trajectory equation, adaptive time step */
  int32_t density_mode, energy_mode, dtP_mode;
  double cfl;
} orc_params;

typedef struct {
  int64_t n;
  double *x, *y, *z, *vx, *vy, *vz, *u, *h, *S;  /* S: 6n */
  int8_t* type; uint8_t* broken;
  /* outputs of the evaluation stages */
  double *D, *rho, *P, *cs, *mu, *Y0, *B;
  double *ax, *ay, *az, *dudt, *dSdt;            /* dSdt: 6n */
  double *sdot;                                  /* S:epsdot/D (energy source) */
  const int32_t* star;                           /* star of each particle (ensembles), or NULL */
  double *dDdt;                                  /* sum m (v_a - v_b) . grad_a W (continuity rate) */
  double *Pprev;                                 /* P of the previous evaluation (dP/dt term) */
  double dtprev;                                 /* time since that evaluation (0: none) */
  double dt_next;                                /* cfl min h / (c_L + |v|) of the last evaluation */
} orc_state;

/* Neighbour sets N(a) = { b != a : |x_a - x_b|^2 < (h_a + h_b)^2 } (section "Solid SPH
 * Equations": the sum runs over particles within the support radius 2 h_ab = h_a + h_b).
 * Output is CSR: offsets[n+1], ids[offsets[n]] with each list ascending.  cap bounds ids;
 * on overflow returns ORC_E_NGB_CAPACITY and offsets[n] holds the size needed.
 * Pinned by: BRUTE vs GRID equality and symmetry on random inputs; 81/93-neighbour lattice. */
int orc_neighbours(const orc_params* p, int64_t n, const double* x, const double* y,
                   const double* z, const double* h, int32_t mode,
                   int64_t* offsets, int32_t* ids, int64_t cap);

/* Smoothing kernel: W(r, h_ab) and F with grad_a W = F (x_a - x_b).
 * Pinned by: unit normalisation, compact support, finite-difference derivative. */
void orc_kernel(int32_t kernel, double r, double hab, double* W, double* F);

/* Largest eigenvalue of symmetric 3x3 matrices (6 comps each, xx,yy,zz,xy,xz,yz; AoS here).
 * Pinned by: LAPACK eigenvalues on random matrices. */
void orc_lambda_max(int64_t n, const double* s6, double* out);

/* Density D = sum m W, then rho, P, c_s, mu, Y0, B per particle.  Pinned by: lattice density. */
int orc_density(const orc_params* p, orc_state* st, const int64_t* offsets, const int32_t* ids);

/* Velocity gradient, strain/rotation rates and dS/dt (eqs. solid4-solid6); sdot = S:epsdot/D.
 * Pinned by: affine-velocity and rigid-rotation tests. */
int orc_stress_rate(const orc_params* p, orc_state* st, const int64_t* offsets, const int32_t* ids,
                    double* kappa_G /* optional n: sum |m v_ba grad W| */);

/* Pair forces (eqs. solid2, solid3) and the fixed-background trajectory equation.
 * Pinned by: pairwise antisymmetry, power balance, static-lattice zero force;
 * the fixed-background form has "parity unpinned" pieces (see the source). */
int orc_forces(const orc_params* p, orc_state* st, const int64_t* offsets, const int32_t* ids,
               double* kappa_a /* optional n */, double* kappa_u /* optional n */);

/* Pair force matrix for the antisymmetry pin: F[a*n + b] (3 comps, AoS) = the contribution of
 * pair (a,b) to m * (-A^P + A^S) of a, Newtonian.  n <= 4096. */
int orc_pair_forces(const orc_params* p, orc_state* st, double* F);

/* Von Mises yield scaling of S in place with per-particle Y0 (section "Solid SPH Equations"). */
void orc_yield(const orc_params* p, int64_t n, double* S, const double* Y0);

/* nsteps kick-drift-kick steps of size dt.  On entry the rates (ax..dSdt) and the per-particle
 * Y0/B/mu must hold a full evaluation at the current state. */
int orc_step(const orc_params* p, orc_state* st, double dt, int32_t nsteps, int32_t ngb_mode);

/* Modification step after relaxation (section "Setting up Neutron Stars"): u of every particle
 * from the real EoS's profile u(r) (u_of_r on r_i = i dr, linear, the last entry beyond), r the
 * distance from the star centre; velocities set to zero.
 * Pinned by: a linear profile, reproduced exactly at every radius. */
void orc_modify_energy(const orc_params* p, orc_state* st, const double* u_of_r, int32_t nr, double dr);

/* Oscillation diagnostics of one state (sections "Spherically symmetric and static neutron star
 * tests" and "Neutron Star Oscillations with a solid crust"): kinetic energy, its toroidal part
 * about the z axis, total internal energy, the mean u of the radial band [r_lo, r_hi) (radial
 * modes are read from u), and the linear least-squares fit v_theta = c0 + c_r (r - slab_r) +
 * c_th (theta - slab_th) over the slab |r - slab_r| <= slab_dr, |theta - slab_th| <= slab_dth
 * (non-radial modes), and the amplitude of the l = 2 toroidal mode, the projection of v_phi on
 * f(theta) = 3 sin(theta) cos(theta) = -d P_2(cos theta) / d theta (the crust shell's oscillation).
 * About the origin, theta from +z.
 * Pinned by: a linear v_theta field recovered exactly; closed-form kinetic energies. */
typedef struct { double r_lo, r_hi, slab_r, slab_dr, slab_th, slab_dth; } orc_diag_params;
typedef struct {
  double kinetic, toroidal, internal, u_band, slab_c0, slab_cr, slab_cth;
  int64_t n_band, n_slab;
  double tor_l2;   /* l = 2 toroidal mode: sum m v_phi f / sum m f^2, f = 3 sin(theta) cos(theta) */
} orc_diag;
void orc_diagnostics(const orc_params* p, const orc_state* st, const orc_diag_params* dp, orc_diag* out);

/* OpenMP threads of the parallel loops (1 without OpenMP). */
int32_t orc_threads(void);

/* One full evaluation: neighbours, density, stress rate, forces. */
int orc_evaluate(const orc_params* p, orc_state* st, int32_t ngb_mode);

#ifdef __cplusplus
}
#endif
/* ---- EoS surrogate network ------------------------------------------------------------------
 * A multilayer perceptron 2 -> 64 -> 64 -> 64 -> 2 with SiLU activations, silu(z) = z/(1+e^-z),
 * mapping normalised (ln rho, ln u) to normalised (ln P, ln c_s^2).  Parameters are a flat array
 * of ORC_MLP_NPARAM doubles in the order
 *   W1[64][2], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[2][64], b4[2]
 * with W[out][in] row-major.  The training loss over n samples is
 *   L = 1/(2n) sum_s sum_o (y_so - t_so)^2.
 * Parity: pinned by central finite differences of L and by closed-form special cases. */
#define ORC_MLP_H 64
#define ORC_MLP_NPARAM 8642

/* y[2n] = network(x[2n]) (sample-major pairs). */
void orc_mlp_forward(const double* w, int64_t n, const double* x, double* y);

/* h[64n] = the last hidden layer silu(z3) of each sample (sample-major): the inputs of the
 * readout y = W4 h + b4. */
void orc_mlp_features(const double* w, int64_t n, const double* x, double* h);

/* Returns L and writes dL/dw to grad[ORC_MLP_NPARAM] (backpropagation, summed over samples). */
double orc_mlp_loss_grad(const double* w, int64_t n, const double* x, const double* t, double* grad);

#endif

/*
 * sph.h - C ABI of the MI355X (gfx950) SPH particle loop for neutron stars with a solid crust,
 * after Tsao, Sagert, Korobkin, Tews, Lim, Dilts, Loiseau, "Modeling Neutron Star
 * Oscillations in a Fixed General Relativistic Background Including Solid Crust Dynamics"
 * (arXiv:2107.07315).
 *
 * One step of the method is: neighbour search -> density summation (with the equation of
 * state) -> velocity gradient and deviatoric stress rate -> momentum/energy pair forces in the
 * fixed background -> kick-drift-kick integration with von Mises yield and maximum-strain
 * breaking.  Each stage below is one call; sph_step runs whole steps.
 *
 * Conventions
 *  - Units: G = c = Msun = 1 (section "Fixed metric background", conventions).
 *  - Memory: every array pointer in sph_state and the table pointers in sph_params are DEVICE
 *    pointers owned by the caller; the library never frees or reallocates them.  Arrays are
 *    structure-of-arrays of length n; S and dSdt hold 6*n doubles, component-major in the order
 *    xx, yy, zz, xy, xz, yz.  Library scratch (sort buffers, cell tables, neighbour lists,
 *    half-step copies, mixed-precision shadows) is allocated by sph_create for `capacity`
 *    particles and freed by sph_destroy.
 *  - Streams: every call is enqueued on the HIP stream given to sph_create and returns without
 *    waiting, except sph_sync, sph_export_neighbours, the statistics and timing getters, and
 *    (with skin > 0) sph_build_cells and sph_step, which wait for a one-word drift test per
 *    evaluation.
 *  - Errors: argument and call-order errors return immediately with nothing enqueued.  Errors
 *    found on the device (non-finite fields, neighbour-list overflow, states outside the EoS
 *    table) are latched in a device status word with the first offending particle and are
 *    returned by the next sph_sync.
 *  - Order: sph_build_cells -> sph_density -> sph_stress_rate -> sph_forces.  A stage called
 *    before its predecessor for the current positions returns SPH_E_ORDER.
 *  - Reordering: sph_build_cells (and sph_step, whenever it rebuilds the lists) permutes every
 *    particle array of the state in place into the order it uses (id follows the particles);
 *    results are reported in that order.
 *  - Threads: one host thread per context.
 */
#ifndef SPH_H
#define SPH_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sph_ctx sph_ctx;

typedef enum {
  SPH_OK = 0,
  SPH_E_ARG = 1,           /* invalid argument (null pointer, size, mode)                  */
  SPH_E_HIP = 2,           /* HIP runtime error                                             */
  SPH_E_OOM = 3,           /* device allocation failed                                      */
  SPH_E_ORDER = 4,         /* stage called out of order                                     */
  SPH_E_NGB_CAPACITY = 5,  /* a neighbour list exceeded max_neighbours                      */
  SPH_E_NONFINITE = 6,     /* a field became NaN/Inf                                        */
  SPH_E_EOS_DOMAIN = 7     /* (rho, u) outside the tabulated equation of state              */
} sph_status;

enum { SPH_WC2 = 0, SPH_WC4 = 1 };                         /* Wendland kernels, support 2h  */
enum { SPH_H_FIXED = 0, SPH_H_ADAPTIVE = 1 };
enum { SPH_NEWTONIAN = 0, SPH_TOV = 1 };
enum { SPH_EOS_GAMMA = 0, SPH_EOS_TABLE = 1, SPH_EOS_MLP = 2 };
enum { SPH_MU_CONST = 0, SPH_MU_PFACTOR = 1 };
enum { SPH_YIELD_PAPER = 0, SPH_YIELD_RADIAL = 1 };
enum { SPH_Y0_CONST = 0, SPH_Y0_EFACTOR = 1 };
enum { SPH_BREAK_OFF = 0, SPH_BREAK_ONSET = 1, SPH_BREAK_FLUIDIZE = 2 };
enum { SPH_ROT_OBJECTIVE = 0, SPH_ROT_LITERAL = 1 };
enum { SPH_FP64 = 0, SPH_FP32 = 1 };
enum { SPH_EXT_NONE = 0, SPH_EXT_RADIAL = 1 };
enum { SPH_DENS_SUMMATION = 0, SPH_DENS_CONTINUITY = 1 };
enum { SPH_ENERGY_PAPER = 0, SPH_ENERGY_FIRST_LAW = 1 };
enum { SPH_DTP_OFF = 0, SPH_DTP_LAGGED = 1 };

/* Particle state (section "Solid SPH Equations": per-particle position, velocity, internal
 * energy, deviatoric stress; equal mass per particle, section "Fixed metric background").
 * x,y,z: coordinate positions (isotropic coordinates with the TOV background).
 * vx,vy,vz: coordinate velocity dx/dt.  u: specific internal energy.  h: smoothing length.
 * S: deviatoric stress (6 comps).  type: 0 fluid core, 1 solid crust; a fluid particle carries no
 * deviatoric stress: every candidate-list build (sph_build_cells, and sph_step when particles
 * have moved past the skin) sets S and dSdt of type-0 particles to 0.  broken: 1 once the
 * maximum-strain criterion fired.  id: caller's particle id, permuted with the particles.
 * star: optional (may be NULL) index into the ensemble table of sph_ensemble_set.
 * Outputs: D computational density, rho rest-mass density, P pressure, cs sound speed,
 * ax..az coordinate acceleration, dudt, dSdt. */
typedef struct {
  int64_t n;
  double *x, *y, *z, *vx, *vy, *vz, *u, *h, *S;
  int8_t* type;
  uint8_t* broken;
  int32_t* id;
  int32_t* star;
  double *D, *rho, *P, *cs, *ax, *ay, *az, *dudt, *dSdt;
} sph_state;

/* Method parameters.  Where the paper leaves a choice open, the field selects it; the defaults
 * used throughout are noted. */
typedef struct {
  int32_t kernel;          /* SPH_WC2 | SPH_WC4                                               */
  int32_t h_mode;          /* FIXED, or ADAPTIVE: h = eta (m/D)^(1/3) after each step         */
  int32_t background;      /* NEWTONIAN, or TOV: static isotropic metric from bg table        */
  int32_t periodic;        /* periodic cube [0, box)^3 with minimum-image pairs               */
  double eta, box, m;      /* m: particle mass (equal baryon mass per particle)               */
  const double* bg;        /* device: 4*bg_n doubles alpha, dalpha/drbar, psi, dpsi/drbar    */
  int32_t bg_n;            /*   on rbar_i = i*bg_dr; exterior Schwarzschild with mass bg_M    */
  double bg_dr, bg_M;
  double visc_alpha, visc_beta, visc_eps;   /* Monaghan viscosity (default 1, 2, 0.01)        */
  int32_t eos;             /* GAMMA: P=(gamma-1) rho u; TABLE: bilinear ln P, ln cs^2;         */
  double gamma;            /*   MLP: surrogate with table fallback (sph_mlp_*)                */
  const double* tab_lnP;   /* device: [i_rho * tab_nu + i_u]; NULL: the table of               */
                           /*   sph_eos_table_create (stage calls return SPH_E_ARG without one) */
  const double* tab_lncs2;
  int32_t tab_nr, tab_nu;
  double tab_lnr0, tab_dlnr, tab_lnu0, tab_dlnu;
  int32_t mu_mode;         /* shear modulus of crust particles: CONST mu_const or mu_pfactor*P */
  double mu_const, mu_pfactor;
  int32_t yield_mode;      /* PAPER f = min(Y0^2/sigma_v^2, 1) (default) or RADIAL Y0/sigma_v  */
  int32_t y0_mode;         /* CONST y0_const, or EFACTOR y0_over_E * E                         */
  double y0_const, y0_over_E;
  int32_t break_mode;      /* OFF, ONSET (flag only), FLUIDIZE (flag, then S = 0 and mu = 0)   */
  double eps_break;        /* breaking strain                                                  */
  int32_t rotation;        /* OBJECTIVE R S - S R (default) or LITERAL S R - R S               */
  int32_t precision;       /* FP64, or FP32 pair sums with FP64 positions/integration/metric  */
  int32_t max_neighbours;  /* exact-list capacity per particle (0: 512); candidate lists hold  */
                           /*   twice as many                                                  */
  int32_t cell_div;        /* cells per smoothing diameter of the finest level (0: 1)          */
  double tile_cut;         /* a 64-particle tile is cut where the Morton curve jumps farther  */
                           /*   than tile_cut smoothing lengths (0: 10)                        */
  double skin;             /* relative Verlet skin s: candidate lists hold every b with       */
                           /*   |x_a - x_b| < (1 + s)(h_a + h_b) and are rebuilt only when a    */
                           /*   particle has moved, plus grown in h, by more than s h since the */
                           /*   last build.  0: rebuild at every evaluation.  Values in (0,     */
                           /*   1e-4) act as 0; periodic runs clip s so that (1+s)(h_a+h_b)     */
                           /*   stays below half the box.                                       */
  int32_t pass_blocks;     /* workgroups of the pair passes: 0 = one per tile (at most 65536),  */
                           /*   else a persistent grid of that many (rounded up to 8) that     */
                           /*   loops over the tiles                                            */
  int32_t graph;           /* sph_step: 1 = replay captured HIP graphs of each step's kernels  */
                           /*   (needs skin > 0; stage timers are not recorded)                */
  int32_t lanes;           /* lanes per target particle in the pair passes: 1, 2 or 4 (0: 4);  */
                           /*   a tile of up to 64 targets is one workgroup of 64 * lanes     */
                           /*   threads, the lanes of a target splitting its list             */
  /* External effective potential and potential walls (section "Setting up Neutron Stars":
   * relaxation in phi_eff with g_eff = -grad phi_eff, confined by walls; section "Neutron stars
   * with a solid crust in SPH": a crust shell held by phi_eff and walls).  With ext =
   * SPH_EXT_RADIAL the force pass adds g(r) n, r the distance from the star centre (the
   * isotropic radius with the TOV background), n = x / r, g linear in ext_g[i] on r_i = i ext_dr
   * (ext_g: device, ext_n entries, positive outward; 0 beyond the last entry), plus the walls
   * wall_k (wall_in - r) n where r < wall_in and -wall_k (r - wall_out) n where r > wall_out (a
   * wall radius of 0 means no wall), plus -damping v (a relaxation drag; 0: none).  Walls and
   * drag also act with ext = SPH_EXT_NONE (e.g. settling a star in the fixed background). */
  int32_t ext;             /* SPH_EXT_NONE | SPH_EXT_RADIAL                                    */
  int32_t ext_n;
  const double* ext_g;
  double ext_dr, wall_in, wall_out, wall_k, damping;
  /* Method variants (defaults: the paper's equations as read above). */
  int32_t density_mode;    /* SUMMATION: D = sum m W; CONTINUITY (eq. solid1): D is state,    */
                           /*   integrated with dD/dt = sum_b m (v_a - v_b) . grad_a W         */
  int32_t energy_mode;     /* PAPER: eq. solid3 with D; FIRST_LAW: du/dt = (P/rho^2) drho/dt  */
                           /*   along the trajectory (rho = D / (psi^6 W_L)), plus the viscous   */
                           /*   heating and stress work of eq. solid3                           */
  int32_t dtP_mode;        /* OFF: the dP/dt entry (lambda = 0 row) of the trajectory equation  */
                           /*   dropped; LAGGED: with dP/dt = (P - P_prev)/dt_prev - v . grad P  */
  int32_t reserved;
  double cfl;              /* sph_step with dt <= 0: each step's dt = cfl min_a h_a /           */
                           /*   (c_L,a + |v_a|), c_L^2 = c_s^2 + 4 mu / (3 rho), from the last    */
                           /*   evaluation, on the device (0: 0.3)                              */
} sph_params;

/* Neighbour-list statistics (sph_neighbour_stats). */
typedef struct {
  int64_t pairs;           /* exact list entries (ordered pairs a->b, b != a) of the last density */
  int32_t max_count;       /* longest exact list                                               */
  int32_t pad;
  int64_t tiles;           /* tiles (at most 64 particles sharing one neighbour union)          */
  int64_t union_total;     /* summed tile-union sizes                                          */
  int64_t candidates;      /* summed candidate-list lengths (exact lists plus the skin)        */
  int64_t rebuilds;        /* candidate-list builds since sph_create                           */
} sph_list_stats;

/* Create a context for up to `capacity` particles on the current HIP device (capacity rounded up
 * to 64 times twice max_neighbours must stay below 2^32); all work is
 * enqueued on `hip_stream` (a hipStream_t, may be NULL for the default stream).
 * Returns SPH_E_ARG for a bad parameter set, SPH_E_OOM if scratch does not fit. */
sph_status sph_create(const sph_params* params, void* hip_stream, int64_t capacity, sph_ctx** out);
void sph_destroy(sph_ctx* ctx);

/* Replace the parameters (same capacity).  Invalidates the stage order. */
sph_status sph_set_params(sph_ctx* ctx, const sph_params* params);

/* Neighbour search set-up (the summation runs over particles within the support radius,
 * section "Solid SPH Equations").  If the candidate lists are stale (first call, new n or
 * parameters, skin 0, or a particle moved or grew past the skin bound since the last build):
 * permute all state arrays along a global Morton curve, sort particles into a multi-level cell
 * grid (levels by h) and build candidate lists { b != a : |x_a - x_b| < (1 + skin)(h_a + h_b) }
 * per tile of at most 64 consecutive particles.  The exact sets
 * N(a) = { b != a : |x_a - x_b|^2 < (h_a + h_b)^2 }, evaluated in FP64 without contraction,
 * are extracted from the candidates by sph_density.  With skin > 0 this call waits for the
 * one-word drift test on the device before deciding. */
sph_status sph_build_cells(sph_ctx* ctx, sph_state* st);

/* Density summation D_a = sum_b m W(r_ab, h_ab) including b = a (section "Fixed metric
 * background": the computational density D = rho sqrt(gamma) W_L recovered by the standard
 * SPH sum), then rho = D / (psi^6 W_L), P and c_s from the EoS (eq. poly_eos family; the
 * relativistic sound speed of the setup section), the crust shear modulus and yield stress.
 * Also extracts the exact neighbour lists the later stages use.  Writes D, rho, P, cs. */
sph_status sph_density(sph_ctx* ctx, sph_state* st);

/* Velocity gradient and stress rate (eqs. solid4-solid6): strain and rotation rates from
 * G^ij = sum_b m (v_b - v_a)^i d_j W_ab, dS/dt = 2 mu (epsdot - tr/3) + rotation terms, and
 * the stress work S:epsdot/D for the energy equation.  Crust particles only; dSdt = 0 elsewhere. */
sph_status sph_stress_rate(sph_ctx* ctx, sph_state* st);

/* Pair forces (eqs. solid2, solid3) with artificial viscosity, and in TOV mode the fluid
 * trajectory equation of the fixed-background section with zero shift.  Writes ax..az, dudt. */
sph_status sph_forces(sph_ctx* ctx, sph_state* st);

/* nsteps kick-drift-kick steps of size dt; dt <= 0: each step takes the Courant step
 * cfl min_a h_a / (c_L,a + |v_a|) of the evaluation before it, computed on the device (the host
 * never waits for it; sph_get_time reports the simulated time; not with graph replay).  With
 * damping > 0 a fixed dt needs damping dt < 1.  On entry the rates must be those of a full
 * evaluation at the current state (build_cells, density, stress_rate, forces).  Applies the
 * von Mises yield scaling after each stress update and the maximum-strain breaking test
 * (section "Solid SPH Equations"), and the adaptive smoothing length.  Within one call the final
 * kick of a step and the kick-drift of the next run as one kernel, so the state between two steps
 * of the call is never written out; on return the state is the end of the last step and the
 * rates are those of its evaluation, except that a particle broken (FLUIDIZE) in the last step has
 * its stress and stress rate set to zero. */
sph_status sph_step(sph_ctx* ctx, sph_state* st, double dt, int32_t nsteps);

/* Modification step after relaxation (section "Setting up Neutron Stars": once the star is relaxed
 * to the desired density profile, u is assigned from the profile and the real EoS, after which the
 * star is evolved).  Sets u of every particle to the profile u(r) of the real EoS, u_of_r (device,
 * nr >= 2 entries on r_i = i dr, linear between entries, the last entry beyond it), r the distance
 * from the particle's star centre (isotropic radius with the TOV background), and zeroes the
 * velocities.  Positions and lists are kept; the next stage call must be sph_density (or
 * sph_build_cells).  Stream-ordered. */
sph_status sph_modify_energy(sph_ctx* ctx, sph_state* st, const double* u_of_r, int32_t nr, double dr);

/* Oscillation diagnostics of the current state (section "Spherically symmetric and static neutron
 * star tests": radial modes are read from the internal energy, non-radial ones from v_theta of the
 * particles in a slab r = slab_r +- slab_dr, theta = slab_th +- slab_dth, described by a linear
 * fit in r and theta; section "Neutron Star Oscillations with a solid crust": the kinetic energy
 * of the toroidally oscillating crust).  r, theta (from +z) and phi are taken about the origin,
 * with coordinate velocities.  `out` is a DEVICE pointer to one sph_diag: calls are
 * stream-ordered, so a time series can be recorded between sph_step calls without waiting. */
typedef struct {
  double r_lo, r_hi;        /* radial band of the mean u: r_lo <= r < r_hi                     */
  double slab_r, slab_dr;   /* v_theta slab in radius ...                                      */
  double slab_th, slab_dth; /*   ... and in theta (radians)                                     */
} sph_diag_params;
typedef struct {
  double kinetic;           /* sum m |v|^2 / 2                                                 */
  double toroidal;          /* sum m (v . e_phi)^2 / 2                                         */
  double internal;          /* sum m u                                                          */
  double u_band;            /* mean u over the radial band                                     */
  double slab_c0, slab_cr, slab_cth;  /* least squares v_theta = c0 + c_r (r - slab_r) +          */
                                      /*   c_th (theta - slab_th) over the slab (0 if < 3 there) */
  int64_t n_band, n_slab;   /* particles in the band and in the slab                           */
  double tor_l2;            /* l = 2 toroidal mode amplitude: sum m v_phi f / sum m f^2 with     */
                            /*   f = 3 sin(theta) cos(theta) = -d P_2(cos theta) / d theta       */
} sph_diag;
sph_status sph_diagnostics(sph_ctx* ctx, const sph_state* st, const sph_diag_params* params, sph_diag* out);

/* Ensembles of independent stars in one particle set: star_info (host) holds nstars rows of
 * (centre x, y, z, particle mass, shear factor); each particle's star (state field `star`,
 * required while an ensemble is set) selects its mass, its crust shear factor (mu = factor * P)
 * and the centre about which the fixed background is evaluated.  Pair sums take the particle's
 * own star mass, so stars must lie farther apart than any particle's support (no pair crosses
 * stars).  nstars = 0 returns to a single star.  Waits; invalidates the stage order. */
sph_status sph_ensemble_set(sph_ctx* ctx, int32_t nstars, const double* star_info);

/* Launch autotuner: under candidate settings of lanes, pass_blocks, tile_cut and skin, one parameter
 * at a time (coordinate descent from the current settings), times one sph_step call of
 * `steps_per_trial` steps (with the candidate-list rebuilds they need) on a copy of the state (the
 * caller's state is not changed), and keeps the setting with the least time per step; a setting
 * replaces the best only if it is more than 2% faster.  Use enough steps for several rebuilds
 * (64 or more at the default skin).  The context then needs a new evaluation (sph_build_cells ...) before
 * sph_step.  Waits. */
typedef struct {
  int32_t pass_blocks;
  int32_t trials;          /* configurations timed                                              */
  int32_t lanes;
  int32_t pad;
  double tile_cut, skin;
  double ms_per_step;      /* of the chosen configuration, rebuilds amortised                   */
  double ms_per_step_start;/* of the starting configuration                                     */
} sph_tune_result;
sph_status sph_autotune(sph_ctx* ctx, const sph_state* st, double dt, int32_t steps_per_trial,
                        sph_tune_result* out);

/* Simulated time: the sum of the steps' dt since sph_create.  Waits. */
sph_status sph_get_time(sph_ctx* ctx, double* t);

/* Wait for the context's stream; return and clear the first latched device error. */
sph_status sph_sync(sph_ctx* ctx);

/* Array index (in the state's current order, i.e. after the last sph_build_cells reordering)
 * of the particle that raised the error returned by the last failing sph_sync, or -1 when the
 * error has no particle (a tile-level overflow) or no sph_sync has failed.  Does not wait. */
int32_t sph_error_particle(const sph_ctx* ctx);

/* Copy the exact neighbour lists of the last sph_density to host memory as CSR in the
 * particles' current order: offsets[n+1] (host), ids[offsets[n]] (host, indices into the
 * current order).  Lists are written unsorted.  Returns SPH_E_ORDER before the first density
 * evaluation, SPH_E_NGB_CAPACITY (and offsets) if cap is too small.  Waits. */
sph_status sph_export_neighbours(sph_ctx* ctx, int64_t* offsets, int32_t* ids, int64_t cap);

/* Statistics of the current lists (see sph_list_stats).  Waits. */
sph_status sph_neighbour_stats(sph_ctx* ctx, sph_list_stats* out);

/* The same statistics for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): no allocation at all.  The
 * counters live in a fixed 64-byte array in the library's device memory, one copy per GPU, held
 * until the process ends and looked up by sph_create; any list size a context holds fits it (the
 * counters are 64-bit).  Every call on a GPU shares that copy and clears it first, so calls that
 * overlap on one GPU (two host threads, or two contexts on different streams) race; calls in
 * sequence do not.  Same result as sph_neighbour_stats.  Waits. */
sph_status sph_neighbour_stats_noalloc(sph_ctx* ctx, sph_list_stats* out);

/* ---- EoS surrogate network (extension of the tabulated EoS) ---------------------------------
 * The setup section names tabulated equations of state; this extension fits a network
 * 2 -> 64 -> 64 -> 64 -> 2 with SiLU activations to the context's EoS table, mapping normalised
 * (ln rho, ln u) to normalised (ln P, ln c_s^2).  The two 64x64 layers run on the matrix cores
 * with BF16 weights (rounded from FP32 master weights) and FP32 accumulation, their input
 * activations carried as two BF16 parts (hi + lo); the input layer, the readout and the biases
 * are FP32.  Training runs Adam on the master weights with a cosine learning-rate schedule, on
 * the GPU, and the readout can then be fitted by least squares (sph_mlp_fit_readout).  With
 * eos = SPH_EOS_MLP the density pass uses the network in every table cell the trust mask accepts
 * and table interpolation elsewhere (and everywhere while no network is loaded).
 * Parameters are SPH_MLP_NPARAM floats: W1[64][2], b1[64], W2[64][64], b2[64], W3[64][64],
 * b3[64], W4[2][64], b4[2] (W[out][in], row-major).  Inputs are normalised to [-1, 1] over the
 * network's domain (the table's box unless sph_mlp_set_domain narrows it), outputs by the value
 * range of the table nodes that cover it (sph_mlp_get_norm).  Every call needs the EoS table in
 * the context's parameters and waits for the stream. */
#define SPH_MLP_NPARAM 8642

/* Load FP32 master weights (host array); resets the optimiser and drops the trust mask. */
sph_status sph_mlp_set_params(sph_ctx* ctx, const float* params);

/* Load a network from its BF16 weights (host array of SPH_MLP_NPARAM 16-bit patterns, the upper
 * halves of IEEE FP32 values, in the parameter order above), e.g. weights trained elsewhere:
 * the FP32 masters become exactly these values (so the kernels use them unchanged); resets the
 * optimiser and drops the trust mask.  SPH_E_ARG without an EoS table.  Waits. */
sph_status sph_mlp_load(sph_ctx* ctx, const uint16_t* bf16_weights);

/* Network domain: the box [lnrho_lo, lnrho_hi] x [lnu_lo, lnu_hi] inside the table's box where
 * the network is trained and may serve (the trust mask tests only the table cells inside it).
 * It sets the normalisation, so call it before sph_mlp_set_params / sph_mlp_load and training;
 * drops the trust mask.  SPH_E_ARG for an empty box or one that leaves the table.  Waits. */
sph_status sph_mlp_set_domain(sph_ctx* ctx, double lnrho_lo, double lnrho_hi, double lnu_lo, double lnu_hi);

/* Copy the weights to the host: the FP32 masters, or (rounded != 0) the values the kernels use
 * (W2, W3 rounded to BF16, the rest FP32), as floats.  SPH_E_ARG before sph_mlp_set_params. */
sph_status sph_mlp_get_params(sph_ctx* ctx, float* params, int32_t rounded);

/* Normalisation {in_lo[2], in_scale[2], out_centre[2], out_scale[2]}: x = (v - lo) scale - 1,
 * v = y scale + centre. */
sph_status sph_mlp_get_norm(sph_ctx* ctx, float* norm8);

/* Train on samples[n][2] = (ln rho, ln u) (device, FP64) with table-interpolated targets; the
 * last n_holdout samples are held out.  epochs passes of (n - n_holdout) / batch Adam steps,
 * batch a multiple of 64 and at most 8192, peak learning rate lr.  history (host, may be NULL)
 * receives per epoch {last training-batch loss, holdout loss} (normalised units, loss =
 * 1/(2n) sum of squared output errors).  Drops the trust mask. */
sph_status sph_mlp_train(sph_ctx* ctx, const double* samples, int64_t n, int64_t n_holdout, int32_t epochs,
                         int32_t batch, float lr, float* history);

/* Least-squares readout: with the hidden layers as they are, set W4, b4 to the minimiser of the
 * squared output error over the first n - n_holdout of samples[n][2] (device, FP64, with
 * table-interpolated targets as in sph_mlp_train), from the normal equations with ridge * (mean
 * diagonal) added to the diagonal, solved by Cholesky in FP64 on the device.  holdout_loss (host,
 * may be NULL) receives the loss over the last n_holdout samples afterwards.  Drops the trust
 * mask.  SPH_E_ARG for fewer than 64 fit samples or a negative ridge. */
sph_status sph_mlp_fit_readout(sph_ctx* ctx, const double* samples, int64_t n, int64_t n_holdout, double ridge,
                               double* holdout_loss);

/* Gradient of the loss over x[n][2], t[n][2] (device, normalised FP32; n a multiple of 64, at
 * most 8192) with the current BF16 weights, summed in a fixed order: grad[SPH_MLP_NPARAM] and
 * loss on the host.  Changes no weight. */
sph_status sph_mlp_grad(sph_ctx* ctx, const float* x, const float* t, int64_t n, float* grad, double* loss);

/* Network outputs ln P, ln c_s^2 at device arrays (ln rho, ln u), n entries; stream-ordered. */
sph_status sph_mlp_eval(sph_ctx* ctx, const double* lnrho, const double* lnu, int64_t n, double* lnP,
                        double* lncs2);

/* Build the trust mask: a table cell inside the network's domain is trusted when the network's P
 * and c_s^2 are within relative tolerance tol / 2 of the table at 13 points of the cell (its
 * nodes, edge midpoints, centre and four interior points drawn per cell from a counter-based
 * generator); the margin of 2 covers the points in between.  Returns the number of trusted cells
 * of (nr - 1)(nu - 1). */
sph_status sph_mlp_build_trust_mask(sph_ctx* ctx, double tol, int64_t* trusted_cells);

/* Number of particles of the state whose (rho, u) lies in a trusted cell, i.e. that the network
 * serves in an evaluation with eos = SPH_EOS_MLP (0 without a mask).  Waits. */
sph_status sph_mlp_count_served(sph_ctx* ctx, const sph_state* st, int64_t* served);

/* Human-readable name of a status code (static string). */
const char* sph_status_string(sph_status s);

/* Why the last failing call on this context failed: the status name followed by the argument
 * or condition at fault (which array is NULL, which parameter is out of range, which stage has
 * to come first), or, for a device error returned by sph_sync, the particle that latched it and
 * what the code means.  With ctx NULL: the last failure of a call made without a context
 * (sph_create) on this host thread.  The string belongs to the context (or the thread) and stays
 * valid until its next failing call. */
const char* sph_last_error_detail(const sph_ctx* ctx);

/* Tabulated equation of state (section "Setting up Neutron Stars": tabulated EoS, here a table of
 * ln P and ln c_s^2 on a uniform grid in (ln rho, ln u), interpolated bilinearly): copies the host
 * arrays lnP[nr * nu], lncs2[nr * nu] (index i_rho * nu + i_u; NaN marks states outside the
 * EoS's domain) into device memory the context owns, and points the context's table parameters at
 * it; a later sph_set_params whose table pointers are NULL keeps using it.  Grid: ln rho_i =
 * lnr0 + i dlnr, ln u_j = lnu0 + j dlnu.  A network loaded for the previous table is dropped.
 * SPH_E_ARG for NULL arrays, nr or nu < 2 or non-positive spacing; SPH_E_OOM if the copy does not
 * fit.  Invalidates the stage order.  Waits. */
sph_status sph_eos_table_create(sph_ctx* ctx, const double* lnP, const double* lncs2, int32_t nr, int32_t nu,
                                double lnr0, double dlnr, double lnu0, double dlnu);

/* Kernel timing since timing was last enabled: launches and total milliseconds of one stage,
 * measured with HIP events on the context stream (0 while timing is off).  Stages: "cells"
 * (candidate-list builds), "density" (pair loop of the density pass), "eos" (its per-particle
 * epilogue: EoS, moduli, packed records), "stress", "forces", "kdk" (kick-drift and final kick).
 * Graph-replayed steps record no times.  Waits. */
sph_status sph_set_timing(sph_ctx* ctx, int32_t enable);
sph_status sph_get_timing(sph_ctx* ctx, const char* stage, int32_t* launches, double* ms);

#ifdef __cplusplus
}
#endif
#endif

/*
 * ccake.h -- C ABI of the MI355X (gfx950) implementation of one Runge-Kutta
 * stage of the relativistic viscous SPH of CCAKE 2.0 (arXiv 2511.22852).
 *
 * The calls follow the paper's problem statement: an equation of state
 * ("Equation of state", "EoS inverter"), a particle system carrying the
 * dynamical variables {r, u, s/sigma, Pi/sigma, pi/sigma, n_q/sigma}
 * ("Equations of motion", SPH subsection), the conservation laws with
 * minimal Israel-Stewart relaxation (eq. conservation_source, eq. min_bul_rel,
 * eq. min_she_rel) and a time step.
 *
 * Conventions
 *   - Every call returns a ccake_status; 0 is success.  On failure the handle
 *     keeps a message readable with ccake_last_error(handle).
 *   - Units: hbar = c = 1; lengths and times in fm; T, mu in fm^-1; densities
 *     in fm^-3; energy density and pressure in fm^-4.
 *   - Arrays are FP64 structure-of-arrays, row-major [row][n], in the caller's
 *     particle order (index 0..n-1) unless stated otherwise.
 *   - mem = CCAKE_HOST: host pointers (copied synchronously);
 *     mem = CCAKE_DEVICE: device pointers valid on the library's device; the
 *     copy is enqueued on the handle's stream and the pointer must stay valid
 *     until the stream reaches it.
 *   - The state layout (26 rows, CCAKE_ROW_*) is the exchange format of
 *     ccake_set_state / ccake_get_state (checkpoint / restore).
 *   - Handles are not thread-safe; one simulation per stream.
 */
#ifndef CCAKE_H
#define CCAKE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ccake_status;
enum {
  CCAKE_OK = 0,
  CCAKE_E_ARG = 1,         /* invalid argument (sizes, non-finite or negative input) */
  CCAKE_E_HIP = 2,         /* HIP runtime error (message in ccake_last_error) */
  CCAKE_E_NONFINITE = 3,   /* a particle update produced a non-finite value (sticky) */
  CCAKE_E_EOS_NOCONV = 4,  /* an EoS inversion did not converge, backup included (sticky) */
  CCAKE_E_CAPACITY = 5,    /* workspace, cell grid or server capacity exceeded */
  CCAKE_E_STATE = 6,       /* call out of sequence (e.g. step before init) */
  CCAKE_E_NOMEM = 7        /* device allocation failed */
};

enum { CCAKE_HOST = 0, CCAKE_DEVICE = 1 };
enum { CCAKE_CARTESIAN = 0, CCAKE_HYPERBOLIC = 1 };
enum { CCAKE_FP64 = 0, CCAKE_MIXED = 1 };
/* density_mode: how the rest-frame s and n_q of a particle are formed
 *   SMOOTHED: s_a = sum_b S_b W_ab / (gamma_a sqrt(-g))  (SPH interpolation of
 *             the lab-frame density, "SPH interpretation of a fluid element")
 *   SPECIFIC: s_a = S_a sigma_a with sigma_a = sigma*_a / (gamma_a sqrt(-g))
 *             (the particle's own s/sigma, "Equations of motion") */
enum { CCAKE_DENS_SMOOTHED = 0, CCAKE_DENS_SPECIFIC = 1 };
/* dens_kind of ccake_init_particles */
enum { CCAKE_INIT_S = 0, CCAKE_INIT_E = 1 };

/* rows of the state exchange format: x^k, u^k, S = s/sigma, N_q = n_q/sigma,
 * B = Pi/sigma, P^{ij} = pi^{ij}/sigma, and J^k_q/sigma (the charge diffusion
 * currents, contravariant spatial components; zero without diffusion) */
enum {
  CCAKE_ROW_X1 = 0, CCAKE_ROW_X2, CCAKE_ROW_X3, CCAKE_ROW_U1, CCAKE_ROW_U2, CCAKE_ROW_U3,
  CCAKE_ROW_S, CCAKE_ROW_NB, CCAKE_ROW_NS, CCAKE_ROW_NQ, CCAKE_ROW_B,
  CCAKE_ROW_P11, CCAKE_ROW_P12, CCAKE_ROW_P13, CCAKE_ROW_P22, CCAKE_ROW_P23, CCAKE_ROW_P33,
  CCAKE_ROW_JB1, CCAKE_ROW_JB2, CCAKE_ROW_JB3, CCAKE_ROW_JS1, CCAKE_ROW_JS2, CCAKE_ROW_JS3,
  CCAKE_ROW_JQ1, CCAKE_ROW_JQ2, CCAKE_ROW_JQ3,
  CCAKE_NROW
};

/* per-particle diagnostics of one right-hand-side evaluation (ccake_rhs, ccake_read);
 * NEWTON is the number of Newton iterations of the particle's EoS inversion and
 * EOS_EVALS the number of residual evaluations (step halvings included).  The
 * Knudsen and inverse Reynolds numbers ("Particlization", eq. knudsen-reynolds)
 * are KN_SHEAR = tau_pi sqrt(sigma:sigma), REINV_SHEAR = sqrt(pi:pi)/p,
 * KN_BULK = tau_Pi theta, REINV_BULK = |Pi|/p, zero for ideal runs.  The
 * freeze-out surface element ("Freeze-out hypersurface construction") is
 * DE0..DE3 = d_mu e (spatial part in the n = 1 SPH difference form, d_0 e from
 * the energy equation D e = -(e + p + Pi) theta + pi:sigma + u.I) and
 * DSIG0..DSIG3 = d sigma_mu = n_mu / (sigma |u^mu n_mu|) with the outward
 * normal n_mu = -d_mu e / sqrt(|d e . d e|); zero where the normal is
 * undefined or orthogonal to u.  Lower indices; index 3 is eta or z. */
enum {
  CCAKE_AUX_SIGSTAR = 0, CCAKE_AUX_S, CCAKE_AUX_NB, CCAKE_AUX_NS, CCAKE_AUX_NQ, CCAKE_AUX_T,
  CCAKE_AUX_MUB, CCAKE_AUX_MUS, CCAKE_AUX_MUQ, CCAKE_AUX_P, CCAKE_AUX_E, CCAKE_AUX_CS2,
  CCAKE_AUX_INTABLE, CCAKE_AUX_GAMMA, CCAKE_AUX_THETA, CCAKE_AUX_NNB, CCAKE_AUX_F1,
  CCAKE_AUX_F2, CCAKE_AUX_F3, CCAKE_AUX_NEWTON, CCAKE_AUX_EOS_EVALS, CCAKE_AUX_KN_SHEAR,
  CCAKE_AUX_REINV_SHEAR, CCAKE_AUX_KN_BULK, CCAKE_AUX_REINV_BULK, CCAKE_AUX_DE0, CCAKE_AUX_DE1,
  CCAKE_AUX_DE2, CCAKE_AUX_DE3, CCAKE_AUX_DSIG0, CCAKE_AUX_DSIG1, CCAKE_AUX_DSIG2, CCAKE_AUX_DSIG3,
  CCAKE_NAUX
};

typedef struct ccake_eos ccake_eos;
typedef struct ccake_sim ccake_sim;
typedef struct ccake_server ccake_server;

/* Run parameters ("Equations of motion", "Transport coefficients", kernel h).
 *   dim            spatial dimensions carried by particles: 2 or 3
 *   coords         CCAKE_CARTESIAN (t,x,y[,z]) or CCAKE_HYPERBOLIC (tau,x,y[,eta])
 *   viscous        0 ideal; 1 minimal Israel-Stewart shear + bulk
 *   precision      CCAKE_FP64, or CCAKE_MIXED (pair sums in FP32 with Kahan
 *                  compensation; state, Newton, update and totals in FP64)
 *   ncharge        0 or 3 (B, S, Q)
 *   density_mode   CCAKE_DENS_SMOOTHED or CCAKE_DENS_SPECIFIC
 *   h              smoothing length (fm)
 *   eta_over_s     constant eta/s (eta = eta_over_s * s)
 *   zeta_*         zeta/s = zeta_peak exp(-(T - zeta_Tpeak)^2 / (2 zeta_width^2)), T in fm^-1
 *   taupi_coeff    tau_pi = taupi_coeff * eta / (e + p)
 *   tauPi_ratio    tau_Pi = tauPi_ratio * tau_pi
 *   c_PiPi,c_Pipi  first-order DNMR-type bulk couplings / tau_Pi (minimal IS: 1, 0)
 *   c_pipi,c_piPi  first-order DNMR-type shear couplings / tau_pi (minimal IS: 4/3, 0)
 *   skin           cell edge = 2h + skin; must exceed 2 dt max(1, 1/x0)
 *   diffusion      0 off; 1 BSQ charge diffusion ("BSQ diffusion", eq. min_dif_rel,
 *                  needs ncharge 3): J^mu_q relaxes towards +kappa_{qq'} nabla^mu
 *                  alpha_{q'} (alpha = mu/T, nabla^i alpha = g^{ii} d_i alpha) over
 *                  tau_J; the charges move by the n = -1 SPH divergence of
 *                  J - v J^0 and the entropy by -mu_q/T per unit charge moved
 *   kappa_T2       kappa_{qq'}/T^2, row-major (B, S, Q), constant
 *   tauJ_coeff     tau_J = tauJ_coeff / T (the paper's example: 0.2)
 *   c_JJ           coefficient of the -c_JJ tau_J J^mu theta term (0 by default)
 *   c_pisig        coefficient (Lambda_pipi / (beta tau_pi) of eq. diffusion-evol)
 *                  of the shear term pi_lambda^<mu sigma^nu>lambda; 0 by default,
 *                  must be finite, read only by viscous runs
 *   d_JPi          delta_JPi^q / beta (B, S, Q) of the coupling of the currents
 *                  to the bulk-pressure gradient (eq. diffusion-evol): the
 *                  relaxation target becomes kappa_{qq'} g^{ii} (d_i alpha_{q'}
 *                  + d_JPi[q'] d_i Pi); 0 by default, must be finite, read only
 *                  by viscous runs with diffusion */
typedef struct ccake_config {
  int32_t dim, coords, viscous, precision, ncharge, density_mode;
  double h;
  double eta_over_s;
  double zeta_peak, zeta_Tpeak, zeta_width;
  double taupi_coeff, tauPi_ratio;
  double c_PiPi, c_Pipi, c_pipi, c_piPi;
  double skin;
  int32_t diffusion, pad0;
  double kappa_T2[9];
  double tauJ_coeff, c_JJ;
  double c_pisig;
  double d_JPi[3];
} ccake_config;

/* Per-event counters of the last evaluation (ccake_totals).  newton_hist[k]
 * counts the particles whose EoS inversion took k Newton iterations (gas and
 * table solves together), k = 0 .. CCAKE_NEWTON_BINS - 2; the last bin holds
 * CCAKE_NEWTON_BINS - 1 iterations or more. */
enum { CCAKE_NEWTON_BINS = 12 };
typedef struct ccake_counters {
  uint32_t nonfinite;      /* sticky: non-finite particle updates */
  uint32_t noconv;         /* sticky: EoS inversions that failed */
  uint32_t backup;         /* last stage: inversions served by the backup EoS */
  uint32_t newton_iters;   /* last stage: total Newton iterations */
  int32_t first_bad;       /* lowest particle index with a non-finite update, or -1 */
  uint32_t capacity_err;   /* sticky: cell-grid capacity problems */
  int64_t in_table;        /* particles whose inversion the table answered */
  int64_t newton_hist[CCAKE_NEWTON_BINS];
} ccake_counters;

/* ---------------------------------------------------------------- EoS ---- */

/* Conformal EoS e = fstar T^4, p = e/3 (charges ignored); inversion in closed
 * form.  Paper: conformal EoS of the Gubser checks ("Code validation").      */
ccake_status ccake_eos_create_conformal(ccake_eos** out, double fstar);

/* Analytic massless gas of u, d, s quarks and gluons,
 * p = (19 pi^2/36) T^4 + sum_f [mu_f^2 T^2/2 + mu_f^4/(4 pi^2)];
 * inverted by damped Newton with the analytic Jacobian.                      */
ccake_status ccake_eos_create_gas(ccake_eos** out, int32_t max_iter, double tol);

/* Tabulated 4D EoS on a regular (T, muB, muS, muQ) grid ("Equation of state",
 * online inverter of "EoS inverter") with the analytic gas as backup EoS.
 *   n[4]        nodes per axis (>= 2 each)
 *   lo[4],hi[4] axis ranges in fm^-1
 *   cols        host array [7][n0][n1][n2][n3]: p/T^4, s/T^3, nB/T^3,
 *               nS/T^3, nQ/T^3, c_s^2, (dp/de)_n (dimensionless); copied to a
 *               device table owned by the EoS (node-major, 64 B per node)
 *   max_iter    Newton iterations per solve; tol: max scaled residual
 * Inversion: the backup gas root is found first; when it lies inside the axes
 * the table interpolant is solved from it and used if it converges inside.  */
ccake_status ccake_eos_create_table(ccake_eos** out, const int32_t n[4], const double lo[4], const double hi[4],
                                    const double* cols, int32_t max_iter, double tol);

ccake_status ccake_eos_destroy(ccake_eos* eos);

/* Batch inversion (s or e, nB, nS, nQ) -> (T, muB, muS, muQ) on the device.
 *   mode     0: entropy density given; 1: energy density given
 *   in, out  device arrays [4][n]; in_table (optional, device int32[n]) gets 1
 *            when the table answered, 0 when the backup did
 *   stream   hipStream_t (NULL = default stream); asynchronous
 * Returns CCAKE_E_EOS_NOCONV after synchronising when some solve failed.     */
ccake_status ccake_eos_invert(ccake_eos* eos, int32_t mode, int32_t ncharge, int64_t n, const double* in,
                              double* out, int32_t* in_table, void* stream);

/* Allocation-free form of ccake_eos_invert, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and errors.  Its only
 * scratch, the count of failed inversions, lives in a 256-byte device array
 * of the library that every call on a device shares (its size does not depend
 * on n, so no n is too large for it); calls that overlap on one device race
 * on that count.  Allocates nothing (no hipMalloc, no pinned memory); clears
 * the count with a kernel; synchronises the stream like ccake_eos_invert.     */
ccake_status ccake_eos_invert_noalloc(ccake_eos* eos, int32_t mode, int32_t ncharge, int64_t n, const double* in,
                                      double* out, int32_t* in_table, void* stream);

/* Offline inverter ("EoS inverter", offline option): the thermodynamics are
 * converted once onto a fixed grid in the hydrodynamic variables, and the
 * stages then interpolate instead of root-finding.  The s nodes are evenly
 * spaced inside logarithmic decades, 10^d (1 + 9 m / per_decade) for
 * decade_lo <= d < decade_hi and m = 0 .. per_decade - 1, then
 * 10^decade_hi (fm^-3); with ncharge = 3 the ratios x_q = n_q / s (B, S, Q)
 * take nx[q] >= 2 uniform values in [x_lo[q], x_hi[q]].  At most 2^28 nodes. */
typedef struct ccake_inv_grid {
  int32_t ncharge;              /* 0 (s only, mu = 0) or 3 */
  int32_t decade_lo, decade_hi;
  int32_t per_decade;
  int32_t nx[3];
  int32_t pad;
  double x_lo[3], x_hi[3];
} ccake_inv_grid;

/* Builds the offline table of eos on the device: every node is inverted
 * once by the online inverter (cold start) and T, mu_B, mu_S, mu_Q, p, e,
 * c_s^2, (dp/de)_n and the table/backup origin are stored (replacing any
 * previous table; the device memory belongs to eos).  Simulations and servers
 * created afterwards with eos interpolate it multilinearly in (s, x_B, x_S,
 * x_Q) for the (s, n) inversions of their stages, invert online off the grid,
 * and must have the table's ncharge.  A point is reported in the table when
 * every corner node with a weight above 1e-9 is.  ccake_eos_invert stays online.
 * Synchronises the stream.  Errors: CCAKE_E_ARG for a bad grid,
 * CCAKE_E_CAPACITY above 2^28 nodes, CCAKE_E_EOS_NOCONV when a node does not
 * converge (no table is attached then).                                      */
ccake_status ccake_eos_build_inverted(ccake_eos* eos, const ccake_inv_grid* grid, void* stream);

/* Lookups in the offline table at n points in = [4][n] (s, nB, nS, nQ),
 * device pointers: out [9][n] = T, muB, muS, muQ, p, e, c_s^2, (dp/de)_n,
 * in_table (0/1); inside[n] = 1 for points on the grid.  Points off the grid
 * are inverted online when fallback != 0, else set to NaN.  Synchronises.
 * CCAKE_E_STATE when eos has no offline table.                              */
ccake_status ccake_eos_offline_eval(ccake_eos* eos, int32_t fallback, int64_t n, const double* in, double* out,
                                    int32_t* inside, void* stream);

/* --------------------------------------------------------- simulation ---- */

/* Device bytes a simulation of n particles needs; the caller allocates them
 * (e.g. a torch uint8 tensor) and passes the pointer to ccake_create.        */
ccake_status ccake_workspace_bytes(const ccake_config* cfg, int64_t n, size_t* bytes);

/* Creates a simulation of n particles in a caller-owned device workspace of at
 * least ccake_workspace_bytes bytes (256-byte aligned).  The workspace and the
 * EoS must outlive the simulation.  stream: hipStream_t (NULL = default).    */
ccake_status ccake_create(ccake_sim** out, const ccake_config* cfg, const ccake_eos* eos, int64_t n,
                          void* workspace, size_t bytes, void* stream);

/* Initial condition at x0 = t0 ("SPH interpretation of a fluid element",
 * m_b = 1): positions xi [dim][n], flow u^i [dim][n] (contravariant), and
 * dens [4][n] = (s or e, nB, nS, nQ) in the rest frame (dens_kind
 * CCAKE_INIT_S or CCAKE_INIT_E).  Computes sigma*_a = sum_b W_ab and sets
 * S_a = s_a gamma_a sqrt(-g)/sigma*_a, N_a likewise, Pi = pi = 0.
 * CCAKE_E_ARG on non-finite input or negative s / e.  Synchronises.          */
ccake_status ccake_init_particles(ccake_sim* sim, double t0, const double* xi, const double* u, int32_t dens_kind,
                                  const double* dens, int32_t mem);

/* Raw state upload / download in the CCAKE_NROW-row exchange format (checkpoint and
 * restore).  get_state synchronises.                                         */
ccake_status ccake_set_state(ccake_sim* sim, double t, const double* y, int32_t mem);
ccake_status ccake_get_state(ccake_sim* sim, double* y, int32_t mem);
ccake_status ccake_time(const ccake_sim* sim, double* t);

/* nsteps Heun (second-order Runge-Kutta) steps of size dt; each stage bins the
 * particles, forms the density sums, inverts the EoS, forms the gradient sums
 * and solves the local equations of motion.  Asynchronous on the stream;
 * returns a sticky error (CCAKE_E_NONFINITE / CCAKE_E_EOS_NOCONV /
 * CCAKE_E_CAPACITY) already observed from an earlier call.                   */
ccake_status ccake_step(ccake_sim* sim, double dt, int32_t nsteps);

/* External sources of energy-momentum and charge, I^nu and I_q of
 * eq. conservation_source, deposited as in the smeared parton source of the
 * dynamical-initialisation section: each source is a normalised Gaussian in
 * the particle coordinates (the third one is eta times 1 fm, as in the kernel
 * distance) whose centre moves with constant coordinate velocity, active for
 * t_on <= x0 < t_off, with densities
 *     I^mu = (dp^mu/dx0) G / sqrt(-g),    I_q = (dN_q/dx0) G / sqrt(-g),
 * so that the deposited totals per unit x0 are dpdt and dndt (per unit
 * rapidity in 2+1D hyperbolic runs).  They enter the energy equation through
 * u.I, the momentum balance through the spatial components, the entropy
 * through (u.I - mu_q I_q)/T (eq. dsdnrewr) and the charges through
 * dN_q/dx0 = I_q/(gamma sigma).                                              */
typedef struct ccake_source {
  double x0[3];     /* centre at x0 = t_on (fm; eta for the third axis of hyperbolic runs) */
  double vel[3];    /* d centre / dx0 */
  double width[3];  /* Gaussian widths (> 0 on the dim axes used) */
  double t_on, t_off;
  double dpdt[4];   /* contravariant dp^mu/dx0 deposited, fm^-2 */
  double dndt[3];   /* dN_q/dx0 deposited (B, S, Q), fm^-1 */
} ccake_source;

enum { CCAKE_MAX_SOURCES = 16 };

/* Replaces the simulation's sources (nsrc = 0 removes them).  Copied to the
 * device on the simulation's stream, ordered after the steps already enqueued
 * and before later ones; synchronises.  CCAKE_E_ARG when nsrc exceeds
 * CCAKE_MAX_SOURCES or a width on a used axis is not positive.               */
ccake_status ccake_set_sources(ccake_sim* sim, int32_t nsrc, const ccake_source* src);

/* Synchronises and reports the sticky per-particle error state.             */
ccake_status ccake_check(ccake_sim* sim);

/* Measurement support.  With profiling enabled, ccake_step launches its
 * kernels directly (no HIP graph) on the simulation's stream, with HIP timing
 * events recorded around the binning kernels and, for each kernel of both
 * Heun stages, by the kernel's own dispatch (start and stop, so the gaps
 * between launches are not counted), and synchronises at the end of the
 * call.  Enabling resets
 * the accumulators.  ccake_kernel_times returns, per group (0 binning, 1
 * density sums, 2 EoS inversion, 3 gradient sums, 4 equations of motion and
 * update), the summed milliseconds and the number of launches.              */
enum { CCAKE_NPROF = 5 };
ccake_status ccake_set_profiling(ccake_sim* sim, int32_t enable);
ccake_status ccake_kernel_times(ccake_sim* sim, double ms[CCAKE_NPROF], int64_t launches[CCAKE_NPROF]);

/* One evaluation of the right-hand side at the current state, without
 * stepping: rates f [CCAKE_NROW][n] and diagnostics aux [CCAKE_NAUX][n] (either may be
 * NULL), caller order.  Synchronises.                                        */
ccake_status ccake_rhs(ccake_sim* sim, double* f, double* aux, int32_t mem);

/* One diagnostic field (CCAKE_AUX_*) at the current state, caller order.     */
ccake_status ccake_read(ccake_sim* sim, int32_t field, double* out, int32_t mem);

/* Several diagnostic fields from one evaluation at the current state: bit k
 * of mask selects CCAKE_AUX_k, whose n values (caller order) go to out[k]
 * (host or device per mem; entries of unselected fields are not read).  The
 * state rows themselves come from ccake_get_state.  CCAKE_E_ARG for a mask
 * with bits at or beyond CCAKE_NAUX or a selected NULL output.  Synchronises. */
ccake_status ccake_read_fields(ccake_sim* sim, uint64_t mask, double* const* out, int32_t mem);

/* Totals at the current state: out[8] = (S, N_B, N_S, N_Q, E, M_1, M_2, M_3)
 * with E = sum sqrt(-g) T^00/sigma* and M_i = sum sqrt(-g) G_ii T^0i/sigma*;
 * with diffusion a particle's charge is N_q + sqrt(-g) J^0_q/sigma*
 * (conserved energy and momentum in Cartesian coordinates; "Exact
 * conservation").  cnt (optional) receives the counters of that evaluation:
 * the backup count, the in-table count and the histogram of Newton
 * iterations per particle ("EoS inverter").  Synchronises.                  */
ccake_status ccake_totals(ccake_sim* sim, double* out, ccake_counters* cnt);

/* Test support: the neighbour relation {(a, b) : |x_a - x_b|^2 < (2h)^2}
 * (self included) at the current positions, as caller indices, in no
 * particular order.  a, b: device int32 arrays of capacity cap; npairs gets
 * the total (pairs beyond cap are counted but not written).  Synchronises.  */
ccake_status ccake_debug_pairs(ccake_sim* sim, int64_t cap, int32_t* a, int32_t* b, int64_t* npairs);

/* Test support: the pairs that the density pass of the next step accepts,
 * exported by that pass itself (the same kernel, neighbour tiles and pair
 * test) at the current positions through the neighbour rows of the last
 * binning, without binning again ("Neighbor search" and the kernel support
 * of "Kernel function": |x_a - x_b|^2 < (2h)^2, self included).  Same output
 * convention as ccake_debug_pairs.  CCAKE_E_STATE when the next step bins
 * first (right after initialisation or a state upload).  Synchronises.      */
ccake_status ccake_debug_pairs_cached(ccake_sim* sim, int64_t cap, int32_t* a, int32_t* b, int64_t* npairs);

/* Freeze-out hypersurface ("Freeze-out hypersurface construction", eq.
 * efo_surface and eq. fonormal).  With e_fo > 0 every step looks, at its
 * start x^0 = t_k, for the particles whose energy density fell below e_fo
 * since the previous step start (e(t_{k-1}) >= e_fo > e(t_k)), each particle
 * once.  A crossing particle gets one record of CCAKE_FO_NCOL doubles:
 *   ID        caller index of the particle (as a double)
 *   T         x^0 of the crossing, t_k - (t_k - t_{k-1}) (e_fo - e_k) / (e_{k-1} - e_k)
 *   X1..X3    position moved back to that x^0 along dx^i/dx^0 = u^i/u^0
 *   U1..U3    u^i at t_k
 *   TEMP, MUB, MUS, MUQ   T and mu_q at t_k (fm^-1)
 *   DS0..DS3  d sigma_mu at t_k as in CCAKE_AUX_DSIG0..3
 * (unused spatial components zero).  The step start's energy densities come
 * from the step's own first stage, so the surface costs no extra evaluation.
 * ccake_set_freezeout(e_fo) (0 switches the surface off) forgets the records
 * and every particle's history; so do ccake_init_particles and
 * ccake_set_state.  Synchronises.  CCAKE_E_ARG for a negative or non-finite
 * e_fo.                                                                       */
enum {
  CCAKE_FO_ID = 0, CCAKE_FO_T, CCAKE_FO_X1, CCAKE_FO_X2, CCAKE_FO_X3, CCAKE_FO_U1, CCAKE_FO_U2,
  CCAKE_FO_U3, CCAKE_FO_TEMP, CCAKE_FO_MUB, CCAKE_FO_MUS, CCAKE_FO_MUQ, CCAKE_FO_DS0, CCAKE_FO_DS1,
  CCAKE_FO_DS2, CCAKE_FO_DS3,
  CCAKE_FO_NCOL
};
ccake_status ccake_set_freezeout(ccake_sim* sim, double e_fo);

/* The records found so far, in the order found (not sorted by particle):
 * count gets their number (at most n) and out [count][CCAKE_FO_NCOL] (host
 * or device per mem) the first min(count, cap) of them.  Synchronises.       */
ccake_status ccake_freezeout_records(ccake_sim* sim, int64_t cap, double* out, int64_t* count, int32_t mem);

ccake_status ccake_destroy(ccake_sim* sim);

/* ------------------------------------------------------------ serving ---- */

/* A persistent serving loop: events of uneven particle count are submitted
 * as they arrive, admitted when their device footprint fits the budget and a
 * slot is free, advanced together by batched launches (one Heun step over all
 * resident events per iteration), and returned when they reach t_end.  A
 * host thread owns the loop; the device work runs on the server's stream.
 *   budget_bytes     device bytes the resident events may occupy
 *   max_particles    resident particle capacity; max_events: slot capacity
 *   dt               step of every event                                     */
typedef struct ccake_event_desc {
  int64_t n;              /* particles */
  double t0, t_end;       /* start and end of the evolution */
  const double* xi;       /* host [dim][n] */
  const double* u;        /* host [dim][n] */
  int32_t dens_kind;      /* CCAKE_INIT_S or CCAKE_INIT_E */
  const double* dens;     /* host [4][n]; copied at submission */
  int64_t user_tag;
} ccake_event_desc;

typedef struct ccake_event_result {
  int64_t ticket, user_tag, n;
  int32_t status;         /* ccake_status of the event */
  int32_t steps;
  double t_submit, t_admit, t_finish;  /* seconds on the server's clock */
  double* state;          /* host [CCAKE_NROW][n], owned by the server until ccake_server_release */
  double totals[8];
} ccake_event_result;

/* Device bytes of a server's arena (every resident event's state, the cell
 * grid and the event table) for max_particles and max_events.               */
ccake_status ccake_server_workspace_bytes(const ccake_config* cfg, int64_t max_particles, int32_t max_events,
                                          size_t* bytes);
/* workspace: caller-owned device memory of at least ws_bytes >=
 * ccake_server_workspace_bytes bytes (256-byte aligned), which must outlive
 * the server; NULL lets the server allocate (and free) its arena itself.    */
ccake_status ccake_server_create(ccake_server** out, const ccake_config* cfg, const ccake_eos* eos,
                                 size_t budget_bytes, int64_t max_particles, int32_t max_events, double dt,
                                 void* stream, void* workspace, size_t ws_bytes);
/* Copies the event's arrays and queues it; returns its ticket.  Rejects with
 * CCAKE_E_CAPACITY an event that can never fit the budget or capacity.      */
ccake_status ccake_server_submit(ccake_server* srv, const ccake_event_desc* ev, int64_t* ticket);
/* Moves up to cap finished events into res; *count gets how many.           */
ccake_status ccake_server_poll(ccake_server* srv, ccake_event_result* res, int32_t cap, int32_t* count);
/* Blocks until every submitted event has finished.                           */
ccake_status ccake_server_drain(ccake_server* srv);
ccake_status ccake_server_release(ccake_server* srv, ccake_event_result* res);
/* Server clock (seconds since creation) and counters. */
ccake_status ccake_server_stats(ccake_server* srv, double* now, int64_t* steps, int64_t* particle_steps,
                                int32_t* resident);
ccake_status ccake_server_destroy(ccake_server* srv);

/* Message of the last failure on a handle (eos, sim or server); never NULL. */
const char* ccake_last_error(const void* handle);

#ifdef __cplusplus
}
#endif

#endif /* CCAKE_H */

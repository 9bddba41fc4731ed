/*
 * ccake_oracle.c -- plain FP64 CPU reference for one Runge-Kutta stage of
 * relativistic viscous SPH with B/S/Q charges (CCAKE 2.0, arXiv 2511.22852).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no source,
 * header, table or helper with the HIP library; the two meet only through
 * the seeded input generators.
 *
 * Everything is written the slow, obvious way: double precision, brute-force
 * O(N^2) neighbour search unless a uniform grid is requested (the grid search
 * is checked against brute force by the tests), sums in ascending particle
 * order, one particle at a time.
 *
 * Units: hbar = c = 1, lengths in fm, T and mu in fm^-1, s and n in fm^-3,
 * energy density and pressure in fm^-4.
 *
 * Paper passages followed (section names of the paper):
 *   kernel and its gradient ............ "Kernel function" (cubic spline)
 *   density sums, sigma*, m_b = 1 ...... "SPH interpretation of a fluid element"
 *   n = -1 / n = 1 derivative forms .... "Derivatives in relativistic SPH"
 *   state {r, u, s/sigma, Pi/sigma, pi/sigma, n/sigma} and the
 *   M du/dx0 = F solve ................. "Equations of motion" (SPH), eq. genform,
 *                                        eq. unugeneral, eq. dsdnrewr
 *   conservation laws, decomposition .... eq. conservation_source, Eq. energy-Decom
 *   minimal Israel-Stewart ............. eq. min_bul_rel, eq. min_she_rel
 *   first-order DNMR-type couplings .... eq. dnmr (coefficients supplied by caller)
 *   online EoS inverter + backup ....... "EoS inverter", backup-EoS chain
 *   offline inverted table ............. "EoS inverter" (offline option; grid
 *                                        evenly spaced inside log decades of s)
 *   modified conformal EoS ............. Appendix "Modified EoS to permit lower eps_min"
 *
 * Readings where the paper is silent or garbled are restated at the point
 * of use below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- state layout: 26 rows of n doubles, original particle order ----
 * The last nine are the charge diffusion currents J^k_q / sigma (q = B, S, Q;
 * k = 1..3 contravariant spatial), zero unless diffusion is on. */
enum {
  V_X1, V_X2, V_X3, V_U1, V_U2, V_U3, V_S, V_NB, V_NS, V_NQ, V_B,
  V_P11, V_P12, V_P13, V_P22, V_P23, V_P33,
  V_JB1, V_JB2, V_JB3, V_JS1, V_JS2, V_JS3, V_JQ1, V_JQ2, V_JQ3, NVAR
};
/* ---- auxiliary outputs of one right-hand-side evaluation ---- */
enum {
  A_SIGSTAR, A_S, A_NB, A_NS, A_NQ, A_T, A_MUB, A_MUS, A_MUQ, A_P, A_E,
  A_CS2, A_INTABLE, A_GAMMA, A_THETA, A_NNB, A_F1, A_F2, A_F3,
  A_KN_SHEAR, A_REINV_SHEAR, A_KN_BULK, A_REINV_BULK,
  A_DE0, A_DE1, A_DE2, A_DE3, A_DSIG0, A_DSIG1, A_DSIG2, A_DSIG3, NAUX
};

typedef struct {
  int32_t dim;         /* spatial dimensions carried by particles: 2 or 3 */
  int32_t hyperbolic;  /* 1: (tau, x, y, eta), 0: Cartesian (t, x, y, z) */
  int32_t viscous;     /* 0 ideal, 1 minimal IS (+ optional DNMR couplings) */
  int32_t ncharge;     /* 0 or 3 */
  int32_t use_cells;   /* 0 brute-force search, 1 uniform-grid search */
  int32_t nthreads;    /* OpenMP threads, <= 0: runtime default */
  int32_t density_mode;/* 0: s = sum_b S_b W_ab / (gamma sqrt(-g)); 1: s = S sigma */
  int32_t pad0;
  double h;
  double eta_over_s;
  double zeta_peak, zeta_Tpeak, zeta_width; /* zeta/s Gaussian; T in fm^-1 */
  double taupi_coeff;  /* tau_pi = taupi_coeff * eta / w */
  double tauPi_ratio;  /* tau_Pi = tauPi_ratio * tau_pi */
  double c_PiPi;       /* delta_PiPi / tau_Pi  (minimal IS: 1)   */
  double c_Pipi;       /* lambda_Pipi / tau_Pi (minimal IS: 0)   */
  double c_pipi;       /* delta_pipi / tau_pi  (minimal IS: 4/3) */
  double c_piPi;       /* lambda_piPi / tau_pi (minimal IS: 0)   */
  int32_t nsrc;        /* external sources (eq. conservation_source), 0 = isolated */
  int32_t pad1;
  const struct orc_source *src;
  /* BSQ charge diffusion ("BSQ diffusion", eq. min_dif_rel); needs ncharge 3 */
  int32_t diffusion;   /* 0 off, 1 on */
  int32_t pad2;
  double kappa_T2[9];  /* kappa_{qq'} / T^2, row-major q*3+q' (constant matrix) */
  double tauJ_coeff;   /* tau_{qq'} = tauJ_coeff delta_{qq'} / T */
  double c_JJ;         /* coefficient of -tau_J J^mu theta (reading; 0 by default) */
  double c_pisig;      /* Lambda_pipi / (beta tau_pi) of the ADNH term pi_lambda^<mu sigma^nu>lambda */
  double d_JPi[3];     /* delta_JPi^q / beta of the ADNH diffusion term -kappa_qq' delta_JPi^q'/beta nabla^mu Pi */
} orc_params;

/* One external source of energy-momentum and charge (eq. conservation_source;
 * deposition smeared over the fluid as for the partons of the dynamical
 * initialisation).  Reading: a normalised Gaussian of widths w_k in the
 * particle coordinates (the third one is eta times 1 fm, as in the kernel
 * distance) whose centre moves with constant coordinate velocity, active for
 * t_on <= x0 < t_off.  The densities are
 *     I^mu = (dp^mu/dx0) G / sqrt(-g),   I_q = (dN_q/dx0) G / sqrt(-g),
 * so that the deposited totals per unit x0 are dp/dx0 and dN/dx0.  */
typedef struct orc_source {
  double x0[3];       /* centre at x0 = t_on */
  double vel[3];      /* d centre / dx0 */
  double width[3];    /* Gaussian widths */
  double t_on, t_off;
  double dpdt[4];     /* contravariant dp^mu/dx0 */
  double dndt[3];     /* dN_q/dx0 */
} orc_source;

enum { EOS_CONFORMAL = 0, EOS_TABLE = 1, EOS_GAS = 2, EOS_MODCONF = 3 };

typedef struct {
  int32_t kind;
  int32_t nT, nB, nS, nQ;
  int32_t max_iter;
  double fstar;          /* conformal: eps = fstar T^4 */
  double tol;            /* Newton: max scaled residual */
  double lo[4], hi[4];   /* table axes (T, muB, muS, muQ), fm^-1 */
  const double *cols;    /* [7][nT][nB][nS][nQ] dimensionless columns */
  double A0, muq0[3], cq[3]; /* modified conformal parameters (T0 = 1 fm^-1) */
  const struct orc_inv *inv; /* offline inverted table, or NULL (online inversion) */
} orc_eos;

/* table columns: p/T^4, s/T^3, nB/T^3, nS/T^3, nQ/T^3, c_s^2, (dp/de)_n */
enum { C_P, C_S, C_NB, C_NS, C_NQ, C_CS2, C_KAP, NCOL };

typedef struct {
  double T, mu[3], p, e, s, n[3], cs2, kappa;
  int in_table, iters, ok;
} thermo;

static int nthreads_of(const orc_params *prm)
{
#ifdef _OPENMP
  return prm->nthreads > 0 ? prm->nthreads : omp_get_max_threads();
#else
  (void)prm;
  return 1;
#endif
}

/* ========================================================================
 * Cubic-spline kernel ("Kernel function"): W = sigma_d w(q), q = r/h,
 * w = 1 - 1.5 q^2 + 0.75 q^3 (q <= 1), 0.25 (2-q)^3 (1 < q <= 2), 0 beyond;
 * sigma_2 = 10/(7 pi h^2), sigma_3 = 1/(pi h^3).
 * Gradient: (sigma_d/h) w'(q) (r_a - r_b)/r with w' = -3q + 9/4 q^2 or
 * -3/4 (2-q)^2; zero at r = 0 (reading: the direction is undefined there).
 * ======================================================================== */
static double sigma_d(int dim, double h)
{
  if (dim == 2) return 10.0 / (7.0 * M_PI * h * h);
  if (dim == 3) return 1.0 / (M_PI * h * h * h);
  return 2.0 / (3.0 * h);
}

double orc_kernel_w(int dim, double h, double r)
{
  double q = r / h;
  double w;
  if (q <= 1.0) w = 1.0 - 1.5 * q * q + 0.75 * q * q * q;
  else if (q <= 2.0) w = 0.25 * (2.0 - q) * (2.0 - q) * (2.0 - q);
  else w = 0.0;
  return sigma_d(dim, h) * w;
}

/* returns (sigma_d/h) w'(q) / r, so that grad_a W_ab = this * (r_a - r_b) */
double orc_kernel_dw_over_r(int dim, double h, double r)
{
  if (r <= 0.0) return 0.0;
  double q = r / h;
  double dw;
  if (q <= 1.0) dw = -3.0 * q + 2.25 * q * q;
  else if (q <= 2.0) dw = -0.75 * (2.0 - q) * (2.0 - q);
  else dw = 0.0;
  return sigma_d(dim, h) / h * dw / r;
}

/* ========================================================================
 * Neighbour relation: b is a neighbour of a iff d^2 < (2h)^2, d^2 summed
 * over the particle coordinates in axis order, each product and sum rounded
 * separately (this file is compiled without FMA contraction).  Self included.
 * In hyperbolic 3+1D eta enters with a 1 fm factor.
 * ======================================================================== */
static double dist2(int dim, const double *y, int64_t n, int64_t a, int64_t b)
{
  double d2 = 0.0;
  for (int k = 0; k < dim; ++k) {
    double dx = y[(V_X1 + k) * n + a] - y[(V_X1 + k) * n + b];
    d2 = d2 + dx * dx;
  }
  return d2;
}

/* uniform-grid search structure (acceleration only; pair set identical to
 * brute force, which a test checks) */
typedef struct {
  int dim;
  int64_t nc[3];
  double lo[3], edge;
  int64_t *start; /* ncell + 1 */
  int64_t *list;  /* particle ids, ascending within each cell */
  int64_t *cell;  /* cell of each particle */
} grid_t;

static void grid_build(grid_t *g, int dim, double h, const double *y, int64_t n)
{
  g->dim = dim;
  g->edge = 2.0 * h * (1.0 + 1e-9);
  int64_t ncell = 1;
  for (int k = 0; k < 3; ++k) { g->nc[k] = 1; g->lo[k] = 0.0; }
  for (int k = 0; k < dim; ++k) {
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t a = 0; a < n; ++a) {
      double x = y[(V_X1 + k) * n + a];
      if (x < lo) lo = x;
      if (x > hi) hi = x;
    }
    if (n == 0) { lo = 0.0; hi = 0.0; }
    g->lo[k] = lo;
    g->nc[k] = (int64_t)floor((hi - lo) / g->edge) + 1;
    ncell *= g->nc[k];
  }
  g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  g->list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  g->cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t a = 0; a < n; ++a) {
    int64_t c = 0;
    for (int k = dim - 1; k >= 0; --k) {
      int64_t i = (int64_t)floor((y[(V_X1 + k) * n + a] - g->lo[k]) / g->edge);
      if (i < 0) i = 0;
      if (i >= g->nc[k]) i = g->nc[k] - 1;
      c = c * g->nc[k] + i;
    }
    g->cell[a] = c;
    g->start[c + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
  for (int64_t c = 0; c < ncell; ++c) fill[c] = g->start[c];
  for (int64_t a = 0; a < n; ++a) g->list[fill[g->cell[a]]++] = a; /* ascending ids */
  free(fill);
}

static void grid_free(grid_t *g)
{
  free(g->start);
  free(g->list);
  free(g->cell);
}

/* Neighbour list of particle a, ascending in b.  Returns count; the list is
 * grown with realloc. */
static int64_t neighbours(const orc_params *prm, const grid_t *g, const double *y,
                          int64_t n, int64_t a, int64_t **buf, int64_t *cap)
{
  const double r2max = (2.0 * prm->h) * (2.0 * prm->h);
  int64_t cnt = 0;
  if (!prm->use_cells) {
    for (int64_t b = 0; b < n; ++b) {
      if (dist2(prm->dim, y, n, a, b) < r2max) {
        if (cnt == *cap) { *cap = *cap * 2 + 64; *buf = (int64_t *)realloc(*buf, sizeof(int64_t) * (size_t)*cap); }
        (*buf)[cnt++] = b;
      }
    }
    return cnt;
  }
  int64_t ci[3] = {0, 0, 0}, c = g->cell[a];
  for (int k = 0; k < g->dim; ++k) { ci[k] = c % g->nc[k]; c /= g->nc[k]; }
  int64_t lo[3], hi[3];
  for (int k = 0; k < 3; ++k) {
    if (k < g->dim) { lo[k] = ci[k] > 0 ? ci[k] - 1 : 0; hi[k] = ci[k] + 1 < g->nc[k] ? ci[k] + 1 : g->nc[k] - 1; }
    else { lo[k] = 0; hi[k] = 0; }
  }
  for (int64_t i2 = lo[2]; i2 <= hi[2]; ++i2)
    for (int64_t i1 = lo[1]; i1 <= hi[1]; ++i1)
      for (int64_t i0 = lo[0]; i0 <= hi[0]; ++i0) {
        int64_t cc = (i2 * g->nc[1] + i1) * g->nc[0] + i0;
        for (int64_t j = g->start[cc]; j < g->start[cc + 1]; ++j) {
          int64_t b = g->list[j];
          if (dist2(prm->dim, y, n, a, b) < r2max) {
            if (cnt == *cap) { *cap = *cap * 2 + 64; *buf = (int64_t *)realloc(*buf, sizeof(int64_t) * (size_t)*cap); }
            (*buf)[cnt++] = b;
          }
        }
      }
  /* sort ascending so that sums run in particle order as with brute force */
  for (int64_t i = 1; i < cnt; ++i) {
    int64_t v = (*buf)[i], j = i - 1;
    while (j >= 0 && (*buf)[j] > v) { (*buf)[j + 1] = (*buf)[j]; --j; }
    (*buf)[j + 1] = v;
  }
  return cnt;
}

/* All ordered pairs (a, b), a ascending then b ascending.  Returns the total
 * count; writes at most cap pairs. */
int64_t orc_pairs(const orc_params *prm, int64_t n, const double *y, int64_t cap,
                  int32_t *pa, int32_t *pb)
{
  grid_t g;
  memset(&g, 0, sizeof g);
  if (prm->use_cells) grid_build(&g, prm->dim, prm->h, y, n);
  int64_t tot = 0, bcap = 0;
  int64_t *buf = NULL;
  for (int64_t a = 0; a < n; ++a) {
    int64_t c = neighbours(prm, &g, y, n, a, &buf, &bcap);
    for (int64_t j = 0; j < c; ++j) {
      if (tot < cap) { pa[tot] = (int32_t)a; pb[tot] = (int32_t)buf[j]; }
      ++tot;
    }
  }
  free(buf);
  if (prm->use_cells) grid_free(&g);
  return tot;
}

/* ========================================================================
 * Equation of state.
 *
 * Massless gas of u, d, s quarks and gluons (the synthetic EoS of the
 * lumpy-IC workloads):
 *   p = (19 pi^2/36) T^4 + sum_f [ mu_f^2 T^2 / 2 + mu_f^4 / (4 pi^2) ],
 *   mu_f = B_f muB + S_f muS + Q_f muQ.
 * It doubles as the analytic backup EoS of the table (reading of the backup
 * chain: for the synthetic table the backup is the same analytic gas).
 * ======================================================================== */
static const double FLAV[3][3] = {
  {1.0 / 3.0, 0.0, 2.0 / 3.0},   /* u: B, S, Q */
  {1.0 / 3.0, 0.0, -1.0 / 3.0},  /* d */
  {1.0 / 3.0, -1.0, -1.0 / 3.0}, /* s */
};

static void gas_eval(double T, const double mu[3], double *p, double *s, double n[3], double J[4][4])
{
  const double ag = 19.0 * M_PI * M_PI / 36.0;
  double mf[3];
  for (int f = 0; f < 3; ++f) mf[f] = FLAV[f][0] * mu[0] + FLAV[f][1] * mu[1] + FLAV[f][2] * mu[2];
  double pp = ag * T * T * T * T, ss = 4.0 * ag * T * T * T;
  double nf[3];
  for (int f = 0; f < 3; ++f) {
    pp += 0.5 * mf[f] * mf[f] * T * T + mf[f] * mf[f] * mf[f] * mf[f] / (4.0 * M_PI * M_PI);
    ss += mf[f] * mf[f] * T;
    nf[f] = mf[f] * T * T + mf[f] * mf[f] * mf[f] / (M_PI * M_PI);
  }
  if (p) *p = pp;
  if (s) *s = ss;
  if (n) for (int q = 0; q < 3; ++q) { n[q] = 0.0; for (int f = 0; f < 3; ++f) n[q] += FLAV[f][q] * nf[f]; }
  if (J) {
    J[0][0] = 12.0 * ag * T * T;
    for (int f = 0; f < 3; ++f) J[0][0] += mf[f] * mf[f];
    for (int q = 0; q < 3; ++q) {
      double d = 0.0;
      for (int f = 0; f < 3; ++f) d += 2.0 * mf[f] * T * FLAV[f][q];
      J[0][1 + q] = d;
      J[1 + q][0] = d;
      for (int r = 0; r < 3; ++r) {
        double c = 0.0;
        for (int f = 0; f < 3; ++f) c += FLAV[f][q] * FLAV[f][r] * (T * T + 3.0 * mf[f] * mf[f] / (M_PI * M_PI));
        J[1 + q][1 + r] = c;
      }
    }
  }
}

/* Modified conformal EoS (Appendix), T0 = 1 fm^-1:
 *   p = A0 [ T^4 + sum_q (mu_q/mu_q0)^4 + sum_q c_q T^2 (mu_q/mu_q0)^2 ]. */
static void mc_eval(const orc_eos *e, double T, const double mu[3], double *p, double *s, double n[3], double J[4][4])
{
  double A0 = e->A0;
  double pp = T * T * T * T, ss = 4.0 * T * T * T, jtt = 12.0 * T * T;
  for (int q = 0; q < 3; ++q) {
    double m0 = e->muq0[q], x = mu[q] / m0, c = e->cq[q];
    pp += x * x * x * x + c * T * T * x * x;
    ss += 2.0 * c * T * x * x;
    jtt += 2.0 * c * x * x;
    if (n) n[q] = A0 * (4.0 * x * x * x / m0 + 2.0 * c * T * T * x / m0);
    if (J) {
      J[0][1 + q] = J[1 + q][0] = A0 * 4.0 * c * T * x / m0;
      for (int r = 0; r < 3; ++r) J[1 + q][1 + r] = 0.0;
      J[1 + q][1 + q] = A0 * (12.0 * x * x / (m0 * m0) + 2.0 * c * T * T / (m0 * m0));
    }
  }
  if (p) *p = A0 * pp;
  if (s) *s = A0 * ss;
  if (J) J[0][0] = A0 * jtt;
}

/* Quadrilinear interpolation of table column c at x = (T, muB, muS, muQ);
 * value and gradient with respect to x.  Cells are located by floor and
 * clamped to the grid, so outside the grid the edge cell continues linearly
 * (the Newton iterates may pass there; accepted roots lie inside). */
static void tab_interp(const orc_eos *e, int c, const double x[4], double *val, double grad[4])
{
  const int nn[4] = {e->nT, e->nB, e->nS, e->nQ};
  int i0[4];
  double f[4], d[4];
  for (int k = 0; k < 4; ++k) {
    d[k] = (e->hi[k] - e->lo[k]) / (double)(nn[k] - 1);
    double u = (x[k] - e->lo[k]) / d[k];
    int i = (int)floor(u);
    if (i < 0) i = 0;
    if (i > nn[k] - 2) i = nn[k] - 2;
    i0[k] = i;
    f[k] = u - (double)i;
  }
  double v = 0.0, g[4] = {0.0, 0.0, 0.0, 0.0};
  for (int corner = 0; corner < 16; ++corner) {
    int bit[4];
    for (int k = 0; k < 4; ++k) bit[k] = (corner >> (3 - k)) & 1;
    size_t idx = (size_t)c;
    for (int k = 0; k < 4; ++k) idx = idx * (size_t)nn[k] + (size_t)(i0[k] + bit[k]);
    double val_c = e->cols[idx];
    double wk[4], dwk[4];
    for (int k = 0; k < 4; ++k) {
      wk[k] = bit[k] ? f[k] : 1.0 - f[k];
      dwk[k] = (bit[k] ? 1.0 : -1.0) / d[k];
    }
    v += wk[0] * wk[1] * wk[2] * wk[3] * val_c;
    for (int k = 0; k < 4; ++k) {
      double prod = dwk[k];
      for (int j = 0; j < 4; ++j) if (j != k) prod *= wk[j];
      g[k] += prod * val_c;
    }
  }
  *val = v;
  if (grad) for (int k = 0; k < 4; ++k) grad[k] = g[k];
}

/* s, n and their Jacobian from the table interpolant: s = T^3 I_s, n = T^3 I_n. */
static void tab_sn(const orc_eos *e, const double x[4], double sn[4], double J[4][4])
{
  double T = x[0];
  for (int r = 0; r < 4; ++r) {
    double v, g[4];
    tab_interp(e, C_S + r, x, &v, g);
    sn[r] = T * T * T * v;
    if (J) {
      J[r][0] = 3.0 * T * T * v + T * T * T * g[0];
      for (int k = 1; k < 4; ++k) J[r][k] = T * T * T * g[k];
    }
  }
}

/* thermodynamics at a point (T, mu) for the given EoS kind; table = 1 uses
 * the table interpolant, 0 the analytic form of the kind / backup */
static void thermo_at(const orc_eos *e, int use_table, double T, const double mu[3], thermo *th)
{
  th->T = T;
  for (int q = 0; q < 3; ++q) th->mu[q] = mu[q];
  if (e->kind == EOS_CONFORMAL) {
    th->e = e->fstar * T * T * T * T;
    th->p = th->e / 3.0;
    th->s = 4.0 * e->fstar * T * T * T / 3.0;
    for (int q = 0; q < 3; ++q) { th->n[q] = 0.0; th->mu[q] = 0.0; }
    th->cs2 = 1.0 / 3.0;
    th->kappa = 1.0 / 3.0;
    return;
  }
  if (e->kind == EOS_TABLE && use_table) {
    double x[4] = {T, mu[0], mu[1], mu[2]}, v;
    tab_interp(e, C_P, x, &v, NULL);
    th->p = T * T * T * T * v;
    double sn[4];
    tab_sn(e, x, sn, NULL);
    th->s = sn[0];
    for (int q = 0; q < 3; ++q) th->n[q] = sn[1 + q];
    th->e = T * th->s + mu[0] * th->n[0] + mu[1] * th->n[1] + mu[2] * th->n[2] - th->p;
    tab_interp(e, C_CS2, x, &th->cs2, NULL);
    tab_interp(e, C_KAP, x, &th->kappa, NULL);
    return;
  }
  if (e->kind == EOS_MODCONF) mc_eval(e, T, mu, &th->p, &th->s, th->n, NULL);
  else gas_eval(T, mu, &th->p, &th->s, th->n, NULL);
  th->e = 3.0 * th->p;
  th->cs2 = 1.0 / 3.0;
  th->kappa = 1.0 / 3.0;
}

/* ---- 4x4 linear solve, Gaussian elimination with partial pivoting ---- */
static int solve_n(int n, double A[4][4], double b[4], double x[4])
{
  double M[4][5];
  for (int i = 0; i < n; ++i) { for (int j = 0; j < n; ++j) M[i][j] = A[i][j]; M[i][n] = b[i]; }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r) if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
    if (M[piv][col] == 0.0 || !isfinite(M[piv][col])) return 0;
    if (piv != col) for (int j = 0; j <= n; ++j) { double t = M[col][j]; M[col][j] = M[piv][j]; M[piv][j] = t; }
    for (int r = col + 1; r < n; ++r) {
      double fct = M[r][col] / M[col][col];
      for (int j = col; j <= n; ++j) M[r][j] -= fct * M[col][j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double acc = M[i][n];
    for (int j = i + 1; j < n; ++j) acc -= M[i][j] * x[j];
    x[i] = acc / M[i][i];
  }
  return 1;
}

/* Scaled residual of the inversion problem at x = (T, mu).
 * mode 0: (s(x) - s0, n(x) - n0) / s0
 * mode 1: ((e(x) - e0)/e0, (n(x) - n0)/e0^(3/4))                           */
typedef struct {
  const orc_eos *e;
  int use_table, mode;
  double target[4];
} inv_ctx;

static void inv_resid(const inv_ctx *c, const double x[4], double r[4], double J[4][4])
{
  double sn[4], Jsn[4][4], p = 0.0, gp[4] = {0, 0, 0, 0};
  const orc_eos *e = c->e;
  if (e->kind == EOS_TABLE && c->use_table) {
    tab_sn(e, x, sn, Jsn);
    if (c->mode == 1) {
      double v, g[4], T = x[0];
      tab_interp(e, C_P, x, &v, g);
      p = T * T * T * T * v;
      gp[0] = 4.0 * T * T * T * v + T * T * T * T * g[0];
      for (int k = 1; k < 4; ++k) gp[k] = T * T * T * T * g[k];
    }
  } else if (e->kind == EOS_MODCONF) {
    mc_eval(e, x[0], x + 1, &p, &sn[0], sn + 1, Jsn);
    for (int k = 0; k < 4; ++k) gp[k] = sn[k]; /* grad p = (s, n) analytically */
  } else {
    gas_eval(x[0], x + 1, &p, &sn[0], sn + 1, Jsn);
    for (int k = 0; k < 4; ++k) gp[k] = sn[k];
  }
  if (c->mode == 0) {
    double sc = c->target[0];
    for (int i = 0; i < 4; ++i) {
      r[i] = (sn[i] - c->target[i]) / sc;
      for (int k = 0; k < 4; ++k) J[i][k] = Jsn[i][k] / sc;
    }
  } else {
    /* e = T s + mu.n - p */
    double en = x[0] * sn[0] + x[1] * sn[1] + x[2] * sn[2] + x[3] * sn[3] - p;
    double ge[4];
    for (int k = 0; k < 4; ++k) {
      ge[k] = x[0] * Jsn[0][k] + x[1] * Jsn[1][k] + x[2] * Jsn[2][k] + x[3] * Jsn[3][k] - gp[k];
    }
    ge[0] += sn[0];
    for (int q = 0; q < 3; ++q) ge[1 + q] += sn[1 + q];
    double e0 = c->target[0], ns = pow(e0, 0.75);
    r[0] = (en - e0) / e0;
    for (int k = 0; k < 4; ++k) J[0][k] = ge[k] / e0;
    for (int q = 1; q < 4; ++q) {
      r[q] = (sn[q] - c->target[q]) / ns;
      for (int k = 0; k < 4; ++k) J[q][k] = Jsn[q][k] / ns;
    }
  }
}

static double maxabs4(const double r[4])
{
  double m = 0.0;
  for (int k = 0; k < 4; ++k) { double a = fabs(r[k]); if (!(a <= m)) m = a; }
  return m;
}

/* Damped Newton: full step, halved until the max-norm of the scaled residual
 * decreases.  Unknowns are (T, muB, muS, muQ); with nq = 0 only T is solved
 * (mu = 0).  Table iterates are not confined to the axes: outside them the
 * interpolant continues linearly from the boundary cells, so a root that lies
 * outside is found as such (and then rejected by the caller) instead of
 * stalling against the boundary.  Returns 1 when the residual is below tol. */
static int newton(const inv_ctx *c, double x[4], int nq, int max_iter, double tol, int *iters)
{
  int nu = nq > 0 ? 4 : 1;
  double r[4], J[4][4];
  inv_resid(c, x, r, J);
  double nr = nq > 0 ? maxabs4(r) : fabs(r[0]);
  int it = 0;
  for (; it < max_iter; ++it) {
    if (nr <= tol) break;
    double rhs[4], dx[4] = {0, 0, 0, 0};
    for (int k = 0; k < nu; ++k) rhs[k] = -r[k];
    if (!solve_n(nu, J, rhs, dx)) break;
    double lam = 1.0, xt[4], rt[4], Jt[4][4], nrt = INFINITY;
    int accepted = 0;
    for (int hv = 0; hv < 40; ++hv) {
      for (int k = 0; k < 4; ++k) xt[k] = x[k] + (k < nu ? lam * dx[k] : 0.0);
      if (xt[0] <= 0.0) xt[0] = 0.5 * x[0];
      inv_resid(c, xt, rt, Jt);
      nrt = nq > 0 ? maxabs4(rt) : fabs(rt[0]);
      if (nrt < nr) { accepted = 1; break; }
      lam *= 0.5;
    }
    if (!accepted) break;
    memcpy(x, xt, sizeof xt);
    memcpy(r, rt, sizeof rt);
    memcpy(J, Jt, sizeof Jt);
    nr = nrt;
  }
  if (iters) *iters += it;
  return nr <= tol;
}

static int inside_table(const orc_eos *e, const double x[4])
{
  for (int k = 0; k < 4; ++k) if (!(x[k] >= e->lo[k] && x[k] <= e->hi[k])) return 0;
  return 1;
}

/* Invert (s or e, nB, nS, nQ) -> (T, mu) and fill the thermodynamics.
 * Conformal: closed form (charges ignored).  Gas / modified conformal:
 * Newton on the analytic form.  Table: the analytic gas is solved first; if
 * its root lies inside the table axes, Newton on the table interpolant starts
 * from it and is accepted when it converges inside the axes; otherwise the
 * analytic gas (backup) result is kept. */
static void invert(const orc_eos *e, int mode, int ncharge, const double in[4], thermo *th)
{
  double mu0[3] = {0.0, 0.0, 0.0};
  th->iters = 0;
  th->in_table = 0;
  th->ok = 1;
  if (e->kind == EOS_CONFORMAL) {
    double T = mode == 0 ? cbrt(3.0 * in[0] / (4.0 * e->fstar)) : pow(in[0] / e->fstar, 0.25);
    thermo_at(e, 0, T, mu0, th);
    return;
  }
  int nq = ncharge;
  inv_ctx c;
  c.e = e;
  c.mode = mode;
  for (int k = 0; k < 4; ++k) c.target[k] = (k == 0 || nq > 0) ? in[k] : 0.0;
  /* analytic (gas or modified conformal) solve from the mu = 0 guess */
  double a0 = e->kind == EOS_MODCONF ? e->A0 : 19.0 * M_PI * M_PI / 36.0;
  double x[4] = {mode == 0 ? cbrt(in[0] / (4.0 * a0)) : pow(in[0] / (3.0 * a0), 0.25), 0.0, 0.0, 0.0};
  c.use_table = 0;
  int ok = newton(&c, x, nq, e->max_iter * 4, e->tol, &th->iters);
  if (e->kind == EOS_TABLE && ok && inside_table(e, x)) {
    double xt[4];
    memcpy(xt, x, sizeof xt);
    c.use_table = 1;
    int okt = newton(&c, xt, nq, e->max_iter, e->tol, &th->iters);
    if (okt && inside_table(e, xt)) {
      thermo_at(e, 1, xt[0], xt + 1, th);
      th->in_table = 1;
      return;
    }
  }
  th->ok = ok;
  thermo_at(e, 0, x[0], x + 1, th);
}

int orc_eos_invert(const orc_eos *e, int mode, int ncharge, int64_t n, const double *in,
                   double *out, int32_t *in_table)
{
  int bad = 0;
#pragma omp parallel for reduction(+:bad) schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double v[4] = {in[i], in[n + i], in[2 * n + i], in[3 * n + i]};
    thermo th;
    invert(e, mode, ncharge, v, &th);
    out[i] = th.T;
    out[n + i] = th.mu[0];
    out[2 * n + i] = th.mu[1];
    out[3 * n + i] = th.mu[2];
    if (in_table) in_table[i] = th.in_table;
    if (!th.ok) bad++;
  }
  return bad;
}

/* ========================================================================
 * Offline inverter ("EoS inverter", offline option): the thermodynamics are
 * converted once, by the online inverter, onto a fixed grid in the
 * hydrodynamic variables, and a stage only interpolates.  The paper fixes
 * the idea and the s grid (evenly spaced inside logarithmic decades, e.g.
 * s = 0.01, 0.02, ..., 0.1, 0.2, ..., 1, 2, ..., 10); the rest is read as
 * follows:
 *  - s nodes: 10^d (1 + 9 m / P), m = 0..P-1, for decades d0 <= d < d1, then
 *    10^d1 (so the spacing is uniform inside a decade and continuous at its
 *    upper end);
 *  - charge coordinates: the ratios x_q = n_q / s (which can have either
 *    sign) on uniform grids [x_lo, x_hi] with nx nodes each;
 *  - each node stores T, mu_B, mu_S, mu_Q, p, e, c_s^2, kappa and whether the
 *    online inverter answered from the table (1) or the backup (0);
 *  - between nodes every stored quantity is multilinear in (s, x_B, x_S,
 *    x_Q), i.e. linear in s inside the decade segment; the point counts as a
 *    table point when every corner node with a weight above 1e-9 does (a
 *    point on a node face is decided by the nodes of that face, whatever
 *    the last bits of its coordinates);
 *  - a point outside the grid is inverted online.
 * ======================================================================== */
enum { I_T, I_MUB, I_MUS, I_MUQ, I_P, I_E, I_CS2, I_KAP, I_TAB, NINV };

typedef struct orc_inv {
  int32_t ncharge;      /* 0: table in s alone (mu = 0); 3: (s, x_B, x_S, x_Q) */
  int32_t d0, d1;       /* s from 10^d0 to 10^d1 fm^-3 */
  int32_t per_decade;   /* P: nodes per decade */
  int32_t nx[3];        /* nodes of x_q (ncharge 3; >= 2 each) */
  int32_t pad;
  double xlo[3], xhi[3];
  double *val;          /* [ns][nx_B][nx_S][nx_Q][NINV] */
} orc_inv;

/* 10^d by repeated multiplication (d small) */
static double pow10i(int d)
{
  double p = 1.0;
  for (int k = 0; k < (d < 0 ? -d : d); ++k) p *= 10.0;
  return d >= 0 ? p : 1.0 / p;
}

int64_t orc_inv_ns(const orc_inv *v) { return (int64_t)(v->d1 - v->d0) * v->per_decade + 1; }

static double inv_s_node(const orc_inv *v, int64_t g)
{
  if (g >= (int64_t)(v->d1 - v->d0) * v->per_decade) return pow10i(v->d1);
  int d = v->d0 + (int)(g / v->per_decade), m = (int)(g % v->per_decade);
  return pow10i(d) * (1.0 + 9.0 * m / v->per_decade);
}

static double inv_x_node(const orc_inv *v, int q, int k)
{
  return v->xlo[q] + (v->xhi[q] - v->xlo[q]) * k / (v->nx[q] - 1);
}

static int64_t inv_charge_nodes(const orc_inv *v)
{
  return v->ncharge ? (int64_t)v->nx[0] * v->nx[1] * v->nx[2] : 1;
}

/* Fills v->val by inverting every node online with the forward EoS e. */
int orc_inv_build(const orc_eos *e, orc_inv *v)
{
  const int64_t ns = orc_inv_ns(v), nc = inv_charge_nodes(v);
  int bad = 0;
#pragma omp parallel for reduction(+:bad) schedule(static)
  for (int64_t i = 0; i < ns * nc; ++i) {
    const int64_t g = i / nc;
    int64_t r = i % nc;
    double in[4] = {inv_s_node(v, g), 0.0, 0.0, 0.0};
    if (v->ncharge) {
      int k[3];
      k[2] = (int)(r % v->nx[2]);
      r /= v->nx[2];
      k[1] = (int)(r % v->nx[1]);
      k[0] = (int)(r / v->nx[1]);
      for (int q = 0; q < 3; ++q) in[1 + q] = inv_x_node(v, q, k[q]) * in[0];
    }
    thermo th;
    invert(e, 0, v->ncharge, in, &th);
    double *o = v->val + i * NINV;
    o[I_T] = th.T;
    for (int q = 0; q < 3; ++q) o[I_MUB + q] = th.mu[q];
    o[I_P] = th.p;
    o[I_E] = th.e;
    o[I_CS2] = th.cs2;
    o[I_KAP] = th.kappa;
    o[I_TAB] = th.in_table ? 1.0 : 0.0;
    if (!th.ok) bad++;
  }
  return bad;
}

/* Interpolated thermodynamics at in = (s, nB, nS, nQ); 0 when outside the grid. */
static int inv_lookup(const orc_inv *v, const double in[4], thermo *th)
{
  const double s = in[0];
  const int64_t ns = orc_inv_ns(v);
  if (!(s >= inv_s_node(v, 0) && s <= inv_s_node(v, ns - 1))) return 0;
  /* decade, then the segment inside it */
  int d = v->d0;
  while (d + 1 < v->d1 && s >= pow10i(d + 1)) ++d;
  int m = (int)floor((s / pow10i(d) - 1.0) * v->per_decade / 9.0);
  if (m < 0) m = 0;
  if (m > v->per_decade - 1) m = v->per_decade - 1;
  const int64_t g = (int64_t)(d - v->d0) * v->per_decade + m;
  const double s0 = inv_s_node(v, g), s1 = inv_s_node(v, g + 1);
  double f[4] = {(s - s0) / (s1 - s0), 0.0, 0.0, 0.0};
  int64_t k[4] = {g, 0, 0, 0};
  if (v->ncharge) {
    for (int q = 0; q < 3; ++q) {
      const double x = in[1 + q] / s;
      const double u = (x - v->xlo[q]) / (v->xhi[q] - v->xlo[q]) * (v->nx[q] - 1);
      if (!(u >= 0.0 && u <= v->nx[q] - 1)) return 0;
      int64_t kk = (int64_t)floor(u);
      if (kk > v->nx[q] - 2) kk = v->nx[q] - 2;
      k[1 + q] = kk;
      f[1 + q] = u - kk;
    }
  }
  const int nd = v->ncharge ? 4 : 1;
  double acc[NINV] = {0.0};
  int all_table = 1;
  for (int c = 0; c < (1 << nd); ++c) {
    double wgt = 1.0;
    int64_t idx = 0;
    for (int a = 0; a < nd; ++a) {
      const int bit = (c >> (nd - 1 - a)) & 1;
      wgt *= bit ? f[a] : 1.0 - f[a];
      const int64_t dim_n = a == 0 ? ns : v->nx[a - 1];
      idx = idx * dim_n + k[a] + bit;
    }
    const double *o = v->val + idx * NINV;
    for (int q = 0; q < NINV; ++q) acc[q] += wgt * o[q];
    if (wgt > 1e-9 && !(o[I_TAB] > 0.5)) all_table = 0;
  }
  th->T = acc[I_T];
  for (int q = 0; q < 3; ++q) {
    th->mu[q] = v->ncharge ? acc[I_MUB + q] : 0.0;
    th->n[q] = v->ncharge ? in[1 + q] : 0.0;
  }
  th->p = acc[I_P];
  th->e = acc[I_E];
  th->s = s;
  th->cs2 = acc[I_CS2];
  th->kappa = acc[I_KAP];
  th->in_table = all_table;
  th->iters = 0;
  th->ok = 1;
  return 1;
}

/* (s, n) -> thermodynamics for a stage: the offline table when the EoS
 * carries one and the point lies on its grid, the online inverter otherwise */
static void thermo_of_sn(const orc_eos *e, int ncharge, const double in[4], thermo *th)
{
  if (e->inv && inv_lookup(e->inv, in, th)) return;
  invert(e, 0, ncharge, in, th);
}

/* Offline lookups of n points in = [4][n] (s, nB, nS, nQ): out = [NINV][n]
 * (T, muB, muS, muQ, p, e, cs2, kappa, in_table); inside[i] = 1 when the
 * point was on the grid.  Points off the grid are inverted online when
 * fallback is set, else left as NaN. */
void orc_inv_eval(const orc_eos *e, int fallback, int64_t n, const double *in, double *out, int32_t *inside)
{
  const int ncharge = e->inv ? e->inv->ncharge : 0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double v[4] = {in[i], in[n + i], in[2 * n + i], in[3 * n + i]};
    thermo th;
    int on = e->inv && inv_lookup(e->inv, v, &th);
    inside[i] = on;
    if (!on) {
      if (fallback) {
        invert(e, 0, ncharge, v, &th);
      } else {
        for (int q = 0; q < NINV; ++q) out[q * n + i] = NAN;
        continue;
      }
    }
    out[I_T * n + i] = th.T;
    for (int q = 0; q < 3; ++q) out[(I_MUB + q) * n + i] = th.mu[q];
    out[I_P * n + i] = th.p;
    out[I_E * n + i] = th.e;
    out[I_CS2 * n + i] = th.cs2;
    out[I_KAP * n + i] = th.kappa;
    out[I_TAB * n + i] = th.in_table;
  }
}

int orc_ninv(void) { return NINV; }

/* thermodynamic columns at given (T, mu): p, e, s, nB, nS, nQ, cs2, kappa */
void orc_eos_eval(const orc_eos *e, int use_table, int64_t n, const double *x, double *out)
{
  for (int64_t i = 0; i < n; ++i) {
    double mu[3] = {x[n + i], x[2 * n + i], x[3 * n + i]};
    thermo th;
    thermo_at(e, use_table, x[i], mu, &th);
    out[i] = th.p;
    out[n + i] = th.e;
    out[2 * n + i] = th.s;
    for (int q = 0; q < 3; ++q) out[(3 + q) * n + i] = th.n[q];
    out[6 * n + i] = th.cs2;
    out[7 * n + i] = th.kappa;
  }
}

/* ========================================================================
 * Geometry: metric diag(1, -1, -1, -G3) with G3 = tau^2 (hyperbolic, index 3
 * = eta) or 1 (Cartesian, index 3 = z); sqrt(-g) = tau or 1.  Christoffel
 * symbols of the Milne metric: Gamma^0_33 = tau, Gamma^3_03 = Gamma^3_30 =
 * 1/tau.  In 2+1D index 3 is a symmetry direction: u^3 = 0, d_3 = 0.
 * ======================================================================== */
typedef struct {
  double g[4], ginv[4], G[4], Gdot[4];
  double sqrtg, dlnsqrtg;
  double Gam[4][4][4];
} geom;

static void geom_at(int hyperbolic, double t, geom *m)
{
  memset(m, 0, sizeof *m);
  double G3 = hyperbolic ? t * t : 1.0;
  m->g[0] = 1.0; m->g[1] = -1.0; m->g[2] = -1.0; m->g[3] = -G3;
  for (int k = 0; k < 4; ++k) m->ginv[k] = 1.0 / m->g[k];
  m->G[0] = 0.0; m->G[1] = 1.0; m->G[2] = 1.0; m->G[3] = G3;
  m->Gdot[3] = hyperbolic ? 2.0 * t : 0.0;
  m->sqrtg = hyperbolic ? t : 1.0;
  m->dlnsqrtg = hyperbolic ? 1.0 / t : 0.0;
  if (hyperbolic) {
    m->Gam[0][3][3] = t;
    m->Gam[3][0][3] = 1.0 / t;
    m->Gam[3][3][0] = 1.0 / t;
  }
}

/* ========================================================================
 * Per-particle equation-of-motion evaluation.
 *
 * For a trial acceleration a = du^i/dx0 every quantity the paper expresses as
 * "M du/dx0 + F" is evaluated numerically; the momentum balance residual
 * R(a) is affine in a, so the matrix of eq. unugeneral is recovered as
 * R(e_j) - R(0) and the system solved by elimination.
 *
 * Momentum balance (reading of the momentum row, which the paper does not
 * write out): the covariant spatial momentum per particle
 *     M_i/(sigma gamma) = (w+Pi) Q_i / sigma + G_i pi^{0i}/(sigma gamma),
 *     Q_i = G_i u^i,
 * obeys d/dx0 [M_i/(sigma gamma)] = -sqrt(-g) F_i, where F_i is the n = -1
 * SPH form of (1/sigma*)[d_i(p+Pi) + G_i d_j(pi^{ji} - v^j pi^{0i})].
 * The time derivative of (w+Pi)/sigma uses the energy equation:
 *     D((w+Pi)/sigma) = (pi:sigma + Dp + DPi)/sigma,
 *     Dp = -c_s^2 w theta + (dp/de)_n (-Pi theta + pi:sigma).
 * theta = dgamma/dx0 + gamma (div v + d ln sqrt(-g)/dx0).
 * Relaxation (eq. min_bul_rel, eq. min_she_rel, DNMR-type couplings):
 *     DPi = -(Pi + zeta theta)/tau_Pi - c_PiPi Pi theta + c_Pipi pi:sigma
 *     gamma d(pi^ij/sigma)/dx0 = (1/sigma)[(2 eta sigma^ij - pi^ij)/tau_pi
 *         + (1 - c_pipi) pi^ij theta + c_piPi Pi sigma^ij + c_pisig Q^ij
 *         - (u^i pi^{jl} + u^j pi^{il}) Du_l - u^l (Gam^i_lk pi^kj + Gam^j_lk pi^ik)]
 * with the ADNH shear term of eq. diffusion-evol, Q^{mu nu} = pi_lambda^<mu
 * sigma^nu>lambda: the symmetric, traceless, transverse part of
 * A^{mu nu} = pi^{mu lambda} g_{lambda lambda} sigma^{lambda nu}; both factors are
 * transverse, so Q^{mu nu} = (A^{mu nu} + A^{nu mu})/2 - Delta^{mu nu} pi:sigma / 3
 * (the term's theta/3 part has the form of the c_pipi term).
 * Entropy (eq. dsdnrewr, no diffusion):
 *     gamma sigma T dS/dx0 = u.I - mu_q I_q - Pi theta + pi:sigma.
 * External sources (eq. conservation_source): u.I adds to D eps (eq.
 * e_conservation), the covariant spatial components of I^nu to the momentum
 * balance, d/dx0 [M_i/(sigma gamma)] = -sqrt(-g) F_i + G_i I^i/(sigma gamma),
 * and I_q to the charges (eq. charge_conservation), dN_q/dx0 = I_q/(gamma sigma).
 * In Dp the source heats at fixed n: Dp gains (dp/de)_n u.I; the charge
 * source's (dp/dn_q)_e I_q is taken as zero (reading; exact for p = eps/3).
 *
 * BSQ diffusion ("BSQ diffusion", eq. min_dif_rel, eq. charge_conservation,
 * eq. genform with R^S_a = -mu_a/T of eq. dsdnrewr).  State V^k_q = J^k_q/sigma.
 * Readings:
 *   - sign: in the mostly-minus metric J^mu relaxes towards
 *     +kappa_{qq'} nabla^mu alpha_{q'} (alpha = mu/T), the sign of eq. dnmr
 *     that moves charge down its chemical-potential gradient;
 *   - nabla^i alpha = g^{ii} d_i alpha: the u^i D alpha part of the
 *     projection is dropped (for these equations of state alpha is a
 *     function of n/s, whose comoving derivative is itself first order);
 *   - the theta term of eq. min_dif_rel (coefficient 1/(2 beta), beta not
 *     given) enters as -c_JJ tau_J J theta with a caller-supplied c_JJ;
 *   - the pressure does not respond to diffusion ((dp/dn_q)_e = 0, as for
 *     the sources), so the momentum solve is unchanged (R^i_b = 0);
 *   - the ADNH bulk-gradient coupling of eq. diffusion-evol,
 *     -kappa_{qq'} delta_JPi^{q'}/beta nabla^mu Pi, written in the same
 *     metric as the alpha term: the target becomes
 *     kappa_{qq'} g^{ii} (d_i alpha_{q'} + d_JPi[q'] d_i Pi), with
 *     d_JPi = delta_JPi/beta caller-supplied (0 by default) and d_i Pi the
 *     n = 1 SPH gradient, like d_i alpha.
 * Relaxation, with Delta^mu_nu D J^nu = DJ^mu + u^mu J^nu Du_nu and
 * DJ^i = gamma dJ^i/dx0 + u^l Gam^i_lk J^k, D sigma = -sigma theta:
 *     gamma sigma dV^i/dx0 = (kappa_{qq'} g^{ii} d_i alpha_{q'} - J^i)/tau_J
 *         + (1 - c_JJ) J^i theta - u^i J^nu Du_nu - u^l Gam^i_lk J^k.
 * Charges: integrating eq. charge_conservation over the particle's
 * coordinate volume 1/sigma* (which moves with v) gives
 *     d/dx0 [N_q + sqrt(-g) J^0_q / sigma*] = [sqrt(-g) I_q - d_i(sqrt(-g) F^i_q)] / sigma*,
 * F^i = J^i - v^i J^0, J^0 = G_k u^k J^k / gamma (u_mu J^mu = 0); the flux
 * divergence takes the n = -1 form, so the charge moved between two
 * particles is equal and opposite and sum_a (N + sqrt(-g) J^0/sigma*) is
 * conserved.  Entropy: gamma sigma T dS/dx0 gains -mu_q gamma sigma dN_q/dx0.
 * ======================================================================== */
typedef struct {
  int D, viscous;
  geom m;
  double u[4], v[4];
  double dudx[4][4]; /* dudx[k][nu] = partial_k u^nu, k spatial */
  double divv;
  double F[4];
  double sigma, w, p, Pi, T, cs2, kappa, eta, zeta, taupi, tauPi;
  double pi[4][4];   /* pi^{mu nu} */
  double P[4][4];    /* pi^{ij} / sigma (spatial) */
  double cPiPi, cPipi, cpipi, cpiPi;
  double I[4], Iq[3], mu[3]; /* source densities I^mu, I_q; chemical potentials */
  int diffusion;
  double J[3][4];     /* J^mu_q (J^0 from orthogonality) */
  double V[3][4];     /* J^k_q / sigma (state) */
  double dalpha[3][4];/* d_k alpha_q, n = 1 form */
  double dPi[4];      /* d_k Pi, n = 1 form */
  double dJPi[3];     /* delta_JPi^q / beta */
  double divF[3];     /* sum_b (F_a/sigma*_a^2 + F_b/sigma*_b^2) . grad W  (~ d_i F^i / sigma*) */
  double kapJ[3][3];  /* diffusion matrix kappa_{qq'} */
  double tauJ, cJJ;
  double cpisig;
} pctx;

typedef struct {
  double R[4];
  double dS, dB, dN[3], dP[4][4], theta, pisig;
  double sigsig;   /* sigma^{mu nu} sigma_{mu nu} */
  double dV[3][4]; /* d(J^k_q/sigma)/dx0 */
} pout;

static void eom_eval(const pctx *c, const double a[4], pout *o)
{
  const geom *m = &c->m;
  const double *u = c->u;
  double gam = u[0];
  double num = 0.0;
  for (int i = 1; i < 4; ++i) num += m->G[i] * u[i] * a[i] + 0.5 * m->Gdot[i] * u[i] * u[i];
  double dgam = num / gam;
  double theta = dgam + gam * (c->divv + m->dlnsqrtg);
  double dudt[4] = {dgam, a[1], a[2], a[3]};
  double nab[4][4];
  for (int nu = 0; nu < 4; ++nu) {
    double d0 = dudt[nu];
    for (int k = 1; k < 4; ++k) d0 -= c->v[k] * c->dudx[k][nu];
    nab[0][nu] = d0;
    for (int k = 1; k < 4; ++k) nab[k][nu] = c->dudx[k][nu];
  }
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = 0; nu < 4; ++nu)
      for (int l = 0; l < 4; ++l) nab[mu][nu] += m->Gam[nu][mu][l] * u[l];
  double Du[4], Dl[4];
  for (int nu = 0; nu < 4; ++nu) {
    double acc = gam * dudt[nu];
    for (int k = 0; k < 4; ++k)
      for (int l = 0; l < 4; ++l) acc += m->Gam[nu][k][l] * u[k] * u[l];
    Du[nu] = acc;
    Dl[nu] = m->g[nu] * acc;
  }
  double sig[4][4];
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = 0; nu < 4; ++nu) {
      double Delta = (mu == nu ? m->ginv[mu] : 0.0) - u[mu] * u[nu];
      sig[mu][nu] = 0.5 * (m->ginv[mu] * nab[mu][nu] + m->ginv[nu] * nab[nu][mu])
                  - 0.5 * (u[mu] * Du[nu] + u[nu] * Du[mu]) - Delta * theta / 3.0;
    }
  double pisig = 0.0, sigsig = 0.0;
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = 0; nu < 4; ++nu) {
      pisig += c->pi[mu][nu] * m->g[mu] * m->g[nu] * sig[mu][nu];
      sigsig += sig[mu][nu] * m->g[mu] * m->g[nu] * sig[mu][nu];
    }
  o->sigsig = sigsig;
  double DPi = 0.0;
  if (c->viscous) DPi = -(c->Pi + c->zeta * theta) / c->tauPi - c->cPiPi * c->Pi * theta + c->cPipi * pisig;
  double uI = 0.0;
  for (int mu = 0; mu < 4; ++mu) uI += m->g[mu] * u[mu] * c->I[mu];
  double Dp = -c->cs2 * c->w * theta + c->kappa * (-c->Pi * theta + pisig + uI);
  memset(o->dP, 0, sizeof o->dP);
  if (c->viscous) {
    for (int i = 1; i < 4; ++i)
      for (int j = i; j < 4; ++j) {
        double val = (2.0 * c->eta * sig[i][j] - c->pi[i][j]) / c->taupi
                   + (1.0 - c->cpipi) * c->pi[i][j] * theta + c->cpiPi * c->Pi * sig[i][j];
        if (c->cpisig != 0.0) {
          double Aij = 0.0, Aji = 0.0;
          for (int l = 0; l < 4; ++l) {
            Aij += c->pi[i][l] * m->g[l] * sig[l][j];
            Aji += c->pi[j][l] * m->g[l] * sig[l][i];
          }
          double Delta = (i == j ? m->ginv[i] : 0.0) - u[i] * u[j];
          val += c->cpisig * (0.5 * (Aij + Aji) - Delta * pisig / 3.0);
        }
        for (int l = 0; l < 4; ++l) val -= (u[i] * c->pi[j][l] + u[j] * c->pi[i][l]) * Dl[l];
        for (int l = 0; l < 4; ++l)
          for (int k = 0; k < 4; ++k)
            val -= u[l] * (m->Gam[i][l][k] * c->pi[k][j] + m->Gam[j][l][k] * c->pi[i][k]);
        o->dP[i][j] = val / (gam * c->sigma);
        o->dP[j][i] = o->dP[i][j];
      }
  }
  o->theta = theta;
  o->pisig = pisig;
  double heat = uI - (c->mu[0] * c->Iq[0] + c->mu[1] * c->Iq[1] + c->mu[2] * c->Iq[2]);
  o->dS = ((c->viscous ? -c->Pi * theta + pisig : 0.0) + heat) / (gam * c->sigma * c->T);
  o->dB = c->viscous ? (DPi + c->Pi * theta) / (gam * c->sigma) : 0.0;
  for (int q = 0; q < 3; ++q) o->dN[q] = c->Iq[q] / (gam * c->sigma);
  memset(o->dV, 0, sizeof o->dV);
  if (c->diffusion) {
    for (int q = 0; q < 3; ++q) {
      double JDu = 0.0;
      for (int nu = 0; nu < 4; ++nu) JDu += c->J[q][nu] * Dl[nu];
      for (int i = 1; i <= c->D; ++i) {
        double target = 0.0;
        for (int r = 0; r < 3; ++r)
          target += c->kapJ[q][r] * m->ginv[i] * (c->dalpha[r][i] + c->dJPi[r] * c->dPi[i]);
        double val = (target - c->J[q][i]) / c->tauJ + (1.0 - c->cJJ) * c->J[q][i] * theta - u[i] * JDu;
        for (int l = 0; l < 4; ++l)
          for (int k = 0; k < 4; ++k) val -= u[l] * m->Gam[i][l][k] * c->J[q][k];
        o->dV[q][i] = val / (gam * c->sigma);
      }
      /* d/dx0 of sqrt(-g) J^0 / sigma* = J^0/(gamma sigma) = (G_k u^k V^k)/gamma^2 */
      double X = 0.0, dX = 0.0;
      for (int k = 1; k < 4; ++k) {
        X += m->G[k] * u[k] * c->V[q][k];
        dX += (m->Gdot[k] * u[k] + m->G[k] * a[k]) * c->V[q][k] + m->G[k] * u[k] * o->dV[q][k];
      }
      double dY = dX / (gam * gam) - 2.0 * X * dgam / (gam * gam * gam);
      double ddiff = -dY - m->sqrtg * c->divF[q];
      o->dN[q] += ddiff;
      o->dS -= c->mu[q] * ddiff / c->T;
    }
  }
  double dwPs = (pisig + Dp + DPi + uI) / (c->sigma * gam);
  for (int i = 0; i < 4; ++i) o->R[i] = 0.0;
  for (int i = 1; i <= c->D; ++i) {
    double Qi = m->G[i] * u[i];
    double dQ = m->G[i] * a[i] + m->Gdot[i] * u[i];
    double sQP = 0.0, dsQP = 0.0;
    for (int j = 1; j < 4; ++j) {
      sQP += m->G[j] * u[j] * c->P[j][i];
      dsQP += (m->G[j] * a[j] + m->Gdot[j] * u[j]) * c->P[j][i] + m->G[j] * u[j] * o->dP[j][i];
    }
    double dX = m->Gdot[i] / (gam * gam) * sQP - 2.0 * m->G[i] / (gam * gam * gam) * dgam * sQP
              + m->G[i] / (gam * gam) * dsQP;
    o->R[i] = (c->w + c->Pi) / c->sigma * dQ + Qi * dwPs + dX + m->sqrtg * c->F[i]
            - m->G[i] * c->I[i] / (gam * c->sigma);
  }
}

/* ========================================================================
 * One evaluation of the right-hand side f(x0, y) of the particle ODE.
 * ======================================================================== */
typedef struct {
  double sigstar, s, n[3];
  thermo th;
  double gam, v[4], u[4];
  double Pi, pi[4][4];
  double eta, zeta, taupi, tauPi;
  double ppi_over_s2;       /* (p + Pi)/sigma*^2 */
  double A_over_s2[4][4];   /* (pi^{ji} - v^j pi^{0i})/sigma*^2, [j][i] */
  double J[3][4];           /* diffusion currents J^mu_q */
  double alpha[3];          /* mu_q / T */
  double F_over_s2[3][4];   /* (J^k_q - v^k J^0_q)/sigma*^2 */
  int nnb;
} pass1_t;

/* Source densities at particle a and time t (see orc_source). */
static void sources_at(const orc_params *prm, const geom *m, double t, const double *y, int64_t n, int64_t a,
                       double I[4], double Iq[3])
{
  for (int k = 0; k < 4; ++k) I[k] = 0.0;
  for (int k = 0; k < 3; ++k) Iq[k] = 0.0;
  for (int k = 0; k < prm->nsrc; ++k) {
    const orc_source *S = &prm->src[k];
    if (!(t >= S->t_on && t < S->t_off)) continue;
    double G = 1.0;
    for (int d = 0; d < prm->dim; ++d) {
      double centre = S->x0[d] + S->vel[d] * (t - S->t_on);
      double dx = y[(V_X1 + d) * n + a] - centre;
      G *= exp(-dx * dx / (2.0 * S->width[d] * S->width[d])) / (sqrt(2.0 * M_PI) * S->width[d]);
    }
    for (int mu = 0; mu < 4; ++mu) I[mu] += S->dpdt[mu] * G / m->sqrtg;
    for (int q = 0; q < 3; ++q) Iq[q] += S->dndt[q] * G / m->sqrtg;
  }
}

static double gamma_of(const geom *m, const double u[4])
{
  return sqrt(1.0 + m->G[1] * u[1] * u[1] + m->G[2] * u[2] * u[2] + m->G[3] * u[3] * u[3]);
}

/* Right-hand side at every particle (targets == NULL; outputs [row][n]) or at
 * the listed target particles only (outputs [row][nt], in the order of the
 * list).  For targets, pass 1 runs on the targets and their neighbours,
 * which is all that their pass 2 reads. */
static int rhs_impl(const orc_params *prm, const orc_eos *eos, double t, int64_t n, const double *y,
                    int64_t nt, const int64_t *targets, double *dydt, double *aux)
{
  const int D = prm->dim;
  geom m;
  geom_at(prm->hyperbolic, t, &m);
  grid_t g;
  memset(&g, 0, sizeof g);
  if (prm->use_cells) grid_build(&g, D, prm->h, y, n);
  pass1_t *P1 = (pass1_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(pass1_t));
  int nthr = nthreads_of(prm);
  int bad = 0;
  const int64_t nout = targets ? nt : n;
  char *need1 = NULL;
  if (targets) {
    need1 = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t *buf = NULL, cap = 0;
    for (int64_t ti = 0; ti < nt; ++ti) {
      int64_t cnt = neighbours(prm, &g, y, n, targets[ti], &buf, &cap);
      for (int64_t j = 0; j < cnt; ++j) need1[buf[j]] = 1;
      need1[targets[ti]] = 1;
    }
    free(buf);
  }

  /* ---- pass 1: density sums, EoS, transport, dissipative tensors ---- */
#pragma omp parallel num_threads(nthr) reduction(+:bad)
  {
    int64_t *buf = NULL, cap = 0;
#pragma omp for schedule(dynamic, 64)
    for (int64_t a = 0; a < n; ++a) {
      if (need1 && !need1[a]) continue;
      pass1_t *q = &P1[a];
      int64_t cnt = neighbours(prm, &g, y, n, a, &buf, &cap);
      double ss = 0.0, st = 0.0, nt[3] = {0.0, 0.0, 0.0};
      for (int64_t j = 0; j < cnt; ++j) {
        int64_t b = buf[j];
        double W = orc_kernel_w(D, prm->h, sqrt(dist2(D, y, n, a, b)));
        ss += W;
        st += y[V_S * n + b] * W;
        for (int k = 0; k < prm->ncharge; ++k) nt[k] += y[(V_NB + k) * n + b] * W;
      }
      q->nnb = (int)cnt;
      q->u[0] = 0.0;
      for (int k = 1; k < 4; ++k) q->u[k] = (k <= D) ? y[(V_U1 + k - 1) * n + a] : 0.0;
      q->gam = gamma_of(&m, q->u);
      q->u[0] = q->gam;
      for (int k = 0; k < 4; ++k) q->v[k] = q->u[k] / q->gam;
      double norm = q->gam * m.sqrtg;
      q->sigstar = ss;
      double sigma = ss / norm;
      if (prm->density_mode == 0) {
        q->s = st / norm;
        for (int k = 0; k < 3; ++k) q->n[k] = nt[k] / norm;
      } else {
        q->s = y[V_S * n + a] * sigma;
        for (int k = 0; k < 3; ++k) q->n[k] = k < prm->ncharge ? y[(V_NB + k) * n + a] * sigma : 0.0;
      }
      double in[4] = {q->s, q->n[0], q->n[1], q->n[2]};
      thermo_of_sn(eos, prm->ncharge, in, &q->th);
      if (!q->th.ok) bad++;
      double w = q->th.e + q->th.p;
      q->eta = prm->eta_over_s * q->s;
      double dT = q->th.T - prm->zeta_Tpeak;
      q->zeta = prm->zeta_width > 0.0
                  ? q->s * prm->zeta_peak * exp(-dT * dT / (2.0 * prm->zeta_width * prm->zeta_width))
                  : 0.0;
      q->taupi = prm->taupi_coeff * q->eta / w;
      q->tauPi = prm->tauPi_ratio * q->taupi;
      memset(q->pi, 0, sizeof q->pi);
      q->Pi = 0.0;
      if (prm->viscous) {
        q->Pi = sigma * y[V_B * n + a];
        static const int rows[4][4] = {
          {-1, -1, -1, -1}, {-1, V_P11, V_P12, V_P13}, {-1, V_P12, V_P22, V_P23}, {-1, V_P13, V_P23, V_P33}};
        for (int i = 1; i < 4; ++i)
          for (int j = 1; j < 4; ++j) q->pi[i][j] = sigma * y[rows[i][j] * n + a];
        for (int i = 1; i < 4; ++i) {
          double acc = 0.0;
          for (int j = 1; j < 4; ++j) acc += m.G[j] * q->u[j] * q->pi[j][i];
          q->pi[0][i] = q->pi[i][0] = acc / q->gam;
        }
        double acc = 0.0;
        for (int i = 1; i < 4; ++i) acc += m.G[i] * q->u[i] * q->pi[0][i];
        q->pi[0][0] = acc / q->gam;
      }
      double s2 = ss * ss;
      q->ppi_over_s2 = (q->th.p + q->Pi) / s2;
      for (int j = 0; j < 4; ++j)
        for (int i = 0; i < 4; ++i) q->A_over_s2[j][i] = (q->pi[j][i] - q->v[j] * q->pi[0][i]) / s2;
      memset(q->J, 0, sizeof q->J);
      memset(q->F_over_s2, 0, sizeof q->F_over_s2);
      for (int c = 0; c < 3; ++c) q->alpha[c] = 0.0;
      if (prm->diffusion) {
        for (int c = 0; c < 3; ++c) {
          double J0 = 0.0;
          for (int k = 1; k <= D; ++k) {
            q->J[c][k] = sigma * y[(V_JB1 + 3 * c + k - 1) * n + a];
            J0 += m.G[k] * q->u[k] * q->J[c][k];
          }
          q->J[c][0] = J0 / q->gam;
          for (int k = 1; k <= D; ++k) q->F_over_s2[c][k] = (q->J[c][k] - q->v[k] * q->J[c][0]) / s2;
          q->alpha[c] = q->th.mu[c] / q->th.T;
        }
      }
    }
    free(buf);
  }

  /* ---- pass 2: gradient sums, then the local EoM solve ---- */
#pragma omp parallel num_threads(nthr)
  {
    int64_t *buf = NULL, cap = 0;
#pragma omp for schedule(dynamic, 64)
    for (int64_t oi = 0; oi < nout; ++oi) {
      const int64_t a = targets ? targets[oi] : oi;
      const pass1_t *qa = &P1[a];
      int64_t cnt = neighbours(prm, &g, y, n, a, &buf, &cap);
      double F[4] = {0, 0, 0, 0}, dudx[4][4], divv = 0.0, de[4] = {0, 0, 0, 0};
      double dal[3][4], divF[3] = {0, 0, 0}, dPi[4] = {0, 0, 0, 0};
      memset(dudx, 0, sizeof dudx);
      memset(dal, 0, sizeof dal);
      for (int64_t j = 0; j < cnt; ++j) {
        int64_t b = buf[j];
        const pass1_t *qb = &P1[b];
        double r = sqrt(dist2(D, y, n, a, b));
        double f = orc_kernel_dw_over_r(D, prm->h, r);
        double dW[4] = {0, 0, 0, 0};
        for (int k = 1; k <= D; ++k) dW[k] = f * (y[(V_X1 + k - 1) * n + a] - y[(V_X1 + k - 1) * n + b]);
        double pp = qa->ppi_over_s2 + qb->ppi_over_s2;
        for (int i = 1; i <= D; ++i) {
          double vis = 0.0;
          for (int jj = 1; jj <= D; ++jj) vis += (qa->A_over_s2[jj][i] + qb->A_over_s2[jj][i]) * dW[jj];
          F[i] += pp * dW[i] + m.G[i] * vis;
        }
        for (int k = 1; k <= D; ++k) {
          for (int nu = 1; nu <= D; ++nu) dudx[k][nu] += (qb->u[nu] - qa->u[nu]) * dW[k];
          divv += (qb->v[k] - qa->v[k]) * dW[k];
          de[k] += (qb->th.e - qa->th.e) * dW[k];
        }
        if (prm->diffusion) {
          for (int k = 1; k <= D; ++k) dPi[k] += (qb->Pi - qa->Pi) * dW[k];
          for (int c = 0; c < 3; ++c)
            for (int k = 1; k <= D; ++k) {
              dal[c][k] += (qb->alpha[c] - qa->alpha[c]) * dW[k];
              divF[c] += (qa->F_over_s2[c][k] + qb->F_over_s2[c][k]) * dW[k];
            }
        }
      }
      pctx c;
      memset(&c, 0, sizeof c);
      c.D = D;
      c.viscous = prm->viscous;
      c.m = m;
      for (int k = 0; k < 4; ++k) { c.u[k] = qa->u[k]; c.v[k] = qa->v[k]; }
      for (int k = 1; k <= D; ++k)
        for (int nu = 1; nu <= D; ++nu) c.dudx[k][nu] = dudx[k][nu] / qa->sigstar;
      for (int k = 1; k < 4; ++k) {
        double acc = 0.0;
        for (int j = 1; j < 4; ++j) acc += m.G[j] * c.u[j] * c.dudx[k][j];
        c.dudx[k][0] = acc / c.u[0];
      }
      c.divv = divv / qa->sigstar;
      for (int i = 1; i <= D; ++i) c.F[i] = F[i];
      c.sigma = qa->sigstar / (qa->gam * m.sqrtg);
      c.w = qa->th.e + qa->th.p;
      c.p = qa->th.p;
      c.Pi = qa->Pi;
      c.T = qa->th.T;
      c.cs2 = qa->th.cs2;
      c.kappa = qa->th.kappa;
      c.eta = qa->eta;
      c.zeta = qa->zeta;
      c.taupi = qa->taupi;
      c.tauPi = qa->tauPi;
      memcpy(c.pi, qa->pi, sizeof c.pi);
      for (int i = 1; i < 4; ++i)
        for (int j = 1; j < 4; ++j) c.P[i][j] = qa->pi[i][j] / c.sigma;
      c.cPiPi = prm->c_PiPi;
      c.cPipi = prm->c_Pipi;
      c.cpipi = prm->c_pipi;
      c.cpiPi = prm->c_piPi;
      c.cpisig = prm->c_pisig;
      sources_at(prm, &m, t, y, n, a, c.I, c.Iq);
      for (int q = 0; q < 3; ++q) {
        c.mu[q] = q < prm->ncharge ? qa->th.mu[q] : 0.0;
        if (q >= prm->ncharge) c.Iq[q] = 0.0;
      }
      c.diffusion = prm->diffusion;
      if (prm->diffusion) {
        memcpy(c.J, qa->J, sizeof c.J);
        for (int q = 0; q < 3; ++q) {
          for (int k = 1; k <= D; ++k) {
            c.V[q][k] = y[(V_JB1 + 3 * q + k - 1) * n + a];
            c.dalpha[q][k] = dal[q][k] / qa->sigstar;
          }
          c.divF[q] = divF[q];
          for (int r = 0; r < 3; ++r) c.kapJ[q][r] = prm->kappa_T2[3 * q + r] * qa->th.T * qa->th.T;
        }
        c.tauJ = prm->tauJ_coeff / qa->th.T;
        c.cJJ = prm->c_JJ;
        for (int k = 1; k <= D; ++k) c.dPi[k] = dPi[k] / qa->sigstar;
        for (int r = 0; r < 3; ++r) c.dJPi[r] = prm->d_JPi[r];
      }

      double zero[4] = {0, 0, 0, 0}, M[4][4], rhs[4], acc_u[4] = {0, 0, 0, 0};
      pout o0, oj;
      eom_eval(&c, zero, &o0);
      for (int j = 1; j <= D; ++j) {
        double ej[4] = {0, 0, 0, 0};
        ej[j] = 1.0;
        eom_eval(&c, ej, &oj);
        for (int i = 1; i <= D; ++i) M[i - 1][j - 1] = oj.R[i] - o0.R[i];
      }
      for (int i = 1; i <= D; ++i) rhs[i - 1] = -o0.R[i];
      double sol[4] = {0, 0, 0, 0};
      solve_n(D, M, rhs, sol);
      for (int i = 1; i <= D; ++i) acc_u[i] = sol[i - 1];
      pout o;
      eom_eval(&c, acc_u, &o);

      for (int v = 0; v < NVAR; ++v) dydt[v * nout + oi] = 0.0;
      for (int k = 1; k <= D; ++k) {
        dydt[(V_X1 + k - 1) * nout + oi] = c.v[k];
        dydt[(V_U1 + k - 1) * nout + oi] = acc_u[k];
      }
      dydt[V_S * nout + oi] = o.dS;
      for (int q = 0; q < prm->ncharge; ++q) dydt[(V_NB + q) * nout + oi] = o.dN[q];
      if (prm->viscous) {
        dydt[V_B * nout + oi] = o.dB;
        dydt[V_P11 * nout + oi] = o.dP[1][1];
        dydt[V_P12 * nout + oi] = o.dP[1][2];
        dydt[V_P13 * nout + oi] = o.dP[1][3];
        dydt[V_P22 * nout + oi] = o.dP[2][2];
        dydt[V_P23 * nout + oi] = o.dP[2][3];
        dydt[V_P33 * nout + oi] = o.dP[3][3];
      }
      if (prm->diffusion)
        for (int q = 0; q < 3; ++q)
          for (int k = 1; k <= D; ++k) dydt[(V_JB1 + 3 * q + k - 1) * nout + oi] = o.dV[q][k];
      if (aux) {
        aux[A_SIGSTAR * nout + oi] = qa->sigstar;
        aux[A_S * nout + oi] = qa->s;
        for (int k = 0; k < 3; ++k) aux[(A_NB + k) * nout + oi] = qa->n[k];
        aux[A_T * nout + oi] = qa->th.T;
        for (int k = 0; k < 3; ++k) aux[(A_MUB + k) * nout + oi] = qa->th.mu[k];
        aux[A_P * nout + oi] = qa->th.p;
        aux[A_E * nout + oi] = qa->th.e;
        aux[A_CS2 * nout + oi] = qa->th.cs2;
        aux[A_INTABLE * nout + oi] = qa->th.in_table;
        aux[A_GAMMA * nout + oi] = qa->gam;
        aux[A_THETA * nout + oi] = o.theta;
        aux[A_NNB * nout + oi] = qa->nnb;
        for (int i = 1; i <= 3; ++i) aux[(A_F1 + i - 1) * nout + oi] = F[i];
        /* Knudsen and inverse Reynolds numbers ("Particlization", eq.
         * knudsen-reynolds): Kn_pi = tau_pi sqrt(sigma:sigma), Re^-1_pi =
         * sqrt(pi:pi)/p, Kn_Pi = tau_Pi theta, Re^-1_Pi = |Pi|/p; zero for
         * ideal runs */
        double pipi = 0.0;
        for (int mu = 0; mu < 4; ++mu)
          for (int nu = 0; nu < 4; ++nu) pipi += qa->pi[mu][nu] * m.g[mu] * m.g[nu] * qa->pi[mu][nu];
        const int vis = prm->viscous;
        aux[A_KN_SHEAR * nout + oi] = vis ? qa->taupi * sqrt(fabs(o.sigsig)) : 0.0;
        aux[A_REINV_SHEAR * nout + oi] = vis ? sqrt(fabs(pipi)) / qa->th.p : 0.0;
        aux[A_KN_BULK * nout + oi] = vis ? qa->tauPi * o.theta : 0.0;
        aux[A_REINV_BULK * nout + oi] = vis ? fabs(qa->Pi) / qa->th.p : 0.0;
        /* Freeze-out surface element ("Freeze-out hypersurface construction"):
         * spatial d_i e in the n = 1 difference form, d_0 e from the energy
         * equation D e = -(e + p + Pi) theta + pi:sigma + u.I with
         * D = gamma d_0 + u^i d_i; normal n_mu = -d_mu e / sqrt(|d e . d e|),
         * |d sigma| = m / (sigma |u^mu n_mu|) with m = 1, d sigma_mu =
         * |d sigma| n_mu (all zero where the normal is undefined) */
        double dmu[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = 1; k <= D; ++k) dmu[k] = de[k] / qa->sigstar;
        double uI = 0.0;
        for (int mu = 0; mu < 4; ++mu) uI += m.g[mu] * c.u[mu] * c.I[mu];
        const double De = -(qa->th.e + qa->th.p + (prm->viscous ? qa->Pi : 0.0)) * o.theta
                        + (prm->viscous ? o.pisig : 0.0) + uI;
        double adv = 0.0;
        for (int k = 1; k <= D; ++k) adv += c.u[k] * dmu[k];
        dmu[0] = (De - adv) / c.u[0];
        double nn = 0.0;
        for (int mu = 0; mu < 4; ++mu) nn += m.ginv[mu] * dmu[mu] * dmu[mu];
        const double norm = sqrt(fabs(nn));
        double nl[4] = {0.0, 0.0, 0.0, 0.0}, un = 0.0;
        if (norm > 0.0)
          for (int mu = 0; mu < 4; ++mu) {
            nl[mu] = -dmu[mu] / norm;
            un += c.u[mu] * nl[mu];
          }
        const double dsig = (norm > 0.0 && fabs(un) > 0.0) ? 1.0 / (c.sigma * fabs(un)) : 0.0;
        for (int mu = 0; mu < 4; ++mu) {
          aux[(A_DE0 + mu) * nout + oi] = dmu[mu];
          aux[(A_DSIG0 + mu) * nout + oi] = dsig * nl[mu];
        }
      }
    }
    free(buf);
  }
  free(P1);
  free(need1);
  if (prm->use_cells) grid_free(&g);
  return bad;
}

int orc_rhs(const orc_params *prm, const orc_eos *eos, double t, int64_t n,
            const double *y, double *dydt, double *aux)
{
  return rhs_impl(prm, eos, t, n, y, 0, NULL, dydt, aux);
}

int orc_rhs_targets(const orc_params *prm, const orc_eos *eos, double t, int64_t n, const double *y,
                    int64_t nt, const int64_t *targets, double *dydt, double *aux)
{
  return rhs_impl(prm, eos, t, n, y, nt, targets, dydt, aux);
}

/* Heun (second-order Runge-Kutta) step, the reading of the paper's
 * unspecified "integration method":
 *   y1 = y0 + dt f(t, y0),  y = (y0 + y1 + dt f(t + dt, y1)) / 2.        */
int orc_heun_step(const orc_params *prm, const orc_eos *eos, double t, double dt, int64_t n,
                  double *y, double *aux)
{
  size_t sz = sizeof(double) * (size_t)NVAR * (size_t)(n > 0 ? n : 1);
  double *k = (double *)malloc(sz), *y1 = (double *)malloc(sz);
  int bad = orc_rhs(prm, eos, t, n, y, k, NULL);
  for (int64_t i = 0; i < (int64_t)NVAR * n; ++i) y1[i] = y[i] + dt * k[i];
  bad += orc_rhs(prm, eos, t + dt, n, y1, k, aux);
  for (int64_t i = 0; i < (int64_t)NVAR * n; ++i) y[i] = 0.5 * (y[i] + y1[i] + dt * k[i]);
  free(k);
  free(y1);
  return bad;
}

/* Initialisation from intensive densities at x0 = t0 (reading of the
 * particle-mass choice m_b = 1): sigma*_a = sum_b W_ab, then
 * S_a = s_a gamma_a sqrt(-g) / sigma*_a and N_a likewise; Pi = pi = 0.
 * dens rows: (s or e, nB, nS, nQ); dens_kind 0 = s, 1 = e. */
int orc_init(const orc_params *prm, const orc_eos *eos, double t0, int64_t n,
             const double *xi, const double *u, int dens_kind, const double *dens, double *y)
{
  const int D = prm->dim;
  geom m;
  geom_at(prm->hyperbolic, t0, &m);
  for (int64_t i = 0; i < (int64_t)NVAR * n; ++i) y[i] = 0.0;
  for (int k = 0; k < D; ++k)
    for (int64_t a = 0; a < n; ++a) {
      y[(V_X1 + k) * n + a] = xi[k * n + a];
      y[(V_U1 + k) * n + a] = u[k * n + a];
    }
  grid_t g;
  memset(&g, 0, sizeof g);
  if (prm->use_cells) grid_build(&g, D, prm->h, y, n);
  int bad = 0;
#pragma omp parallel reduction(+:bad)
  {
    int64_t *buf = NULL, cap = 0;
#pragma omp for schedule(dynamic, 64)
    for (int64_t a = 0; a < n; ++a) {
      int64_t cnt = neighbours(prm, &g, y, n, a, &buf, &cap);
      double ss = 0.0;
      for (int64_t j = 0; j < cnt; ++j) ss += orc_kernel_w(D, prm->h, sqrt(dist2(D, y, n, a, buf[j])));
      double uu[4] = {0, 0, 0, 0};
      for (int k = 1; k <= D; ++k) uu[k] = y[(V_U1 + k - 1) * n + a];
      double gam = gamma_of(&m, uu);
      double in[4] = {dens[a], dens[n + a], dens[2 * n + a], dens[3 * n + a]};
      double s = in[0];
      if (dens_kind == 1) {
        thermo th;
        invert(eos, 1, prm->ncharge, in, &th);
        if (!th.ok) bad++;
        s = th.s;
      }
      double fac = gam * m.sqrtg / ss;
      y[V_S * n + a] = s * fac;
      for (int k = 0; k < prm->ncharge; ++k) y[(V_NB + k) * n + a] = in[1 + k] * fac;
    }
    free(buf);
  }
  if (prm->use_cells) grid_free(&g);
  return bad;
}

/* Per-event totals: S, NB, NS, NQ, E, M1, M2, M3 (charges as conserved with
 * diffusion, N_q + sqrt(-g) J^0_q / sigma*) where
 *   E   = sum_a sqrt(-g) T^{00}_a / sigma*_a,
 *   M_i = sum_a sqrt(-g) G_i T^{0i}_a / sigma*_a.
 * In Cartesian coordinates E and M_i are the conserved energy and momentum. */
void orc_totals(const orc_params *prm, const orc_eos *eos, double t, int64_t n, const double *y,
                double *out)
{
  double *aux = (double *)malloc(sizeof(double) * NAUX * (size_t)(n > 0 ? n : 1));
  double *dy = (double *)malloc(sizeof(double) * NVAR * (size_t)(n > 0 ? n : 1));
  orc_rhs(prm, eos, t, n, y, dy, aux);
  geom m;
  geom_at(prm->hyperbolic, t, &m);
  for (int k = 0; k < 8; ++k) out[k] = 0.0;
  for (int64_t a = 0; a < n; ++a) {
    out[0] += y[V_S * n + a];
    double u[4] = {0, 0, 0, 0};
    for (int k = 1; k <= prm->dim; ++k) u[k] = y[(V_U1 + k - 1) * n + a];
    double gam = gamma_of(&m, u);
    u[0] = gam;
    /* charge of a particle: N_q, plus sqrt(-g) J^0_q / sigma* with diffusion */
    for (int q = 0; q < 3; ++q) {
      double Nq = y[(V_NB + q) * n + a];
      if (prm->diffusion) {
        double X = 0.0;
        for (int k = 1; k <= prm->dim; ++k) X += m.G[k] * u[k] * y[(V_JB1 + 3 * q + k - 1) * n + a];
        Nq += X / (gam * gam);
      }
      out[1 + q] += Nq;
    }
    double sigstar = aux[A_SIGSTAR * n + a];
    double sigma = sigstar / (gam * m.sqrtg);
    double p = aux[A_P * n + a], w = aux[A_E * n + a] + p;
    double Pi = prm->viscous ? sigma * y[V_B * n + a] : 0.0;
    double pi[4][4];
    memset(pi, 0, sizeof pi);
    if (prm->viscous) {
      static const int rows[4][4] = {
        {-1, -1, -1, -1}, {-1, V_P11, V_P12, V_P13}, {-1, V_P12, V_P22, V_P23}, {-1, V_P13, V_P23, V_P33}};
      for (int i = 1; i < 4; ++i)
        for (int j = 1; j < 4; ++j) pi[i][j] = sigma * y[rows[i][j] * n + a];
      for (int i = 1; i < 4; ++i) {
        double acc = 0.0;
        for (int j = 1; j < 4; ++j) acc += m.G[j] * u[j] * pi[j][i];
        pi[0][i] = acc / gam;
      }
      double acc = 0.0;
      for (int i = 1; i < 4; ++i) acc += m.G[i] * u[i] * pi[0][i];
      pi[0][0] = acc / gam;
    }
    double T00 = (w + Pi) * gam * gam - (p + Pi) + pi[0][0];
    out[4] += m.sqrtg * T00 / sigstar;
    for (int i = 1; i <= 3; ++i) {
      double T0i = (w + Pi) * gam * u[i] + pi[0][i];
      out[4 + i] += m.sqrtg * m.G[i] * T0i / sigstar;
    }
  }
  free(aux);
  free(dy);
}

int orc_nvar(void) { return NVAR; }
int orc_naux(void) { return NAUX; }

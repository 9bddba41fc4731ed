// Shared device/host definitions of the CCAKE SPH library (gfx950).
//
// Layout conventions
//   * particle state: 26 rows of FP64, row-major [row][capacity], particles of
//     one event contiguous and, after binning, sorted by (cell, id);
//   * rows: x^1..x^3, u^1..u^3, S = s/sigma, N_B, N_S, N_Q (= n_q/sigma),
//     B = Pi/sigma, P^{ij} = pi^{ij}/sigma for ij = 11,12,13,22,23,33,
//     V^k_q = J^k_q/sigma (charge diffusion currents, q = B,S,Q, k = 1..3)
//     (the dynamical variables of the paper's SPH equations of motion);
//   * the index 3 is eta (hyperbolic) or z (Cartesian); in 2+1D it is a
//     symmetry direction (u^3 = 0, no particle coordinate).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccake {

enum Row {
  R_X1, R_X2, R_X3, R_U1, R_U2, R_U3, R_S, R_NB, R_NS, R_NQ, R_B,
  R_P11, R_P12, R_P13, R_P22, R_P23, R_P33,
  R_JB1, R_JB2, R_JB3, R_JS1, R_JS2, R_JS3, R_JQ1, R_JQ2, R_JQ3, NROW
};

// auxiliary per-particle outputs of a right-hand-side evaluation (debug/parity)
enum Aux {
  X_SIGSTAR, X_S, X_NB, X_NS, X_NQ, X_T, X_MUB, X_MUS, X_MUQ, X_P, X_E,
  X_CS2, X_INTABLE, X_GAMMA, X_THETA, X_NNB, X_F1, X_F2, X_F3, X_NEWTON, X_EOS_EVALS,
  X_KN_SHEAR, X_REINV_SHEAR, X_KN_BULK, X_REINV_BULK, X_DE0, X_DE1, X_DE2, X_DE3, X_DSIG0, X_DSIG1,
  X_DSIG2, X_DSIG3, NAUXROW
};

// per-particle thermodynamic record written by pass 1, read (own particle) by pass 2
enum Th {
  T_SIGSTAR, T_T, T_MUB, T_MUS, T_MUQ, T_P, T_E, T_CS2, T_KAP, T_PI,
  T_ETA, T_ZETA, T_TAUPI, T_TAUPIB, T_S, T_NB, T_NS, T_NQ, T_NNB, NTH
};

// neighbour record written by pass 1, read for every neighbour by pass 2:
// (p+Pi)/sigma*^2, A^{ji}/sigma*^2 (j,i spatial, row-major j*3+i), u^k, v^k
enum Rec { Q_PP, Q_A11, Q_A12, Q_A13, Q_A21, Q_A22, Q_A23, Q_A31, Q_A32, Q_A33,
           Q_U1, Q_U2, Q_U3, Q_V1, Q_V2, Q_V3, NREC };

// neighbour record of the diffusion sums (FP64, written by pass 1):
// alpha_q = mu_q/T and F^k_q/sigma*^2 with F = J - v J^0 (row QD_FB1 + 3q + k-1), and Pi
enum DRec { QD_AB, QD_AS, QD_AQ, QD_FB1, QD_FB2, QD_FB3, QD_FS1, QD_FS2, QD_FS3, QD_FQ1, QD_FQ2, QD_FQ3, QD_PI, NDREC };

// record carried with the particle from step to step: the warm start of the
// EoS inversion (the last root of the analytic backup EoS and, when the table
// answered, the last root of the table interpolant; W_TT = 0 when there is
// none), then the freeze-out bookkeeping (the energy density at the last step
// start, and 1 once the particle has crossed e_fo)
enum Warm { W_GT, W_GMUB, W_GMUS, W_GMUQ, W_TT, W_TMUB, W_TMUS, W_TMUQ, NWARM_EOS,
            W_EPREV = NWARM_EOS, W_FROZEN, NWARM };

// freeze-out surface record ("Freeze-out hypersurface construction"): original
// id, crossing time, position at the crossing, u^i, T, mu_q and d sigma_mu at
// the recording step
enum FoCol { FO_ID, FO_T, FO_X1, FO_X2, FO_X3, FO_U1, FO_U2, FO_U3, FO_TEMP, FO_MUB, FO_MUS, FO_MUQ,
             FO_DS0, FO_DS1, FO_DS2, FO_DS3, FO_NCOL };

// density sums of a particle (lab frame, kernel normalisation applied) and its neighbour count
enum DSum { DS_SIG, DS_S, DS_NB, DS_NS, DS_NQ, DS_NNB, NDSUM };

// gradient sums of a particle: force F_i, d_k u^j (row-major k*3+j, divided by sigma*), div v,
// d_i e (freeze-out), and with diffusion d_k alpha_q (row GS_DAB1 + 3q + k-1, divided by
// sigma*) and the flux sums sum_b (F_a/sigma*_a^2 + F_b/sigma*_b^2) . grad W (GS_DJB + q);
// d_k Pi (GS_DPI1 + k-1, divided by sigma*)
enum GSum { GS_F1, GS_F2, GS_F3, GS_DU11, GS_DU12, GS_DU13, GS_DU21, GS_DU22, GS_DU23, GS_DU31, GS_DU32,
            GS_DU33, GS_DIVV, GS_DE1, GS_DE2, GS_DE3,
            GS_DAB1, GS_DAB2, GS_DAB3, GS_DAS1, GS_DAS2, GS_DAS3, GS_DAQ1, GS_DAQ2, GS_DAQ3,
            GS_DJB, GS_DJS, GS_DJQ, GS_DPI1, GS_DPI2, GS_DPI3, NGSUM };

enum EosKind { EOS_CONFORMAL = 0, EOS_TABLE = 1, EOS_GAS = 2 };

// table node: 8 doubles, the four Newton columns first (32-byte aligned)
enum TabCol { TC_S, TC_NB, TC_NS, TC_NQ, TC_P, TC_CS2, TC_KAP, TC_PAD, TC_STRIDE };

// Offline inverted table ("EoS inverter", offline option): thermodynamics
// at nodes s = 10^d (1 + 9 m / P) (decades d0 <= d < d1, then 10^d1) times
// x_q = n_q / s on uniform grids; val == nullptr: no table.
enum InvCol { IV_T, IV_MUB, IV_MUS, IV_MUQ, IV_P, IV_E, IV_CS2, IV_KAP, IV_TAB, IV_STRIDE };
struct InvDev {
  const double* val;  // [ns][nx_B][nx_S][nx_Q][IV_STRIDE]
  int32_t ncharge, d0, d1, P;
  int32_t nx[3], pad;
  int64_t ns;
  double xlo[3], xhi[3];
};

struct EosDev {
  int32_t kind;
  int32_t n[4];
  int32_t max_iter;
  double lo[4], hi[4], d[4], inv_d[4];  // axis origin, end, spacing, 1/spacing
  double fstar;
  double tol;
  const double* tab;  // node-major [nT][nB][nS][nQ][8]
  InvDev inv;         // offline table of the (s, n) inversions of the stages
};

// one external source, widths folded into 1/(2 w^2) and the normalisation of
// the Gaussian over the dim axes
struct SourceDev {
  double c0[3], vel[3], iw2[3];
  double norm;
  double t_on, t_off;
  double dpdt[4], dndt[3];
};

constexpr int MAX_SOURCES = 16;

struct SourceSet {
  int32_t n, pad;
  SourceDev s[MAX_SOURCES];
};

// cells per kernel support along an axis (2+1D, 3+1D): the grid cell edge is
// (2h + skin) / subcells and a particle's candidates lie within subcells
// cells per axis; finer cells cut the candidate rows closer to the ball
#ifndef CCAKE_SUBCELLS2
#define CCAKE_SUBCELLS2 2
#endif
#ifndef CCAKE_SUBCELLS3
#define CCAKE_SUBCELLS3 2
#endif
// Entries per target of the skin lists (2D, 3D; 0: no lists): about six
// times the mean neighbour count of the 3D benchmark events; a target with
// more falls back to the candidate walk.  In 2D the candidate walk accepts
// most of what it reads and writing the lists costs the density pass more
// than the other passes save.
#ifndef CCAKE_LIST_CAP2
#define CCAKE_LIST_CAP2 0
#endif
#ifndef CCAKE_LIST_CAP3
#define CCAKE_LIST_CAP3 4096
#endif
__host__ __device__ constexpr int list_cap(int dim) { return dim == 3 ? CCAKE_LIST_CAP3 : CCAKE_LIST_CAP2; }
__host__ __device__ constexpr int subcells(int dim) { return dim == 3 ? CCAKE_SUBCELLS3 : CCAKE_SUBCELLS2; }
__host__ __device__ constexpr int row_count(int dim) {
  return dim == 3 ? (2 * subcells(3) + 1) * (2 * subcells(3) + 1) : 2 * subcells(2) + 1;
}
// the first and last candidate slots of a particle's neighbour rows
// (row_count(dim) rows), searched by each binning at the binning-time
// positions and used until the next binning
constexpr int ROW_CACHE = 2 * (row_count(3) > row_count(2) ? row_count(3) : row_count(2));

struct Params {
  int32_t dim, hyperbolic, viscous, ncharge, density_mode, mixed;
  double h;
  double eta_over_s, zeta_peak, zeta_Tpeak, zeta_width;
  double taupi_coeff, tauPi_ratio;
  double c_PiPi, c_Pipi, c_pipi, c_piPi;
  int32_t diffusion, pad_d;
  double kappa_T2[9]; // kappa_{qq'}/T^2, row-major (diffusion)
  double tauJ_coeff;  // tau_J = tauJ_coeff / T
  double c_JJ;        // coefficient of -tau_J J theta
  double c_pisig;     // coefficient of the ADNH shear term pi_lambda^<i sigma^j>lambda
  double d_JPi[3];    // delta_JPi^q / beta: currents coupled to nabla Pi (diffusion)
  double cell_edge;   // >= 2h + skin
  double e_fo;        // freeze-out energy density (fm^-4); 0: no surface
  const SourceSet* src = nullptr;  // external sources (device), or none
};

// one event of a batch (device-resident table)
struct EventDev {
  int64_t p_base;     // first particle slot
  int64_t c_base;     // first cell slot
  int32_t n;          // particles
  int32_t c_cap;      // cell capacity
  int32_t nc[3];      // grid cells per axis (this step)
  int32_t active;
  double lo[3];       // grid origin (this step)
  double edge;        // cell edge (this step, >= cell_edge)
  double t;           // current x^0
  double t_prev;      // x^0 at the start of the previous step
  double dt;          // step size
  uint32_t nonfinite; // count of non-finite state updates (sticky)
  uint32_t noconv;    // count of EoS inversions that failed (sticky)
  uint32_t backup;    // EoS inversions served by the analytic backup (last stage)
  int32_t first_bad;  // lowest original id with a non-finite update, or -1
  uint32_t capacity_err;
  uint32_t newton_iters; // total Newton iterations (last stage)
  int32_t rebin;      // this step bins the event (else it keeps its cells and order)
  int32_t need_bin;   // the next step must bin (fresh state)
  int32_t tile0;      // first workgroup of the event in the pair kernels' grid
  int32_t pad_t;
  double disp;        // displacement bound sum(dt max(1, 1/x0)) since the last binning
  // bounding-box accumulators of the next binning: order-preserving integer
  // images of the coordinates (reset to the empty box after every use)
  unsigned long long bb_min[3], bb_max[3];
};

// order-preserving map double -> unsigned 64-bit (for atomic min / max)
__host__ __device__ inline unsigned long long ordered_bits(double d) {
  union {
    double d;
    unsigned long long u;
  } v;
  v.d = d;
  return (v.u & 0x8000000000000000ull) ? ~v.u : (v.u | 0x8000000000000000ull);
}
__host__ __device__ inline double from_ordered_bits(unsigned long long u) {
  union {
    double d;
    unsigned long long u;
  } v;
  v.u = (u & 0x8000000000000000ull) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
  return v.d;
}
constexpr unsigned long long BB_EMPTY_MIN = 0xFFFFFFFFFFFFFFFFull;
constexpr unsigned long long BB_EMPTY_MAX = 0ull;

// device arrays of a batch (pointers into one workspace)
struct BatchDev {
  double* Y0;        // home state [NROW][cap]
  double* Ys;        // sorted step-start state [NROW][cap]
  double* Y1;        // stage state [NROW][cap]
  double* th;        // [NTH][cap]
  double* rec;       // [NREC][cap] fp64 neighbour records
  float* recf;       // [NREC][cap] fp32 neighbour records (mixed precision)
  double* drec;      // [NDREC][cap] fp64 neighbour records of the diffusion sums
  double* warm;      // home warm start [NWARM][cap]
  double* warms;     // sorted warm start [NWARM][cap]
  double* dsum;      // [NDSUM][cap] density sums (sorted order)
  double* gsum;      // [NGSUM][cap] gradient sums (sorted order)
  int32_t* id;       // home original ids
  int32_t* ids;      // sorted original ids
  int32_t* ev;       // event of each slot (-1 = empty)
  int32_t* key;      // local cell key (home order)
  int32_t* keys;     // local cell key (sorted order)
  int32_t* perm;     // sorted slot -> home slot
  double* xbin;      // x^1 of each slot at its event's last binning (sorted order)
  int32_t* rows;     // [ROW_CACHE][cap] row bounds (lo, hi per row), written by each binning
  double* fo_rec;    // [cap][FO_NCOL] freeze-out records, in the order found
  int32_t* fo_slot;  // [cap] sorted slot of each record's particle (step of its crossing)
  int32_t* fo_mark;  // [cap] per sorted slot: record found in this step's first stage, or -1
  uint32_t* fo_ctr;  // [2] records so far, records before this step
  uint16_t* slist;   // [cap][list_cap(dim)] skin list of each target: halo indices of its candidates within 2h + 2d at a step's first stage, in walk order
  int32_t* scnt;     // [cap] their number, or -1 when they do not fit (the passes walk the candidates)
  int32_t* cell_start;  // [ccap + 1] absolute slot of each cell
  int32_t* cell_fill;   // [ccap] counts / cursors
  EventDev* evt;     // [max_events]
  int64_t cap;       // particle slots
  int64_t ccap;      // cell slots
  int32_t max_events;
};

}  // namespace ccake

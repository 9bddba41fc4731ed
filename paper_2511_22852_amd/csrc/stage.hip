// One Runge-Kutta stage of the SPH update, as four kernels:
//
//   k_density  team of L lanes per particle: sigma*_a = sum_b W_ab and, for
//              the smoothed density form, s*_a = sum_b S_b W_ab and
//              n*_a = sum_b N_b W_ab ("SPH interpretation of a fluid element")
//   k_eos      one thread per particle: rest-frame densities, EoS inversion
//              (online inverter), transport coefficients, dissipative tensors,
//              the neighbour record of pass 2
//   k_grad     team of L lanes per particle: n = -1 force sums of p + Pi and
//              of the viscous tensor, n = 1 sums of d_k u^j and div v
//              ("Derivatives in relativistic SPH"); with BSQ diffusion also
//              d_k (mu/T) and the n = -1 flux sums of the currents
//   k_eom      one thread per particle: local M du/dx0 = F solve, relaxation
//              rates, Heun update
//
// The neighbour loops give each of L consecutive lanes every L-th candidate
// of the particle's trimmed cell rows and combine the partial sums in a fixed
// order through LDS (lane v adds value v of the team's lanes in lane order),
// so the result is deterministic.  Each lane
// takes its candidates U at a time (PairU): the positions of all U are
// loaded together, then the operands of the accepted ones, so that a lane has
// several loads in flight across row boundaries instead of one dependent
// round trip per candidate.  Candidates of particles in the same cell
// coincide, so the lanes of a wave read the same addresses.  In mixed precision the pair terms are formed and accumulated in
// FP32 with Kahan compensation per lane, and the lanes' partials are merged in FP64;
// the pair test itself is always the exact FP64 one.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "common.h"
#include "eom_device.h"
#include "eos_device.h"
#include "kernels.h"
#include "pair_device.h"
#include "sph_device.h"

namespace ccake {

// lanes per particle in the pair loops (2D, 3D)
#ifndef CCAKE_TEAM2
#define CCAKE_TEAM2 16
#endif
#ifndef CCAKE_TEAM3
#define CCAKE_TEAM3 16
#endif
template <int D>
struct Team {
  static constexpr int L = D == 2 ? CCAKE_TEAM2 : CCAKE_TEAM3;
  static constexpr int PER_BLOCK = 256 / L;
};
// candidates per lane in flight in the pair loops (2D, 3D; measured best:
// the 3D loops are longer and issue-bound, so more loads in flight pay)
#ifndef CCAKE_PAIR_U2
#define CCAKE_PAIR_U2 2
#endif
#ifndef CCAKE_PAIR_U3
#define CCAKE_PAIR_U3 4
#endif
template <int D>
struct PairU {
  static constexpr int U = D == 2 ? CCAKE_PAIR_U2 : CCAKE_PAIR_U3;
};

// Takes this lane's next U candidates from the cursor: slot k[u] and
// whether it exists (v[u]); missing ones point at the lane's own particle,
// so every load stays in bounds.
template <int U, class Cursor>
__device__ __forceinline__ void take(Cursor& cur, int32_t self, int32_t k[U], bool v[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    v[u] = cur.valid();
    k[u] = self;
    if (v[u]) k[u] = cur.next();
  }
}

// ---------------------------------------------------------------------------
// NS: smoothed scalars per neighbour (0 specific densities, 1 s*, 4 s* and n*)
template <int D, bool MIXED, int NS>
__global__ void __launch_bounds__(256) k_density(BatchDev b, Params prm, const double* __restrict__ Y,
                                                 int64_t nslots) {
  constexpr int L = Team<D>::L;
  constexpr int ROWS = RowBlock<D>::ROWS;
  __shared__ int32_t s_lo[Team<D>::PER_BLOCK][ROWS], s_hi[Team<D>::PER_BLOCK][ROWS];
  const int64_t tid = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t j = tid / L;
  const int lane = (int)(tid % L);
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0) return;
  const EventDev& E = b.evt[e];
  const int64_t cap = b.cap;
  const double h = prm.h, ih = 1.0 / h, r2max = (2.0 * h) * (2.0 * h);
  const double xa[3] = {row(Y, cap, R_X1, j), row(Y, cap, R_X2, j), D == 3 ? row(Y, cap, R_X3, j) : 0.0};
  const int team = (int)threadIdx.x / L;
  // rows found at the first pass after a binning, kept until the next
  // binning: a pair within 2h now was within 2h + skin then, because the
  // binning is redone before twice the displacement bound exceeds the skin
  if (b.rowstamp[j] == E.bin_serial) {
    rows_load<D, L>(b, j, lane, s_lo[team], s_hi[team]);
  } else {
    team_rows<D, L>(b, E, b.keys[j], xa, prm.cell_edge, lane, s_lo[team], s_hi[team]);
    rows_keep<D, L>(b, j, lane, s_lo[team], s_hi[team]);
    if (lane == 0) b.rowstamp[j] = E.bin_serial;
  }
  RowCursor<L, ROWS> cur;
  cur.start(s_lo[team], s_hi[team], lane);
  DensAcc<MIXED, NS> A;
  A.init();
  const int32_t self = (int32_t)j;
  constexpr int PAIR_U = PairU<D>::U;
  for (;;) {
    int32_t k[PAIR_U];
    bool v[PAIR_U];
    take<PAIR_U>(cur, self, k, v);
    if (!v[0]) break;
    double d2[PAIR_U];
    bool ok[PAIR_U];
#pragma unroll
    for (int u = 0; u < PAIR_U; ++u) {
      const double xb[3] = {row(Y, cap, R_X1, k[u]), row(Y, cap, R_X2, k[u]),
                            D == 3 ? row(Y, cap, R_X3, k[u]) : 0.0};
      d2[u] = dist2<D>(xa, xb);
      ok[u] = v[u] && d2[u] < r2max;
    }
#pragma unroll
    for (int u = 0; u < PAIR_U; ++u) {
      const int32_t m = ok[u] ? k[u] : self;
      double sc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) sc[q] = q < NS ? row(Y, cap, R_S + q, m) : 0.0;
      if (ok[u]) A.add(d2[u], ih, sc);
    }
    if (!v[PAIR_U - 1]) break;
  }
  // lane v < 6 forms row v of the density sums (sigma*, S, N_B, N_S, N_Q, count)
  __shared__ double s_red[Team<D>::PER_BLOCK][L * 6];
  double part[6];
  A.partials(part);
  const double tot = team_sums_lds<L, 6>(s_red[team], lane, part);
  if (lane < 6) b.dsum[(int64_t)(DS_SIG + lane) * b.cap + j] = lane == 5 ? tot : tot * sigma_d<D>(prm.h);
}

// ---------------------------------------------------------------------------
template <int D, bool VISC, bool MIXED, int NQ>
__device__ __forceinline__ void eos_particle(const BatchDev& b, const Params& prm, const EosDev& eos,
                                             const double* __restrict__ Y, int stage, int64_t j, int e, double* aux,
                                             uint32_t& c_backup, uint32_t& c_iters, uint32_t& c_noconv) {
  const EventDev& E = b.evt[e];
  const double t = E.t + stage * E.dt;
  const int64_t cap = b.cap;
  const bool smoothed = prm.density_mode == 0;
  const double ss = b.dsum[(int64_t)DS_SIG * cap + j];

  const double G3 = metric_G3(prm, t);
  double u[4] = {0.0, row(Y, cap, R_U1, j), row(Y, cap, R_U2, j), D == 3 ? row(Y, cap, R_U3, j) : 0.0};
  const double gam = sqrt(1.0 + u[1] * u[1] + u[2] * u[2] + G3 * u[3] * u[3]);
  u[0] = gam;
  const double norm = gam * sqrt_g(prm, t);
  const double sigma = ss / norm;
  double dens[4] = {0.0, 0.0, 0.0, 0.0};
  if (smoothed) {
    dens[0] = b.dsum[(int64_t)DS_S * cap + j] / norm;
    if (NQ)
      for (int q = 0; q < 3; ++q) dens[1 + q] = b.dsum[(int64_t)(DS_NB + q) * cap + j] / norm;
  } else {
    dens[0] = row(Y, cap, R_S, j) * sigma;
    if (NQ)
      for (int q = 0; q < 3; ++q) dens[1 + q] = row(Y, cap, R_NB + q, j) * sigma;
  }

  // EoS inversion (s, n) -> (T, mu): the offline table when the EoS carries
  // one and (s, n) is on its grid, else online, warm-started from the
  // particle's last roots
  Thermo th;
  if (!(eos.inv.val && inv_lookup<NQ>(eos.inv, dens, th))) {
    double warm[NWARM], wnew[NWARM];
#pragma unroll
    for (int w = 0; w < NWARM; ++w) warm[w] = b.warms[(int64_t)w * cap + j];
    eos_invert<NQ>(eos, 0, dens, warm, th, wnew);
#pragma unroll
    for (int w = 0; w < NWARM; ++w) b.warms[(int64_t)w * cap + j] = wnew[w];
  }
  c_noconv = th.ok ? 0u : 1u;
  c_backup = (!th.in_table && eos.kind == EOS_TABLE) ? 1u : 0u;
  c_iters = (uint32_t)th.iters;

  const double w = th.e + th.p;
  const double eta = prm.eta_over_s * dens[0];
  const double dT = th.T - prm.zeta_Tpeak;
  const double zeta = prm.zeta_width > 0.0
                          ? dens[0] * prm.zeta_peak * exp(-dT * dT / (2.0 * prm.zeta_width * prm.zeta_width))
                          : 0.0;
  const double taupi = prm.taupi_coeff * eta / w;
  const double tauPi = prm.tauPi_ratio * taupi;

  double Pi = 0.0;
  double pi[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) pi[m][n] = 0.0;
  if (VISC) {
    Pi = sigma * row(Y, cap, R_B, j);
    pi[1][1] = sigma * row(Y, cap, R_P11, j);
    pi[1][2] = pi[2][1] = sigma * row(Y, cap, R_P12, j);
    pi[2][2] = sigma * row(Y, cap, R_P22, j);
    pi[3][3] = sigma * row(Y, cap, R_P33, j);
    if (D == 3) {
      pi[1][3] = pi[3][1] = sigma * row(Y, cap, R_P13, j);
      pi[2][3] = pi[3][2] = sigma * row(Y, cap, R_P23, j);
    }
    const double Gq[4] = {0.0, 1.0, 1.0, G3};
#pragma unroll
    for (int i = 1; i < 4; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 1; k < 4; ++k) acc += Gq[k] * u[k] * pi[k][i];
      pi[0][i] = pi[i][0] = acc / gam;
    }
  }

  double* T_ = b.th;
  T_[(int64_t)T_SIGSTAR * cap + j] = ss;
  T_[(int64_t)T_T * cap + j] = th.T;
  T_[(int64_t)T_P * cap + j] = th.p;
  T_[(int64_t)T_E * cap + j] = th.e;
  T_[(int64_t)T_CS2 * cap + j] = th.cs2;
  T_[(int64_t)T_KAP * cap + j] = th.kappa;
  if (NQ) {
#pragma unroll
    for (int q = 0; q < 3; ++q) T_[(int64_t)(T_MUB + q) * cap + j] = th.mu[q];
  }
  if (VISC) {
    T_[(int64_t)T_PI * cap + j] = Pi;
    T_[(int64_t)T_ETA * cap + j] = eta;
    T_[(int64_t)T_ZETA * cap + j] = zeta;
    T_[(int64_t)T_TAUPI * cap + j] = taupi;
    T_[(int64_t)T_TAUPIB * cap + j] = tauPi;
  }

  // neighbour record for the gradient sums
  const double is2 = 1.0 / (ss * ss);
  double rec[NREC];
  rec[Q_PP] = (th.p + Pi) * is2;
#pragma unroll
  for (int jj = 1; jj < 4; ++jj)
#pragma unroll
    for (int ii = 1; ii < 4; ++ii)
      rec[Q_A11 + (jj - 1) * 3 + (ii - 1)] = (pi[jj][ii] - (u[jj] / gam) * pi[0][ii]) * is2;
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    rec[Q_U1 + k - 1] = u[k];
    rec[Q_V1 + k - 1] = u[k] / gam;
  }
#pragma unroll
  for (int r = 0; r < NREC; ++r) {
    const bool used = r == Q_PP || (VISC && r >= Q_A11 && r <= Q_A33 && ((r - Q_A11) / 3) < D && ((r - Q_A11) % 3) < D) ||
                      (r >= Q_U1 && r < Q_U1 + D) || (r >= Q_V1 && r < Q_V1 + D);
    if (!used) continue;
    if (MIXED)
      b.recf[(int64_t)r * cap + j] = (float)rec[r];
    else
      b.rec[(int64_t)r * cap + j] = rec[r];
  }
  // record of the diffusion sums (FP64 in both precisions): alpha_q = mu_q/T and
  // F^k_q / sigma*^2 with F = J - v J^0, J^k = sigma V^k, J^0 = G_k u^k J^k / gamma
  if (NQ && prm.diffusion) {
    const double Gq[4] = {0.0, 1.0, 1.0, G3};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double J[3], J0 = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        J[k] = k < D ? sigma * row(Y, cap, R_JB1 + 3 * q + k, j) : 0.0;
        J0 += Gq[1 + k] * u[1 + k] * J[k];
      }
      J0 /= gam;
      b.drec[(int64_t)(QD_AB + q) * cap + j] = th.mu[q] / th.T;
      if (q == 0) b.drec[(int64_t)QD_PI * cap + j] = Pi;
#pragma unroll
      for (int k = 0; k < D; ++k)
        b.drec[(int64_t)(QD_FB1 + 3 * q + k) * cap + j] = (J[k] - (u[1 + k] / gam) * J0) * is2;
    }
  }
  if (aux) {
    const int64_t ii = b.ids[j];
    const int64_t n = E.n;
    aux[X_SIGSTAR * n + ii] = ss;
    aux[X_S * n + ii] = dens[0];
    for (int q = 0; q < 3; ++q) aux[(X_NB + q) * n + ii] = dens[1 + q];
    aux[X_T * n + ii] = th.T;
    for (int q = 0; q < 3; ++q) aux[(X_MUB + q) * n + ii] = th.mu[q];
    aux[X_P * n + ii] = th.p;
    aux[X_E * n + ii] = th.e;
    aux[X_CS2 * n + ii] = th.cs2;
    aux[X_INTABLE * n + ii] = th.in_table;
    aux[X_GAMMA * n + ii] = gam;
    aux[X_NNB * n + ii] = b.dsum[(int64_t)DS_NNB * cap + j];
    aux[X_NEWTON * n + ii] = th.iters;
    aux[X_EOS_EVALS * n + ii] = th.evals;
  }
}

template <int D, bool VISC, bool MIXED, int NQ>
__global__ void __launch_bounds__(128) k_eos(BatchDev b, Params prm, EosDev eos, const double* __restrict__ Y,
                                             int stage, int64_t nslots, double* aux) {
  const int64_t j = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  int e = -1;
  uint32_t c_backup = 0, c_iters = 0, c_noconv = 0;
  if (j < nslots) {
    e = b.ev[j];
    if (e >= 0) eos_particle<D, VISC, MIXED, NQ>(b, prm, eos, Y, stage, j, e, aux, c_backup, c_iters, c_noconv);
  }
  wave_count_eos(b.evt, e, c_backup, c_iters, c_noconv);
}

// own record and geometry of particle j for the gradient sums
template <int D, bool VISC, bool MIXED>
__device__ __forceinline__ void grad_setup(const BatchDev& b, const Params& prm, const double* __restrict__ Y,
                                           double t, int64_t j, GradAcc<D, VISC, MIXED>& A) {
  const int64_t cap = b.cap;
  const double G3 = metric_G3(prm, t);
  A.Gk[0] = 0.0;
  A.Gk[1] = 1.0;
  A.Gk[2] = 1.0;
  A.Gk[3] = G3;
  A.ih = 1.0 / prm.h;
  A.xa[0] = row(Y, cap, R_X1, j);
  A.xa[1] = row(Y, cap, R_X2, j);
  A.xa[2] = D == 3 ? row(Y, cap, R_X3, j) : 0.0;
  auto recv = [&](int q) -> double {
    return MIXED ? (double)b.recf[(int64_t)q * cap + j] : b.rec[(int64_t)q * cap + j];
  };
  A.aPP = recv(Q_PP);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    A.aU[k] = k < D ? recv(Q_U1 + k) : 0.0;
    A.aV[k] = k < D ? recv(Q_V1 + k) : 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) A.aA[k][i] = (VISC && k < D && i < D) ? recv(Q_A11 + k * 3 + i) : 0.0;
  }
  A.init();
}

// DIFF: also the BSQ diffusion sums (DiffAcc) over the same accepted pairs
template <int D, bool VISC, bool MIXED, int DIFF>
__global__ void __launch_bounds__(256) k_grad(BatchDev b, Params prm, const double* __restrict__ Y, int stage,
                                              int64_t nslots) {
  constexpr int L = Team<D>::L;
  constexpr int ROWS = RowBlock<D>::ROWS;
  using RT = typename GradAcc<D, VISC, MIXED>::RT;
  __shared__ int32_t s_lo[Team<D>::PER_BLOCK][ROWS], s_hi[Team<D>::PER_BLOCK][ROWS];
  const int64_t tid = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t j = tid / L;
  const int lane = (int)(tid % L);
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0) return;
  const EventDev& E = b.evt[e];
  const int64_t cap = b.cap;
  const double r2max = (2.0 * prm.h) * (2.0 * prm.h);
  GradAcc<D, VISC, MIXED> A;
  grad_setup<D, VISC, MIXED>(b, prm, Y, E.t + stage * E.dt, j, A);
  DiffAcc<D, DIFF == 2> DA;
  if (DIFF) DA.init(b.drec, cap, j);
  const int team = (int)threadIdx.x / L;
  // the rows the density pass of this stage used for the same particle
  rows_load<D, L>(b, j, lane, s_lo[team], s_hi[team]);
  RowCursor<L, ROWS> cur;
  cur.start(s_lo[team], s_hi[team], lane);
  const RT* rb = MIXED ? (const RT*)b.recf : (const RT*)b.rec;
  const int32_t self = (int32_t)j;
  constexpr int PAIR_U = PairU<D>::U;
  for (;;) {
    int32_t k[PAIR_U];
    bool v[PAIR_U];
    take<PAIR_U>(cur, self, k, v);
    if (!v[0]) break;
    double xb[PAIR_U][3], d2[PAIR_U];
    bool ok[PAIR_U];
#pragma unroll
    for (int u = 0; u < PAIR_U; ++u) {
      xb[u][0] = row(Y, cap, R_X1, k[u]);
      xb[u][1] = row(Y, cap, R_X2, k[u]);
      xb[u][2] = D == 3 ? row(Y, cap, R_X3, k[u]) : 0.0;
      d2[u] = dist2<D>(A.xa, xb[u]);
      ok[u] = v[u] && d2[u] < r2max;
    }
#pragma unroll
    for (int u = 0; u < PAIR_U; ++u) {
      const int32_t m = ok[u] ? k[u] : self;
      RT bA[3][3], bU[3], bV[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        bU[q] = q < D ? rb[(int64_t)(Q_U1 + q) * cap + m] : RT(0);
        bV[q] = q < D ? rb[(int64_t)(Q_V1 + q) * cap + m] : RT(0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
          bA[q][i] = (VISC && q < D && i < D) ? rb[(int64_t)(Q_A11 + q * 3 + i) * cap + m] : RT(0);
      }
      const RT bpp = rb[(int64_t)Q_PP * cap + m];
      double ab[3], Fb[3][3], Pb = 0.0;
      if (DIFF) DiffAcc<D, DIFF == 2>::load(b.drec, cap, m, ab, Fb, Pb);
      if (ok[u]) {
        A.add(xb[u], d2[u], bpp, bA, bU, bV);
        if (DIFF) DA.add(A.xa, xb[u], d2[u], A.ih, ab, Fb, Pb);
      }
    }
    if (!v[PAIR_U - 1]) break;
  }
  {
    // lane v < NP forms gradient sum v: F_i, d_k u^j (row-major), div v
    constexpr int NP = GradAcc<D, VISC, MIXED>::NP;
    __shared__ double s_red[Team<D>::PER_BLOCK][L * NP];
    double part[NP];
    A.partials(part);
    const double tot = team_sums_lds<L, NP>(s_red[team], lane, part);
    if (lane < NP) {
      const double fsd = sigma_d<D>(prm.h) / prm.h;
      int row;
      double scale = fsd;
      if (lane < D) {
        row = GS_F1 + lane;
      } else if (lane < NP - 1) {
        const int kk = (lane - D) / D, nu = (lane - D) % D;
        row = GS_DU11 + kk * 3 + nu;
        scale = fsd / b.th[(int64_t)T_SIGSTAR * cap + j];
      } else {
        row = GS_DIVV;
        scale = fsd / b.th[(int64_t)T_SIGSTAR * cap + j];
      }
      b.gsum[(int64_t)row * cap + j] = tot * scale;
    }
  }
  if (DIFF) DA.template reduce<L>();
  if (lane == 0) {
    if (DIFF) {
      const double fsd = sigma_d<D>(prm.h) / prm.h;
      DA.write(b.gsum, cap, j, fsd, fsd / b.th[(int64_t)T_SIGSTAR * cap + j]);
    }
  }
}

// Spatial gradient of the energy density for the freeze-out surface
// ("Freeze-out hypersurface construction"), n = 1 difference form like
// d_k u^j: d_i e_a = (1/sigma*_a) sum_b (e_b - e_a) d_i W_ab.  One thread per
// particle; runs only for diagnostic evaluations.
template <int D>
__global__ void __launch_bounds__(128) k_fo_grad(BatchDev b, Params prm, const double* __restrict__ Y,
                                                 int64_t nslots) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0) return;
  const EventDev& E = b.evt[e];
  const int64_t cap = b.cap;
  const double h = prm.h, ih = 1.0 / h, r2max = (2.0 * h) * (2.0 * h);
  const double xa[3] = {row(Y, cap, R_X1, j), row(Y, cap, R_X2, j), D == 3 ? row(Y, cap, R_X3, j) : 0.0};
  const double* Ev = b.th + (int64_t)T_E * cap;
  const double ea = Ev[j];
  double de[3] = {0.0, 0.0, 0.0};
  for_each_row<D>(b, E, b.keys[j], xa, prm.cell_edge, [&](int32_t lo, int32_t hi) {
    for (int32_t k = lo; k < hi; ++k) {
      const double xb[3] = {row(Y, cap, R_X1, k), row(Y, cap, R_X2, k), D == 3 ? row(Y, cap, R_X3, k) : 0.0};
      const double d2 = dist2<D>(xa, xb);
      if (!(d2 < r2max)) continue;
      const double r = sqrt(d2);
      if (!(r > 0.0)) continue;
      const double f = spline_dw(r * ih) / r * (Ev[k] - ea);
#pragma unroll
      for (int q = 0; q < D; ++q) de[q] += f * (xa[q] - xb[q]);
    }
  });
  const double isg = sigma_d<D>(h) / h / b.th[(int64_t)T_SIGSTAR * cap + j];
#pragma unroll
  for (int q = 0; q < 3; ++q) b.gsum[(int64_t)(GS_DE1 + q) * cap + j] = q < D ? de[q] * isg : 0.0;
}

// Source densities I^mu, I_q at position x and time t: sum over the active
// sources of the rates times the normalised Gaussian around the moving
// centre, divided by sqrt(-g) (eq. conservation_source with the smeared
// deposition of the dynamical initialisation).
template <int D>
__device__ inline void source_density(const SourceSet& S, double t, double sqg, const double x[3], double I[4],
                                      double Iq[3]) {
  const int ns = S.n;
  for (int k = 0; k < ns; ++k) {
    const SourceDev& s = S.s[k];
    if (!(t >= s.t_on && t < s.t_off)) continue;
    double arg = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double dx = x[d] - (s.c0[d] + s.vel[d] * (t - s.t_on));
      arg += dx * dx * s.iw2[d];
    }
    const double g = s.norm * exp(-arg) / sqg;
#pragma unroll
    for (int m = 0; m < 4; ++m) I[m] += s.dpdt[m] * g;
#pragma unroll
    for (int q = 0; q < 3; ++q) Iq[q] += s.dndt[q] * g;
  }
}

// ---------------------------------------------------------------------------
//   mode 0: Y1 = Ys + dt f(Ys)
//   mode 1: Y0 = (Ys + Y1 + dt f(Y1)) / 2, carry ids and warm starts home
//   mode 2: write f(Y) and diagnostics in the caller's order (no update)
template <int D, bool VISC>
__global__ void __launch_bounds__(128) k_eom(BatchDev b, Params prm, const double* __restrict__ Y, int stage,
                                             int mode, int64_t nslots, double* fout, double* aux) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0) return;
  const EventDev& E = b.evt[e];
  const double t = E.t + stage * E.dt;
  const int64_t cap = b.cap;
  const double G3 = metric_G3(prm, t);
  const double Gk[4] = {0.0, 1.0, 1.0, G3};
  const double sigstar = b.th[(int64_t)T_SIGSTAR * cap + j];

  EomIn in;
  in.t = t;
  in.u[0] = 0.0;
#pragma unroll
  for (int k = 1; k < 4; ++k) in.u[k] = k <= D ? row(Y, cap, R_U1 + k - 1, j) : 0.0;
  const double gam = sqrt(1.0 + in.u[1] * in.u[1] + in.u[2] * in.u[2] + G3 * in.u[3] * in.u[3]);
  in.u[0] = gam;
#pragma unroll
  for (int k = 0; k < 4; ++k) in.v[k] = in.u[k] / gam;
#pragma unroll
  for (int n = 0; n < 4; ++n) in.dudx[0][n] = 0.0;
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int n = 1; n < 4; ++n) {
      const double v = (k <= D && n <= D) ? b.gsum[(int64_t)(GS_DU11 + (k - 1) * 3 + (n - 1)) * cap + j] : 0.0;
      in.dudx[k][n] = v;
      acc += Gk[n] * in.u[n] * v;
    }
    in.dudx[k][0] = acc / gam;
  }
  in.divv = b.gsum[(int64_t)GS_DIVV * cap + j];
  in.F[0] = 0.0;
#pragma unroll
  for (int k = 1; k < 4; ++k) in.F[k] = k <= D ? b.gsum[(int64_t)(GS_F1 + k - 1) * cap + j] : 0.0;
  const double sqg = sqrt_g(prm, t);
  in.sigma = sigstar / (gam * sqg);
  const double* T_ = b.th;
  in.w = T_[(int64_t)T_E * cap + j] + T_[(int64_t)T_P * cap + j];
  in.T = T_[(int64_t)T_T * cap + j];
  in.cs2 = T_[(int64_t)T_CS2 * cap + j];
  in.kappa = T_[(int64_t)T_KAP * cap + j];
  in.Pi = VISC ? T_[(int64_t)T_PI * cap + j] : 0.0;
  in.eta = VISC ? T_[(int64_t)T_ETA * cap + j] : 0.0;
  in.zeta = VISC ? T_[(int64_t)T_ZETA * cap + j] : 0.0;
  in.taupi = VISC ? T_[(int64_t)T_TAUPI * cap + j] : 1.0;
  in.tauPi = VISC ? T_[(int64_t)T_TAUPIB * cap + j] : 1.0;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) in.pi[m][n] = 0.0;
  if (VISC) {
    const double sg = in.sigma;
    in.pi[1][1] = sg * row(Y, cap, R_P11, j);
    in.pi[1][2] = in.pi[2][1] = sg * row(Y, cap, R_P12, j);
    in.pi[2][2] = sg * row(Y, cap, R_P22, j);
    in.pi[3][3] = sg * row(Y, cap, R_P33, j);
    if (D == 3) {
      in.pi[1][3] = in.pi[3][1] = sg * row(Y, cap, R_P13, j);
      in.pi[2][3] = in.pi[3][2] = sg * row(Y, cap, R_P23, j);
    }
#pragma unroll
    for (int i = 1; i < 4; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 1; k < 4; ++k) acc += Gk[k] * in.u[k] * in.pi[k][i];
      in.pi[0][i] = in.pi[i][0] = acc / gam;
    }
    double acc = 0.0;
#pragma unroll
    for (int i = 1; i < 4; ++i) acc += Gk[i] * in.u[i] * in.pi[0][i];
    in.pi[0][0] = acc / gam;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) in.I[k] = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    in.Iq[q] = 0.0;
    in.mu[q] = 0.0;
  }
  // the chemical potentials enter only through the charge sources
  if (prm.src && prm.src->n > 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) in.mu[q] = q < prm.ncharge ? T_[(int64_t)(T_MUB + q) * cap + j] : 0.0;
    double x[3];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = row(Y, cap, R_X1 + k, j);
    source_density<D>(*prm.src, t, sqg, x, in.I, in.Iq);
    if (prm.ncharge == 0) in.Iq[0] = in.Iq[1] = in.Iq[2] = 0.0;
  }
  EomOut o;
  eom_solve<D, VISC>(prm, in, o);
  double dV[3][3], dNd[3] = {0.0, 0.0, 0.0};
  if (prm.diffusion) {
    double V[3][3], dal[3][3], dF[3], dPi[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      dF[q] = b.gsum[(int64_t)(GS_DJB + q) * cap + j];
      dPi[q] = q < D ? b.gsum[(int64_t)(GS_DPI1 + q) * cap + j] : 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        V[q][k] = k < D ? row(Y, cap, R_JB1 + 3 * q + k, j) : 0.0;
        dal[q][k] = k < D ? b.gsum[(int64_t)(GS_DAB1 + 3 * q + k) * cap + j] : 0.0;
      }
    }
    diffusion_rates<D>(prm, in, o, V, dal, dPi, dF, dV, dNd);
  }

  double f[NROW];
#pragma unroll
  for (int r = 0; r < NROW; ++r) f[r] = 0.0;
#pragma unroll
  for (int k = 1; k <= D; ++k) {
    f[R_X1 + k - 1] = in.v[k];
    f[R_U1 + k - 1] = o.a[k];
  }
  f[R_S] = o.dS;
#pragma unroll
  for (int q = 0; q < 3; ++q) f[R_NB + q] = q < prm.ncharge ? o.dN[q] : 0.0;
  if (prm.diffusion) {
    // the charge moved by diffusion, and the entropy it carries (R^S = -mu/T)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      f[R_NB + q] += dNd[q];
      f[R_S] -= T_[(int64_t)(T_MUB + q) * cap + j] * dNd[q] / in.T;
#pragma unroll
      for (int k = 0; k < D; ++k) f[R_JB1 + 3 * q + k] = dV[q][k];
    }
  }
  if (VISC) {
    f[R_B] = o.dB;
    f[R_P11] = o.dP[1][1];
    f[R_P12] = o.dP[1][2];
    f[R_P22] = o.dP[2][2];
    f[R_P33] = o.dP[3][3];
    if (D == 3) {
      f[R_P13] = o.dP[1][3];
      f[R_P23] = o.dP[2][3];
    }
  }

  if (mode == 2) {
    const int64_t ii = b.ids[j];
    const int64_t n = E.n;
#pragma unroll
    for (int r = 0; r < NROW; ++r) fout[(int64_t)r * n + ii] = f[r];
    if (aux) {
      aux[X_THETA * n + ii] = o.theta;
#pragma unroll
      for (int k = 1; k <= 3; ++k) aux[(X_F1 + k - 1) * n + ii] = in.F[k];
      // Knudsen and inverse Reynolds numbers ("Particlization", eq. knudsen-reynolds)
      double kns = 0.0, res = 0.0, knb = 0.0, reb = 0.0;
      if (VISC) {
        const double p = T_[(int64_t)T_P * cap + j];
        const double gm[4] = {1.0, -1.0, -1.0, -Gk[3]};
        double pipi = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int k = 0; k < 4; ++k) pipi += in.pi[m][k] * gm[m] * gm[k] * in.pi[m][k];
        kns = in.taupi * sqrt(fabs(o.sigsig));
        res = sqrt(fabs(pipi)) / p;
        knb = in.tauPi * o.theta;
        reb = fabs(in.Pi) / p;
      }
      aux[X_KN_SHEAR * n + ii] = kns;
      aux[X_REINV_SHEAR * n + ii] = res;
      aux[X_KN_BULK * n + ii] = knb;
      aux[X_REINV_BULK * n + ii] = reb;
      // freeze-out surface element ("Freeze-out hypersurface construction"):
      // d_0 e from D e = -(e + p + Pi) theta + pi:sigma + u.I, D = gamma d_0 + u^i d_i;
      // n_mu = -d_mu e / sqrt(|d e . d e|), d sigma_mu = n_mu / (sigma |u.n|)
      {
        const double ee = T_[(int64_t)T_E * cap + j], pp = T_[(int64_t)T_P * cap + j];
        const double gm[4] = {1.0, -1.0, -1.0, -Gk[3]};
        const double giv[4] = {1.0, -1.0, -1.0, -1.0 / Gk[3]};
        double dmu[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < D; ++q) dmu[1 + q] = b.gsum[(int64_t)(GS_DE1 + q) * cap + j];
        double uI = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) uI += gm[m] * in.u[m] * in.I[m];
        const double De = -(ee + pp + in.Pi) * o.theta + o.pisig + uI;
        double adv = 0.0;
#pragma unroll
        for (int k = 1; k <= D; ++k) adv += in.u[k] * dmu[k];
        dmu[0] = (De - adv) / in.u[0];
        double nn = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) nn += giv[m] * dmu[m] * dmu[m];
        const double norm = sqrt(fabs(nn));
        double nl[4] = {0.0, 0.0, 0.0, 0.0}, un = 0.0;
        if (norm > 0.0) {
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            nl[m] = -dmu[m] / norm;
            un += in.u[m] * nl[m];
          }
        }
        const double dsig = (norm > 0.0 && fabs(un) > 0.0) ? 1.0 / (in.sigma * fabs(un)) : 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          aux[(X_DE0 + m) * n + ii] = dmu[m];
          aux[(X_DSIG0 + m) * n + ii] = dsig * nl[m];
        }
      }
    }
    return;
  }
  const double dt = E.dt;
  bool finite = true;
#pragma unroll
  for (int r = 0; r < NROW; ++r) {
    const bool live = (r <= R_X1 + D - 1) || (r >= R_U1 && r <= R_U1 + D - 1) || r == R_S ||
                      (r >= R_NB && r < R_NB + prm.ncharge) ||
                      (VISC && (r == R_B || r == R_P11 || r == R_P12 || r == R_P22 || r == R_P33 ||
                                (D == 3 && (r == R_P13 || r == R_P23)))) ||
                      (prm.diffusion && r >= R_JB1 && ((r - R_JB1) % 3) < D);
    if (!live) continue;
    double val;
    if (mode == 0) {
      val = row(b.Ys, cap, r, j) + dt * f[r];
      b.Y1[(int64_t)r * cap + j] = val;
    } else {
      val = 0.5 * (row(b.Ys, cap, r, j) + row(b.Y1, cap, r, j) + dt * f[r]);
      b.Y0[(int64_t)r * cap + j] = val;
    }
    finite = finite && isfinite(val);
  }
  if (mode == 1) {
    b.id[j] = b.ids[j];
#pragma unroll
    for (int w = 0; w < NWARM; ++w) b.warm[(int64_t)w * cap + j] = b.warms[(int64_t)w * cap + j];
  }
  if (!finite) {
    atomicAdd(&b.evt[e].nonfinite, 1u);
    atomicMin(&b.evt[e].first_bad, b.ids[j]);
  }
}

// ---------------------------------------------------------------------------
static inline unsigned nblocks(int64_t threads, int bs) { return (unsigned)((threads + bs - 1) / bs); }

// A stage kernel launch.  With profiling events (ev = {start, stop}) the
// dispatch itself records them, so a group's time is its kernel's execution
// without the gaps between launches.
#define CCAKE_STAGE_LAUNCH(EV, KERNEL, GRID, BLOCK, ...)                                  \
  do {                                                                                    \
    if (EV)                                                                               \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, s, (EV)[0], (EV)[1], 0, __VA_ARGS__); \
    else                                                                                  \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, s, __VA_ARGS__);                         \
  } while (0)

// mk (profiling): 8 events, start and stop of the density, EoS, gradient and
// update kernels
template <int D, bool VISC, bool MIXED>
static void stage_t(const BatchDev& b, const Params& prm, const EosDev& eos, int64_t nslots, const double* Y,
                    int stage, int mode, double* fout, double* aux, bool rates, hipStream_t s,
                    const hipEvent_t* mk) {
  constexpr int L = Team<D>::L;
  const unsigned gt = nblocks(nslots * L, 256), gp = nblocks(nslots, 128);
  const hipEvent_t* ed = mk ? mk + 0 : nullptr;
  const hipEvent_t* ee = mk ? mk + 2 : nullptr;
  const hipEvent_t* eg = mk ? mk + 4 : nullptr;
  const hipEvent_t* em = mk ? mk + 6 : nullptr;
  if (prm.density_mode != 0)
    CCAKE_STAGE_LAUNCH(ed, (k_density<D, MIXED, 0>), dim3(gt), dim3(256), b, prm, Y, nslots);
  else if (prm.ncharge)
    CCAKE_STAGE_LAUNCH(ed, (k_density<D, MIXED, 4>), dim3(gt), dim3(256), b, prm, Y, nslots);
  else
    CCAKE_STAGE_LAUNCH(ed, (k_density<D, MIXED, 1>), dim3(gt), dim3(256), b, prm, Y, nslots);
  if (prm.ncharge)
    CCAKE_STAGE_LAUNCH(ee, (k_eos<D, VISC, MIXED, 3>), dim3(gp), dim3(128), b, prm, eos, Y, stage, nslots, aux);
  else
    CCAKE_STAGE_LAUNCH(ee, (k_eos<D, VISC, MIXED, 0>), dim3(gp), dim3(128), b, prm, eos, Y, stage, nslots, aux);
  if (!rates) return;
  // diffusion sums: 1 without, 2 with the bulk-pressure gradient
  if (prm.diffusion && (prm.d_JPi[0] != 0.0 || prm.d_JPi[1] != 0.0 || prm.d_JPi[2] != 0.0))
    CCAKE_STAGE_LAUNCH(eg, (k_grad<D, VISC, MIXED, 2>), dim3(gt), dim3(256), b, prm, Y, stage, nslots);
  else if (prm.diffusion)
    CCAKE_STAGE_LAUNCH(eg, (k_grad<D, VISC, MIXED, 1>), dim3(gt), dim3(256), b, prm, Y, stage, nslots);
  else
    CCAKE_STAGE_LAUNCH(eg, (k_grad<D, VISC, MIXED, 0>), dim3(gt), dim3(256), b, prm, Y, stage, nslots);
  // diagnostic evaluations only (never profiled)
  if (aux) hipLaunchKernelGGL((k_fo_grad<D>), dim3(gp), dim3(128), 0, s, b, prm, Y, nslots);
  CCAKE_STAGE_LAUNCH(em, (k_eom<D, VISC>), dim3(gp), dim3(128), b, prm, Y, stage, mode, nslots, fout, aux);
}

template <int D, bool VISC, bool MIXED>
static void passes_t(const BatchDev& b, const Params& prm, const EosDev& eos, int64_t nslots, int which,
                     double* fout, double* aux, hipStream_t s, const hipEvent_t* marks) {
  if (which == 0) {
    stage_t<D, VISC, MIXED>(b, prm, eos, nslots, b.Ys, 0, 0, nullptr, nullptr, true, s, marks);
    stage_t<D, VISC, MIXED>(b, prm, eos, nslots, b.Y1, 1, 1, nullptr, nullptr, true, s, marks ? marks + 8 : nullptr);
  } else {
    stage_t<D, VISC, MIXED>(b, prm, eos, nslots, b.Ys, 0, 2, fout, aux, fout != nullptr, s, nullptr);
  }
}

hipError_t launch_passes(const BatchDev& b, const Params& prm, const EosDev& eos, int64_t nslots, int which,
                         double* fout, double* aux, hipStream_t s, const hipEvent_t* marks) {
  if (nslots <= 0) return hipSuccess;
  const int key = (prm.dim == 3 ? 4 : 0) + (prm.viscous ? 2 : 0) + (prm.mixed ? 1 : 0);
  switch (key) {
    case 0: passes_t<2, false, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 1: passes_t<2, false, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 2: passes_t<2, true, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 3: passes_t<2, true, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 4: passes_t<3, false, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 5: passes_t<3, false, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 6: passes_t<3, true, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 7: passes_t<3, true, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
  }
  return hipGetLastError();
}

}  // namespace ccake

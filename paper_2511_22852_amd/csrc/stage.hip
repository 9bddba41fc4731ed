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
//              ("Derivatives in relativistic SPH")
//   k_eom      one thread per particle: local M du/dx0 = F solve, relaxation
//              rates, Heun update
//
// The neighbour loops give each of L consecutive lanes every L-th candidate
// of the particle's 3^D-cell block and combine the partial sums with a fixed
// butterfly of lane shuffles, so the result is deterministic.  Candidates of
// particles in the same cell coincide, so the lanes of a wave read the same
// addresses.  In mixed precision the pair terms are formed and accumulated in
// FP32 with Kahan compensation per lane and compensated merges across lanes;
// the pair test itself is always the exact FP64 one.
#include <hip/hip_runtime.h>

#include "common.h"
#include "eom_device.h"
#include "eos_device.h"
#include "kernels.h"
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
};

// first candidate of this lane in range [lo, hi) given acc candidates before it
template <int L>
__device__ __forceinline__ int32_t first_of(int32_t lo, int acc, int lane) {
  int skip = (lane - acc) % L;
  skip += skip < 0 ? L : 0;
  return lo + skip;
}

template <int L>
__device__ __forceinline__ double team_sum(double v) {
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int L>
__device__ __forceinline__ int team_sum_i(int v) {
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int L>
__device__ __forceinline__ double team_sum_k(Kahan k) {
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) {
    const float s2 = __shfl_xor(k.s, off, 64);
    const float c2 = __shfl_xor(k.c, off, 64);
    k.merge(s2, c2);
  }
  return k.value();
}

// ---------------------------------------------------------------------------
template <int D, bool MIXED>
__global__ void __launch_bounds__(256) k_density(BatchDev b, Params prm, const double* __restrict__ Y,
                                                 int64_t nslots) {
  constexpr int L = Team<D>::L;
  const int64_t tid = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t j = tid / L;
  const int lane = (int)(tid % L);
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0) return;
  const EventDev& E = b.evt[e];
  const int64_t cap = b.cap;
  const double h = prm.h, ih = 1.0 / h, r2max = (2.0 * h) * (2.0 * h);
  const bool smoothed = prm.density_mode == 0;
  const int nq = smoothed ? prm.ncharge : 0;
  const double xa[3] = {row(Y, cap, R_X1, j), row(Y, cap, R_X2, j), D == 3 ? row(Y, cap, R_X3, j) : 0.0};
  double ss = 0.0, st = 0.0, sn0 = 0.0, sn1 = 0.0, sn2 = 0.0;
  Kahan ks{0.f, 0.f}, kt{0.f, 0.f}, kn0{0.f, 0.f}, kn1{0.f, 0.f}, kn2{0.f, 0.f};
  int nnb = 0, acc = 0;
  const int team_base = (int)(threadIdx.x & 63) - lane;
  for_each_row_team<D, L>(b, E, b.keys[j], xa, prm.cell_edge, lane, team_base, [&](int32_t lo, int32_t hi) {
    for (int32_t k = first_of<L>(lo, acc, lane); k < hi; k += L) {
      const double xb[3] = {row(Y, cap, R_X1, k), row(Y, cap, R_X2, k), D == 3 ? row(Y, cap, R_X3, k) : 0.0};
      const double d2 = dist2<D>(xa, xb);
      if (!(d2 < r2max)) continue;
      ++nnb;
      if (MIXED) {
        const float W = spline_wf(fast_sqrtf((float)d2) * (float)ih);
        ks.add(W);
        if (smoothed) {
          kt.add((float)row(Y, cap, R_S, k) * W);
          if (nq) {
            kn0.add((float)row(Y, cap, R_NB, k) * W);
            kn1.add((float)row(Y, cap, R_NS, k) * W);
            kn2.add((float)row(Y, cap, R_NQ, k) * W);
          }
        }
      } else {
        const double W = spline_w(sqrt(d2) * ih);
        ss += W;
        if (smoothed) {
          st += row(Y, cap, R_S, k) * W;
          if (nq) {
            sn0 += row(Y, cap, R_NB, k) * W;
            sn1 += row(Y, cap, R_NS, k) * W;
            sn2 += row(Y, cap, R_NQ, k) * W;
          }
        }
      }
    }
    acc += hi - lo;
  });
  if (MIXED) {
    ss = team_sum_k<L>(ks);
    if (smoothed) {
      st = team_sum_k<L>(kt);
      if (nq) {
        sn0 = team_sum_k<L>(kn0);
        sn1 = team_sum_k<L>(kn1);
        sn2 = team_sum_k<L>(kn2);
      }
    }
  } else {
    ss = team_sum<L>(ss);
    if (smoothed) {
      st = team_sum<L>(st);
      if (nq) {
        sn0 = team_sum<L>(sn0);
        sn1 = team_sum<L>(sn1);
        sn2 = team_sum<L>(sn2);
      }
    }
  }
  nnb = team_sum_i<L>(nnb);
  if (lane == 0) {
    const double sd = sigma_d<D>(h);
    b.dsum[(int64_t)DS_SIG * cap + j] = ss * sd;
    b.dsum[(int64_t)DS_S * cap + j] = st * sd;
    b.dsum[(int64_t)DS_NB * cap + j] = sn0 * sd;
    b.dsum[(int64_t)DS_NS * cap + j] = sn1 * sd;
    b.dsum[(int64_t)DS_NQ * cap + j] = sn2 * sd;
    b.dsum[(int64_t)DS_NNB * cap + j] = (double)nnb;
  }
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

  // EoS inversion (s, n) -> (T, mu), warm-started from the particle's last roots
  double warm[NWARM], wnew[NWARM];
#pragma unroll
  for (int w = 0; w < NWARM; ++w) warm[w] = b.warms[(int64_t)w * cap + j];
  Thermo th;
  eos_invert<NQ>(eos, 0, dens, warm, th, wnew);
#pragma unroll
  for (int w = 0; w < NWARM; ++w) b.warms[(int64_t)w * cap + j] = wnew[w];
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

// ---------------------------------------------------------------------------
template <int D, bool VISC, bool MIXED>
__global__ void __launch_bounds__(256) k_grad(BatchDev b, Params prm, const double* __restrict__ Y, int stage,
                                              int64_t nslots) {
  constexpr int L = Team<D>::L;
  constexpr int NA = D * D;  // viscous components A^{ji}
  const int64_t tid = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t j = tid / L;
  const int lane = (int)(tid % L);
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0) return;
  const EventDev& E = b.evt[e];
  const double t = E.t + stage * E.dt;
  const int64_t cap = b.cap;
  const double h = prm.h, ih = 1.0 / h, r2max = (2.0 * h) * (2.0 * h);
  const double G3 = metric_G3(prm, t);
  const double Gk[4] = {0.0, 1.0, 1.0, G3};
  const double xa[3] = {row(Y, cap, R_X1, j), row(Y, cap, R_X2, j), D == 3 ? row(Y, cap, R_X3, j) : 0.0};

  // own record (A stored as [j][i] with stride 3)
  auto recv = [&](int q, int64_t k) -> double {
    return MIXED ? (double)b.recf[(int64_t)q * cap + k] : b.rec[(int64_t)q * cap + k];
  };
  double aPP = recv(Q_PP, j), aU[3], aV[3], aA[3][3];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    aU[k] = recv(Q_U1 + k, j);
    aV[k] = recv(Q_V1 + k, j);
  }
  if (VISC) {
#pragma unroll
    for (int jj = 0; jj < D; ++jj)
#pragma unroll
      for (int ii = 0; ii < D; ++ii) aA[jj][ii] = recv(Q_A11 + jj * 3 + ii, j);
  }

  double F[3] = {0.0, 0.0, 0.0}, du[3][3], dv = 0.0;
  Kahan kF[3], kdu[3][3], kdv{0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    kF[k] = Kahan{0.f, 0.f};
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      du[k][n] = 0.0;
      kdu[k][n] = Kahan{0.f, 0.f};
    }
  }
  int acc = 0;
  const int team_base = (int)(threadIdx.x & 63) - lane;
  for_each_row_team<D, L>(b, E, b.keys[j], xa, prm.cell_edge, lane, team_base, [&](int32_t lo, int32_t hi) {
    for (int32_t k = first_of<L>(lo, acc, lane); k < hi; k += L) {
      const double xb[3] = {row(Y, cap, R_X1, k), row(Y, cap, R_X2, k), D == 3 ? row(Y, cap, R_X3, k) : 0.0};
      const double d2 = dist2<D>(xa, xb);
      if (!(d2 < r2max)) continue;
      if (MIXED) {
        const float d2f = (float)d2;
        if (!(d2f > 0.0f)) continue;  // self pair: grad W = 0
        const float ir = fast_rsqf(d2f);
        const float f = spline_dwf(d2f * ir * (float)ih) * ir;
        float dW[3];
#pragma unroll
        for (int q = 0; q < D; ++q) dW[q] = (float)(xa[q] - xb[q]) * f;
        const float pp = (float)aPP + b.recf[(int64_t)Q_PP * cap + k];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          float val = pp * dW[i];
          if (VISC) {
            float vis = 0.f;
#pragma unroll
            for (int jj = 0; jj < D; ++jj)
              vis += ((float)aA[jj][i] + b.recf[(int64_t)(Q_A11 + jj * 3 + i) * cap + k]) * dW[jj];
            val += (float)Gk[i + 1] * vis;
          }
          kF[i].add(val);
        }
        float dvv = 0.f;
#pragma unroll
        for (int kk = 0; kk < D; ++kk) {
#pragma unroll
          for (int nu = 0; nu < D; ++nu)
            kdu[kk][nu].add((b.recf[(int64_t)(Q_U1 + nu) * cap + k] - (float)aU[nu]) * dW[kk]);
          dvv += (b.recf[(int64_t)(Q_V1 + kk) * cap + k] - (float)aV[kk]) * dW[kk];
        }
        kdv.add(dvv);
      } else {
        const double rr = sqrt(d2);
        if (!(rr > 0.0)) continue;
        const double f = spline_dw(rr * ih) / rr;
        double dW[3];
#pragma unroll
        for (int q = 0; q < D; ++q) dW[q] = (xa[q] - xb[q]) * f;
        const double pp = aPP + b.rec[(int64_t)Q_PP * cap + k];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          double val = pp * dW[i];
          if (VISC) {
            double vis = 0.0;
#pragma unroll
            for (int jj = 0; jj < D; ++jj) vis += (aA[jj][i] + b.rec[(int64_t)(Q_A11 + jj * 3 + i) * cap + k]) * dW[jj];
            val += Gk[i + 1] * vis;
          }
          F[i] += val;
        }
#pragma unroll
        for (int kk = 0; kk < D; ++kk) {
#pragma unroll
          for (int nu = 0; nu < D; ++nu) du[kk][nu] += (b.rec[(int64_t)(Q_U1 + nu) * cap + k] - aU[nu]) * dW[kk];
          dv += (b.rec[(int64_t)(Q_V1 + kk) * cap + k] - aV[kk]) * dW[kk];
        }
      }
    }
    acc += hi - lo;
  });
  (void)NA;
#pragma unroll
  for (int i = 0; i < D; ++i) F[i] = MIXED ? team_sum_k<L>(kF[i]) : team_sum<L>(F[i]);
#pragma unroll
  for (int kk = 0; kk < D; ++kk)
#pragma unroll
    for (int nu = 0; nu < D; ++nu) du[kk][nu] = MIXED ? team_sum_k<L>(kdu[kk][nu]) : team_sum<L>(du[kk][nu]);
  dv = MIXED ? team_sum_k<L>(kdv) : team_sum<L>(dv);
  if (lane == 0) {
    const double fsd = sigma_d<D>(h) * ih;
    const double isg = fsd / b.th[(int64_t)T_SIGSTAR * cap + j];
#pragma unroll
    for (int i = 0; i < D; ++i) b.gsum[(int64_t)(GS_F1 + i) * cap + j] = F[i] * fsd;
#pragma unroll
    for (int kk = 0; kk < D; ++kk)
#pragma unroll
      for (int nu = 0; nu < D; ++nu) b.gsum[(int64_t)(GS_DU11 + kk * 3 + nu) * cap + j] = du[kk][nu] * isg;
    b.gsum[(int64_t)GS_DIVV * cap + j] = dv * isg;
  }
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
                                (D == 3 && (r == R_P13 || r == R_P23))));
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

template <int D, bool VISC, bool MIXED>
static void stage_t(const BatchDev& b, const Params& prm, const EosDev& eos, int64_t nslots, const double* Y,
                    int stage, int mode, double* fout, double* aux, bool rates, hipStream_t s,
                    const hipEvent_t* mk) {
  constexpr int L = Team<D>::L;
  const unsigned gt = nblocks(nslots * L, 256), gp = nblocks(nslots, 128);
  if (mk) (void)hipEventRecord(mk[0], s);
  hipLaunchKernelGGL((k_density<D, MIXED>), dim3(gt), dim3(256), 0, s, b, prm, Y, nslots);
  if (mk) (void)hipEventRecord(mk[1], s);
  if (prm.ncharge)
    hipLaunchKernelGGL((k_eos<D, VISC, MIXED, 3>), dim3(gp), dim3(128), 0, s, b, prm, eos, Y, stage, nslots, aux);
  else
    hipLaunchKernelGGL((k_eos<D, VISC, MIXED, 0>), dim3(gp), dim3(128), 0, s, b, prm, eos, Y, stage, nslots, aux);
  if (mk) (void)hipEventRecord(mk[2], s);
  if (!rates) return;
  hipLaunchKernelGGL((k_grad<D, VISC, MIXED>), dim3(gt), dim3(256), 0, s, b, prm, Y, stage, nslots);
  if (mk) (void)hipEventRecord(mk[3], s);
  hipLaunchKernelGGL((k_eom<D, VISC>), dim3(gp), dim3(128), 0, s, b, prm, Y, stage, mode, nslots, fout, aux);
  if (mk) (void)hipEventRecord(mk[4], s);
}

template <int D, bool VISC, bool MIXED>
static void passes_t(const BatchDev& b, const Params& prm, const EosDev& eos, int64_t nslots, int which,
                     double* fout, double* aux, hipStream_t s, const hipEvent_t* marks) {
  if (which == 0) {
    stage_t<D, VISC, MIXED>(b, prm, eos, nslots, b.Ys, 0, 0, nullptr, nullptr, true, s, marks);
    stage_t<D, VISC, MIXED>(b, prm, eos, nslots, b.Y1, 1, 1, nullptr, nullptr, true, s, marks ? marks + 5 : nullptr);
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

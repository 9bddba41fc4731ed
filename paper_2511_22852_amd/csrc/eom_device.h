// Per-particle equations of motion of relativistic viscous SPH: the local
// solve M du/dx0 = F of eq. unugeneral (no diffusion, so the R-blocks
// vanish), with every rate written as an affine function of the unknown
// acceleration a = du^i/dx0 (eq. genform).
//
// Equations (mostly-minus metric diag(1,-1,-1,-G3), G3 = tau^2 or 1;
// Q_i = G_i u^i; gamma = u^0; sigma = sigma* / (gamma sqrt(-g))):
//   theta = dgamma/dx0 + gamma (div v + d ln sqrt(-g)/dx0)
//   sigma^{mu nu} = 1/2 (nabla^mu u^nu + nabla^nu u^mu) - 1/2 (u^mu Du^nu + u^nu Du^mu)
//                   - 1/3 Delta^{mu nu} theta
//   DPi = -(Pi + zeta theta)/tau_Pi - c_PiPi Pi theta + c_Pipi pi:sigma
//         (eq. min_bul_rel; the c's are the first-order couplings of eq. dnmr)
//   gamma d(pi^{ij}/sigma)/dx0 = (1/sigma)[(2 eta sigma^{ij} - pi^{ij})/tau_pi
//         + (1 - c_pipi) pi^{ij} theta + c_piPi Pi sigma^{ij} + c_pisig pi_l^<i sigma^j>l
//         - (u^i pi^{jl} + u^j pi^{il}) Du_l - Christoffel terms]   (eq. min_she_rel)
//   Dp = -c_s^2 w theta + (dp/de)_n (-Pi theta + pi:sigma + u.I)
//   momentum: d/dx0[(w+Pi) Q_i/sigma + G_i pi^{0i}/(sigma gamma)]
//             = -sqrt(-g) F_i + G_i I^i/(gamma sigma)
//   entropy:  gamma sigma T dS/dx0 = u.I - mu_q I_q - Pi theta + pi:sigma   (eq. dsdnrewr)
//   charges:  dN_q/dx0 = I_q/(gamma sigma)
// I^mu, I_q are the external source densities of eq. conservation_source;
// D eps gains u.I (eq. e_conservation).  The charge source does not enter Dp
// ((dp/dn_q)_e = 0, exact for p = eps/3 equations of state).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace ccake {

// An affine function of the acceleration; in 2+1D the a_3 coefficient is a
// compile-time zero (no storage traffic, no arithmetic).
template <int D>
struct AffT {
  double c0, c1, c2, c3;  // value = c0 + c1 a_1 + c2 a_2 + c3 a_3
};
template <int D>
__device__ __forceinline__ AffT<D> operator+(AffT<D> x, AffT<D> y) {
  return AffT<D>{x.c0 + y.c0, x.c1 + y.c1, x.c2 + y.c2, D == 3 ? x.c3 + y.c3 : 0.0};
}
template <int D>
__device__ __forceinline__ AffT<D> operator-(AffT<D> x, AffT<D> y) {
  return AffT<D>{x.c0 - y.c0, x.c1 - y.c1, x.c2 - y.c2, D == 3 ? x.c3 - y.c3 : 0.0};
}
template <int D>
__device__ __forceinline__ AffT<D> operator*(double s, AffT<D> x) {
  return AffT<D>{s * x.c0, s * x.c1, s * x.c2, D == 3 ? s * x.c3 : 0.0};
}
template <int D>
__device__ __forceinline__ AffT<D> operator+(AffT<D> x, double v) {
  return AffT<D>{x.c0 + v, x.c1, x.c2, D == 3 ? x.c3 : 0.0};
}
template <int D>
__device__ __forceinline__ double at(AffT<D> x, const double a[4]) {
  return D == 3 ? x.c0 + x.c1 * a[1] + x.c2 * a[2] + x.c3 * a[3] : x.c0 + x.c1 * a[1] + x.c2 * a[2];
}

struct EomIn {
  double t;
  double u[4], v[4];
  double dudx[4][4];  // [k][nu] = partial_k u^nu, k = 1..3
  double divv;
  double F[4];        // SPH force sums, i = 1..D
  double sigma, w, Pi, T, cs2, kappa, eta, zeta, taupi, tauPi;
  double pi[4][4];    // pi^{mu nu}
  double I[4], Iq[3]; // source densities (zero without sources)
  double mu[3];       // chemical potentials (zero without charges)
};

struct EomOut {
  double a[4];        // du^i/dx0
  double dS, dB, theta;
  double sigsig;      // sigma^{mu nu} sigma_{mu nu} (viscous runs; 0 otherwise)
  double pisig;       // pi^{mu nu} sigma_{mu nu} (viscous runs; 0 otherwise)
  double dN[3];       // dN_q/dx0
  double dP[4][4];    // d(pi^{ij}/sigma)/dx0
};

template <int D, bool VISC>
__device__ inline void eom_solve(const Params& prm, const EomIn& in, EomOut& out) {
  using Aff = AffT<D>;
  auto aff = [](double v) { return Aff{v, 0.0, 0.0, 0.0}; };
  const bool hyp = prm.hyperbolic != 0;
  const double t = in.t;
  const double G[4] = {0.0, 1.0, 1.0, hyp ? t * t : 1.0};
  const double Gd[4] = {0.0, 0.0, 0.0, hyp ? 2.0 * t : 0.0};
  const double g[4] = {1.0, -1.0, -1.0, -G[3]};
  const double gi[4] = {1.0, -1.0, -1.0, -1.0 / G[3]};
  const double sqrtg = hyp ? t : 1.0;
  const double dlng = hyp ? 1.0 / t : 0.0;
  const double it = hyp ? 1.0 / t : 0.0;  // Christoffel Gamma^3_03 = Gamma^3_30
  const double g033 = hyp ? t : 0.0;      // Christoffel Gamma^0_33
  const double gam = in.u[0];
  const double* u = in.u;
  const double u3 = D == 3 ? u[3] : 0.0;
  // shared reciprocals (one division each instead of one per quotient)
  constexpr double THIRD = 1.0 / 3.0;
  const double igam = 1.0 / gam, isig = 1.0 / in.sigma;
  const double igs = igam * isig;

  Aff A[4];
  A[0] = aff(0.0);
  A[1] = Aff{0.0, 1.0, 0.0, 0.0};
  A[2] = Aff{0.0, 0.0, 1.0, 0.0};
  A[3] = D == 3 ? Aff{0.0, 0.0, 0.0, 1.0} : aff(0.0);

  // dgamma/dx0 and theta
  Aff dgam = igam * ((G[1] * u[1]) * A[1] + (G[2] * u[2]) * A[2] + (G[3] * u3) * A[3] +
                            0.5 * Gd[3] * u3 * u3);
  Aff theta = dgam + gam * (in.divv + dlng);
  Aff dudt[4] = {dgam, A[1], A[2], A[3]};

  // nabla_mu u^nu
  Aff nab[4][4];
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    double adv = 0.0;
#pragma unroll
    for (int k = 1; k < 4; ++k) adv += in.v[k] * in.dudx[k][nu];
    nab[0][nu] = dudt[nu] + (-adv);
#pragma unroll
    for (int k = 1; k < 4; ++k) nab[k][nu] = aff(in.dudx[k][nu]);
  }
  nab[3][0] = nab[3][0] + g033 * u3;
  nab[0][3] = nab[0][3] + it * u3;
  nab[3][3] = nab[3][3] + it * gam;

  // Du^nu and Du_nu
  Aff Du[4], Dl[4];
  Du[0] = gam * dgam + g033 * u3 * u3;
  Du[1] = gam * A[1];
  Du[2] = gam * A[2];
  Du[3] = gam * A[3] + 2.0 * it * gam * u3;
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) Dl[nu] = g[nu] * Du[nu];

  const double uu[4] = {gam, u[1], u[2], u3};
  // shear tensor sigma^{mu nu} (symmetric)
  Aff sg[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = m; n < 4; ++n) {
      const double Delta = (m == n ? gi[m] : 0.0) - uu[m] * uu[n];
      Aff val = 0.5 * (gi[m] * nab[m][n] + gi[n] * nab[n][m]) - 0.5 * (uu[m] * Du[n] + uu[n] * Du[m]) -
                (Delta * THIRD) * theta;
      sg[m][n] = val;
      sg[n][m] = val;
    }

  Aff pisig = aff(0.0);
  if (VISC) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) pisig = pisig + (in.pi[m][n] * g[m] * g[n]) * sg[m][n];
  }
  const double Pi = VISC ? in.Pi : 0.0;
  const double uI = gam * in.I[0] - (u[1] * in.I[1] + u[2] * in.I[2] + G[3] * u3 * in.I[3]);
  Aff DPi = aff(0.0);
  if (VISC) DPi = (-1.0 / in.tauPi) * (in.zeta * theta + Pi) - (prm.c_PiPi * Pi) * theta + prm.c_Pipi * pisig;
  Aff Dp = (-in.cs2 * in.w) * theta + in.kappa * ((-Pi) * theta + pisig + uI);

  // relaxation of pi^{ij}/sigma
  Aff dP[4][4];
  if (VISC) {
    const double itp = 1.0 / in.taupi;
#pragma unroll
    for (int i = 1; i < 4; ++i)
#pragma unroll
      for (int j = i; j < 4; ++j) {
        Aff val = itp * ((2.0 * in.eta) * sg[i][j] + (-in.pi[i][j])) +
                  ((1.0 - prm.c_pipi) * in.pi[i][j]) * theta + (prm.c_piPi * Pi) * sg[i][j];
        if (prm.c_pisig != 0.0) {
          // pi_lambda^<i sigma^j>lambda: both factors are transverse, so the
          // projection is the symmetric part of pi^{il} g_ll sigma^{lj} minus
          // Delta^{ij} pi:sigma / 3
          Aff Aij = aff(0.0), Aji = aff(0.0);
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            Aij = Aij + (in.pi[i][l] * g[l]) * sg[l][j];
            Aji = Aji + (in.pi[j][l] * g[l]) * sg[l][i];
          }
          const double Delta = (i == j ? gi[i] : 0.0) - uu[i] * uu[j];
          val = val + prm.c_pisig * (0.5 * (Aij + Aji) + (-Delta * THIRD) * pisig);
        }
#pragma unroll
        for (int l = 0; l < 4; ++l) val = val - (uu[i] * in.pi[j][l] + uu[j] * in.pi[i][l]) * Dl[l];
        double chr = 0.0;
        if (i == 3) chr += it * (gam * in.pi[3][j] + u3 * in.pi[0][j]);
        if (j == 3) chr += it * (gam * in.pi[i][3] + u3 * in.pi[0][i]);
        val = val + (-chr);
        dP[i][j] = igs * val;
        dP[j][i] = dP[i][j];
      }
  }

  // momentum balance rows
  const double wP = in.w + Pi;
  Aff dwPs = igs * (pisig + Dp + DPi + uI);
  Aff R[4];
#pragma unroll
  for (int i = 1; i <= D; ++i) {
    const double Qi = G[i] * uu[i];
    Aff dQ = G[i] * A[i] + Gd[i] * uu[i];
    Aff r = (wP * isig) * dQ + Qi * dwPs + (sqrtg * in.F[i] - G[i] * in.I[i] * igs);
    if (VISC) {
      double sQP = 0.0;
      Aff dsQP = aff(0.0);
#pragma unroll
      for (int j = 1; j < 4; ++j) {
        const double Pji = in.pi[j][i] * isig;
        sQP += G[j] * uu[j] * Pji;
        dsQP = dsQP + Pji * (G[j] * A[j] + Gd[j] * uu[j]) + (G[j] * uu[j]) * dP[j][i];
      }
      const double ig2 = igam * igam;
      r = r + (Gd[i] * ig2 * sQP) + (-2.0 * G[i] * ig2 * igam * sQP) * dgam + (G[i] * ig2) * dsQP;
    }
    R[i] = r;
  }

  // solve sum_j M_ij a_j = -R_i(0)
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  if (D == 2) {
    const double m11 = R[1].c1, m12 = R[1].c2, m21 = R[2].c1, m22 = R[2].c2;
    const double det = m11 * m22 - m12 * m21;
    const double b1 = -R[1].c0, b2 = -R[2].c0;
    const double id = 1.0 / det;
    a[1] = (b1 * m22 - m12 * b2) * id;
    a[2] = (m11 * b2 - b1 * m21) * id;
  } else {
    double M[3][3], b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      M[i][0] = R[i + 1].c1;
      M[i][1] = R[i + 1].c2;
      M[i][2] = R[i + 1].c3;
      b[i] = -R[i + 1].c0;
    }
    const double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    const double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
    const double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    const double det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
    const double id = 1.0 / det;
    const double i00 = c00 * id, i01 = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * id,
                 i02 = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * id;
    const double i10 = c01 * id, i11 = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * id,
                 i12 = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * id;
    const double i20 = c02 * id, i21 = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * id,
                 i22 = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * id;
    a[1] = i00 * b[0] + i01 * b[1] + i02 * b[2];
    a[2] = i10 * b[0] + i11 * b[1] + i12 * b[2];
    a[3] = i20 * b[0] + i21 * b[1] + i22 * b[2];
  }

#pragma unroll
  for (int k = 0; k < 4; ++k) out.a[k] = a[k];
  out.theta = at(theta, a);
  const double heat = uI - (in.mu[0] * in.Iq[0] + in.mu[1] * in.Iq[1] + in.mu[2] * in.Iq[2]);
#pragma unroll
  for (int q = 0; q < 3; ++q) out.dN[q] = in.Iq[q] * igs;
  out.sigsig = 0.0;
  out.pisig = 0.0;
  if (VISC) {
    double ss = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const double v = at(sg[m][n], a);
        ss += v * g[m] * g[n] * v;
      }
    out.sigsig = ss;
    const double ps = at(pisig, a), th = out.theta;
    out.pisig = ps;
    out.dS = (-Pi * th + ps + heat) * igs / in.T;
    out.dB = (at(DPi, a) + Pi * th) * igs;
#pragma unroll
    for (int i = 1; i < 4; ++i)
#pragma unroll
      for (int j = 1; j < 4; ++j) out.dP[i][j] = at(dP[i][j], a);
  } else {
    out.dS = heat * igs / in.T;
    out.dB = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) out.dP[i][j] = 0.0;
  }
}

// BSQ charge diffusion ("BSQ diffusion", eq. min_dif_rel, eq. charge_conservation,
// eq. dsdnrewr), evaluated at the solved acceleration (the momentum rows do not
// depend on the currents: Landau frame, and the pressure does not respond to
// the charge moved).  V^k_q = J^k_q / sigma, J^0 = G_k u^k J^k / gamma:
//   gamma sigma dV^i/dx0 = (kappa_{qq'} g^{ii} d_i alpha_{q'} - J^i) / tau_J
//                          + (1 - c_JJ) J^i theta - u^i J^nu Du_nu
//                          - Christoffel terms (eta: (gamma J^3 + u^3 J^0) / tau),
//   dN_q/dx0 gains -d/dx0[(G_k u^k V^k) / gamma^2] - sqrt(-g) divF_q,
// with divF_q = sum_b (F_a/sigma*_a^2 + F_b/sigma*_b^2) . grad W, F = J - v J^0
// (the change of the particle's charge N + sqrt(-g) J^0/sigma* is the flux
// through its boundary); kappa_{qq'} = kappa_T2 T^2, tau_J = tauJ_coeff / T.
template <int D>
__device__ inline void diffusion_rates(const Params& prm, const EomIn& in, const EomOut& o, const double V[3][3],
                                       const double dal[3][3], const double dPi[3], const double divF[3], double dV[3][3],
                                       double dNd[3]) {
  const bool hyp = prm.hyperbolic != 0;
  const double t = in.t;
  const double G[4] = {0.0, 1.0, 1.0, hyp ? t * t : 1.0};
  const double Gd[4] = {0.0, 0.0, 0.0, hyp ? 2.0 * t : 0.0};
  const double g[4] = {1.0, -1.0, -1.0, -G[3]};
  const double sqrtg = hyp ? t : 1.0;
  const double it = hyp ? 1.0 / t : 0.0;
  const double g033 = hyp ? t : 0.0;
  const double gam = in.u[0];
  const double u3 = D == 3 ? in.u[3] : 0.0;
  const double* a = o.a;
  const double dgam = (G[1] * in.u[1] * a[1] + G[2] * in.u[2] * a[2] + G[3] * u3 * a[3] + 0.5 * Gd[3] * u3 * u3) / gam;
  double Dl[4];
  Dl[0] = g[0] * (gam * dgam + g033 * u3 * u3);
  Dl[1] = g[1] * (gam * a[1]);
  Dl[2] = g[2] * (gam * a[2]);
  Dl[3] = g[3] * (gam * a[3] + 2.0 * it * gam * u3);
  const double T = in.T, T2 = T * T;
  const double tauJ = prm.tauJ_coeff / T;
  const double igs = 1.0 / (gam * in.sigma);
  const double th = o.theta;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double J[3], J0 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      J[k] = k < D ? in.sigma * V[q][k] : 0.0;
      J0 += G[1 + k] * in.u[1 + k] * J[k];
    }
    J0 /= gam;
    double JDu = J0 * Dl[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) JDu += J[k] * Dl[1 + k];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (i >= D) {
        dV[q][i] = 0.0;
        continue;
      }
      double target = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r)
        target += prm.kappa_T2[3 * q + r] * T2 * (1.0 / g[1 + i]) * (dal[r][i] + prm.d_JPi[r] * dPi[i]);
      double val = (target - J[i]) / tauJ + (1.0 - prm.c_JJ) * J[i] * th - in.u[1 + i] * JDu;
      if (i == 2) val -= it * (gam * J[2] + u3 * J0);
      dV[q][i] = val * igs;
    }
    double X = 0.0, dX = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      X += G[1 + k] * in.u[1 + k] * V[q][k];
      dX += (Gd[1 + k] * in.u[1 + k] + G[1 + k] * a[1 + k]) * V[q][k] + G[1 + k] * in.u[1 + k] * dV[q][k];
    }
    const double dY = dX / (gam * gam) - 2.0 * X * dgam / (gam * gam * gam);
    dNd[q] = -dY - sqrtg * divF[q];
  }
}

}  // namespace ccake

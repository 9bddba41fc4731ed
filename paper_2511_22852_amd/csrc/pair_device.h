// Per-pair arithmetic of the SPH sums of the pair kernels (one team of lanes
// per particle, candidates staged in LDS, any batch).  Every lane visits its
// candidates in a fixed order and the lanes are merged with a fixed order
// (through LDS, lane by lane), so results do not depend on the batch or the
// launch.  Rejected candidates enter with a zero kernel weight (no branch).
// Floating-point contraction is off on the whole pair path and the fused
// multiply-adds are written out.
//
//   density sums ("SPH interpretation of a fluid element"):
//     sigma* = sum_b W_ab, s* = sum_b S_b W_ab, n*_q = sum_b N_q,b W_ab
//   gradient sums ("Derivatives in relativistic SPH"):
//     F_i    = sum_b [(p+Pi)_a/sigma*_a^2 + (p+Pi)_b/sigma*_b^2] d_i W_ab
//              + G_i sum_b [A^{ji}_a/sigma*_a^2 + A^{ji}_b/sigma*_b^2] d_j W_ab   (n = -1)
//     d_k u^j = (1/sigma*_a) sum_b (u^j_b - u^j_a) d_k W_ab                      (n = 1)
//     div v   = (1/sigma*_a) sum_b (v_b - v_a) . grad W_ab
// In the FP32 (mixed) form every lane's sum is compensated (Kahan), the
// lanes' partials are merged in FP64, and the kernel uses the hardware square
// root; the pair test is FP64 in both forms.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "sph_device.h"

namespace ccake {

// FP32 form: blocks of candidate passes summed plainly before each
// compensated addition (KAHAN_BLOCK passes of U candidates per lane)
#ifndef CCAKE_KAHAN_BLOCK
#define CCAKE_KAHAN_BLOCK 4
#endif
constexpr int KAHAN_BLOCK = CCAKE_KAHAN_BLOCK;

template <int L>
__device__ __forceinline__ double team_sum(double v) {
#pragma clang fp contract(off)
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// NS smoothed scalars per neighbour: 0 (specific densities: sigma* only),
// 1 (s*), 4 (s*, n*_B, n*_S, n*_Q)
template <bool MIXED, int NS>
struct DensAcc {
  double ss, sv[4];
  Kahan ks, kv[4];
  float ps, pv[4];  // FP32 block sums not yet added with compensation
  int nnb, nb;

  __device__ __forceinline__ void init() {
    ss = 0.0;
    ks = Kahan{0.f, 0.f};
    ps = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sv[q] = 0.0;
      kv[q] = Kahan{0.f, 0.f};
      pv[q] = 0.f;
    }
    nnb = 0;
    nb = 0;
  }

  // compensated addition of the pending block sums (FP32 form)
  __device__ __forceinline__ void flush() {
    if (MIXED) {
      ks.add(ps);
      ps = 0.f;
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        kv[q].add(pv[q]);
        pv[q] = 0.f;
      }
    }
    nb = 0;
  }

  // U candidates at squared distances d2[u] with the neighbours' scalars
  // v[u] (S, N_B, N_S, N_Q; the first NS are used) in the precision of the
  // sums; those with ok[u] false (rejected or missing) enter with weight
  // zero.  FP32: the terms of KAHAN_BLOCK consecutive calls (B = KAHAN_BLOCK
  // * U terms) are summed plainly and each block total is added with
  // compensation, so the error stays below (B + 1) u sum |terms| + O(n u^2)
  // however many candidates there are (u = 2^-24).  The caller flushes the
  // last partial block (flush) at the end of every chunk of its walk, so
  // the lanes of a wave that are still walking flush on the same calls.
  // FP64: plain fused multiply-adds.
  template <int U, class T>
  __device__ __forceinline__ void add_block(const bool (&ok)[U], const double (&d2)[U], double ih,
                                            const T (&v)[U][4]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int u = 0; u < U; ++u) nnb += ok[u] ? 1 : 0;
    if (MIXED) {
      float W[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float w = spline_wf(fast_sqrtf((float)d2[u]) * (float)ih);
        W[u] = ok[u] ? w : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) ps += W[u];
#pragma unroll
      for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int u = 0; u < U; ++u) pv[q] = fmaf((float)v[u][q], W[u], pv[q]);
      if (++nb == KAHAN_BLOCK) flush();
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double r = d2[u] > 0.0 ? d2[u] * rsqrt_nr(d2[u]) : 0.0;
        const double w = spline_w(r * ih);
        const double W = ok[u] ? w : 0.0;
        ss += W;
#pragma unroll
        for (int q = 0; q < NS; ++q) sv[q] = fma((double)v[u][q], W, sv[q]);
      }
    }
  }

  // this lane's partial sums (sigma*, S, N_B, N_S, N_Q) and candidate count
  __device__ __forceinline__ void partials(double (&p)[6]) const {
    p[0] = MIXED ? ks.value() : ss;
#pragma unroll
    for (int q = 0; q < 4; ++q) p[1 + q] = q < NS ? (MIXED ? kv[q].value() : sv[q]) : 0.0;
    p[5] = (double)nnb;
  }
};

// ---------------------------------------------------------------------------
template <int D, bool VISC, bool MIXED>
struct GradAcc {
  using RT = typename std::conditional<MIXED, float, double>::type;
  double xa[3], Gk[4], ih;
  RT aPP, aA[3][3], aU[3], aV[3];
  double F[3], du[3][3], dv;
  Kahan kF[3], kdu[3][3], kdv;
  float pF[3], pdu[3][3], pdv;  // FP32 block sums not yet added with compensation
  int nb;

  __device__ __forceinline__ void init() {
    dv = 0.0;
    kdv = Kahan{0.f, 0.f};
    pdv = 0.f;
    nb = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      F[k] = 0.0;
      kF[k] = Kahan{0.f, 0.f};
      pF[k] = 0.f;
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        du[k][n] = 0.0;
        kdu[k][n] = Kahan{0.f, 0.f};
        pdu[k][n] = 0.f;
      }
    }
  }

  // compensated addition of the pending block sums (FP32 form)
  __device__ __forceinline__ void flush() {
    if (MIXED) {
#pragma unroll
      for (int i = 0; i < D; ++i) {
        kF[i].add(pF[i]);
        pF[i] = 0.f;
#pragma unroll
        for (int n = 0; n < D; ++n) {
          kdu[i][n].add(pdu[i][n]);
          pdu[i][n] = 0.f;
        }
      }
      kdv.add(pdv);
      pdv = 0.f;
    }
    nb = 0;
  }

  // U candidates at positions xb[u] and squared distances d2[u] with their
  // records r[u] = (p+Pi)/sigma*^2, u^1..u^D, v^1..v^D, A^{ji}/sigma*^2
  // (j*D + i) in the precision of the sums; a candidate is a pair when
  // ok[u] (which must exclude the self pair, whose kernel gradient is zero),
  // otherwise it enters with weight zero.  FP32: blocks of KAHAN_BLOCK calls
  // summed plainly before each compensated addition, flushed by the caller
  // at the end of every chunk, as for the density sums.
  template <int U>
  __device__ __forceinline__ void add_block(const bool (&ok)[U], const double (&xb)[U][3], const double (&d2)[U],
                                            const RT (*r)[4 * ((1 + 2 * D + (VISC ? D * D : 0) + 3) / 4)]) {
#pragma clang fp contract(off)
    if (MIXED) {
      float dW[U][3];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float d2f = (float)d2[u];
        const float ir = fast_rsqf(d2f);
        float f = spline_dwf(d2f * ir * (float)ih) * ir;
        f = ok[u] ? f : 0.0f;
#pragma unroll
        for (int q = 0; q < D; ++q) dW[u][q] = (float)(xa[q] - xb[u][q]) * f;
      }
      // forces: (p+Pi) terms and, viscous, G_i sum_j (A_a + A_b)^{ji} d_j W
#pragma unroll
      for (int i = 0; i < D; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const float pp = (float)aPP + (float)r[u][0];
          float term = pp * dW[u][i];
          if (VISC) {
            float vis = 0.f;
#pragma unroll
            for (int jj = 0; jj < D; ++jj)
              vis = fmaf((float)aA[jj][i] + (float)r[u][1 + 2 * D + jj * D + i], dW[u][jj], vis);
            term = fmaf((float)Gk[i + 1], vis, term);
          }
          pF[i] += term;
        }
      }
      // velocity gradients and divergence (n = 1 differences)
#pragma unroll
      for (int kk = 0; kk < D; ++kk)
#pragma unroll
        for (int nu = 0; nu < D; ++nu) {
#pragma unroll
          for (int u = 0; u < U; ++u) pdu[kk][nu] = fmaf((float)r[u][1 + nu] - (float)aU[nu], dW[u][kk], pdu[kk][nu]);
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int kk = 0; kk < D; ++kk) pdv = fmaf((float)r[u][1 + D + kk] - (float)aV[kk], dW[u][kk], pdv);
      if (++nb == KAHAN_BLOCK) flush();
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double ir = rsqrt_nr(d2[u]);
        double f = spline_dw(d2[u] * ir * ih) * ir;
        f = ok[u] ? f : 0.0;
        double dW[3];
#pragma unroll
        for (int q = 0; q < D; ++q) dW[q] = (xa[q] - xb[u][q]) * f;
        const double pp = aPP + (double)r[u][0];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          if (VISC) {
            double vis = 0.0;
#pragma unroll
            for (int jj = 0; jj < D; ++jj) vis = fma(aA[jj][i] + (double)r[u][1 + 2 * D + jj * D + i], dW[jj], vis);
            F[i] += fma(Gk[i + 1], vis, pp * dW[i]);
          } else {
            F[i] = fma(pp, dW[i], F[i]);
          }
        }
#pragma unroll
        for (int kk = 0; kk < D; ++kk) {
#pragma unroll
          for (int nu = 0; nu < D; ++nu) du[kk][nu] = fma((double)r[u][1 + nu] - aU[nu], dW[kk], du[kk][nu]);
          dv = fma((double)r[u][1 + D + kk] - aV[kk], dW[kk], dv);
        }
      }
    }
  }

  // this lane's partial sums: F_i, d_k u^j (row-major), div v
  static constexpr int NP = D + D * D + 1;
  __device__ __forceinline__ void partials(double (&p)[NP]) const {
#pragma unroll
    for (int i = 0; i < D; ++i) p[i] = MIXED ? kF[i].value() : F[i];
#pragma unroll
    for (int kk = 0; kk < D; ++kk)
#pragma unroll
      for (int nu = 0; nu < D; ++nu) p[D + kk * D + nu] = MIXED ? kdu[kk][nu].value() : du[kk][nu];
    p[NP - 1] = MIXED ? kdv.value() : dv;
  }
};

// ---------------------------------------------------------------------------
// BSQ diffusion sums ("BSQ diffusion"), FP64 in both precisions, formed in the
// gradient pass from the same accepted pairs:
//   d_k alpha_q = (1/sigma*_a) sum_b (alpha_b - alpha_a) d_k W_ab        (n = 1)
//   divF_q      = sum_b (F_a/sigma*_a^2 + F_b/sigma*_b^2) . grad_a W_ab   (n = -1)
// with alpha = mu/T and F = J - v J^0 (so the flux from a to b is minus the
// flux from b to a).  PI: also d_k Pi (the bulk-gradient coupling).
template <int D, bool PI>
struct DiffAcc {
  double al[3], Fa[3][3], Pa;
  double da[3][3], dj[3], dp[3];

  __device__ __forceinline__ void init(const double* __restrict__ dr, int64_t cap, int64_t j) {
    Pa = PI ? dr[(int64_t)QD_PI * cap + j] : 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      al[q] = dr[(int64_t)(QD_AB + q) * cap + j];
      dj[q] = 0.0;
      dp[q] = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        Fa[q][k] = k < D ? dr[(int64_t)(QD_FB1 + 3 * q + k) * cap + j] : 0.0;
        da[q][k] = 0.0;
      }
    }
  }

  // the neighbour's record: alpha_q, F^k_q / sigma*^2 and (PI) Pi
  __device__ __forceinline__ static void load(const double* __restrict__ dr, int64_t cap, int32_t m, double ab[3],
                                              double Fb[3][3], double& Pb) {
    Pb = PI ? dr[(int64_t)QD_PI * cap + m] : 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      ab[q] = dr[(int64_t)(QD_AB + q) * cap + m];
#pragma unroll
      for (int k = 0; k < 3; ++k) Fb[q][k] = k < D ? dr[(int64_t)(QD_FB1 + 3 * q + k) * cap + m] : 0.0;
    }
  }

  __device__ __forceinline__ void add(const double xa[3], const double xb[3], double d2, double ih, const double ab[3],
                                      const double Fb[3][3], double Pb) {
    if (!(d2 > 0.0)) return;  // self pair: grad W = 0
    const double ir = rsqrt_nr(d2);
    const double f = spline_dw(d2 * ir * ih) * ir;
    double dW[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) dW[k] = k < D ? f * (xa[k] - xb[k]) : 0.0;
    if (PI) {
      const double dPb = Pb - Pa;
#pragma unroll
      for (int k = 0; k < D; ++k) dp[k] += dPb * dW[k];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double dal = ab[q] - al[q];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        da[q][k] += dal * dW[k];
        dj[q] += (Fa[q][k] + Fb[q][k]) * dW[k];
      }
    }
  }

  template <int L>
  __device__ __forceinline__ void reduce() {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      dj[q] = team_sum<L>(dj[q]);
      if (PI && q < D) dp[q] = team_sum<L>(dp[q]);
#pragma unroll
      for (int k = 0; k < D; ++k) da[q][k] = team_sum<L>(da[q][k]);
    }
  }

  // gradient sums rows: d_k alpha_q (kernel normalisation, 1/sigma*) and divF_q
  __device__ __forceinline__ void write(double* gsum, int64_t cap, int64_t j, double fsd, double isg) const {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      gsum[(int64_t)(GS_DJB + q) * cap + j] = dj[q] * fsd;
      gsum[(int64_t)(GS_DPI1 + q) * cap + j] = (PI && q < D) ? dp[q] * isg : 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) gsum[(int64_t)(GS_DAB1 + 3 * q + k) * cap + j] = k < D ? da[q][k] * isg : 0.0;
    }
  }
};

}  // namespace ccake

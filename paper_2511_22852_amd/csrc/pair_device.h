// Per-pair arithmetic of the SPH sums of the pair kernels (one team of lanes
// per particle, candidates read from global memory, any batch).  Every lane
// visits its candidates in a fixed order and the lanes are merged with a
// fixed order (through LDS, lane by lane), so results do not depend on the
// batch or the launch.
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

template <int L>
__device__ __forceinline__ double team_sum(double v) {
#pragma clang fp contract(off)
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// FP64 team sums through LDS: lane k of the team stores its NV partials at
// buf[k * NV + v]; after a wavefront barrier (a team lies inside one wave)
// lane v < NV adds value v of the L lanes in lane order and returns it (the
// other lanes return 0).  One store and L loads and adds per lane instead of
// log2(L) dependent cross-lane exchanges per value.
template <int L, int NV>
__device__ __forceinline__ double team_sums_lds(double* __restrict__ buf, int lane, const double (&v)[NV]) {
#pragma clang fp contract(off)
  static_assert(NV <= L, "one value per lane");
#pragma unroll
  for (int q = 0; q < NV; ++q) buf[lane * NV + q] = v[q];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double acc = 0.0;
  if (lane < NV) {
#pragma unroll
    for (int k = 0; k < L; ++k) acc += buf[k * NV + lane];
  }
  return acc;
}

// ---------------------------------------------------------------------------
// NS smoothed scalars per neighbour: 0 (specific densities: sigma* only),
// 1 (s*), 4 (s*, n*_B, n*_S, n*_Q)
template <bool MIXED, int NS>
struct DensAcc {
  double ss, sv[4];
  Kahan ks, kv[4];
  int nnb;

  __device__ __forceinline__ void init() {
    ss = 0.0;
    ks = Kahan{0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sv[q] = 0.0;
      kv[q] = Kahan{0.f, 0.f};
    }
    nnb = 0;
  }

  // one accepted pair at squared distance d2 with the neighbour's scalars v
  // (S, N_B, N_S, N_Q; the first NS are used)
  __device__ __forceinline__ void add(double d2, double ih, const double v[4]) {
#pragma clang fp contract(off)
    ++nnb;
    if (MIXED) {
      const float W = spline_wf(fast_sqrtf((float)d2) * (float)ih);
      ks.add(W);
#pragma unroll
      for (int q = 0; q < NS; ++q) kv[q].add_prod((float)v[q], W);
    } else {
      const double W = spline_w(sqrt(d2) * ih);
      ss += W;
#pragma unroll
      for (int q = 0; q < NS; ++q) sv[q] = fma(v[q], W, sv[q]);
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

  __device__ __forceinline__ void init() {
    dv = 0.0;
    kdv = Kahan{0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      F[k] = 0.0;
      kF[k] = Kahan{0.f, 0.f};
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        du[k][n] = 0.0;
        kdu[k][n] = Kahan{0.f, 0.f};
      }
    }
  }

  // one accepted pair: neighbour position xb at squared distance d2 and its
  // record (p+Pi)/sigma*^2, A^{ji}/sigma*^2 ([j][i]), u, v
  __device__ __forceinline__ void add(const double xb[3], double d2, RT bpp, const RT bA[3][3], const RT bU[3],
                                      const RT bV[3]) {
#pragma clang fp contract(off)
    if (MIXED) {
      const float d2f = (float)d2;
      if (!(d2f > 0.0f)) return;  // self pair: grad W = 0
      const float ir = fast_rsqf(d2f);
      const float f = spline_dwf(d2f * ir * (float)ih) * ir;
      float dW[3];
#pragma unroll
      for (int q = 0; q < D; ++q) dW[q] = (float)(xa[q] - xb[q]) * f;
      const float pp = (float)aPP + (float)bpp;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        if (VISC) {
          float vis = 0.f;
#pragma unroll
          for (int jj = 0; jj < D; ++jj) vis = fmaf((float)aA[jj][i] + (float)bA[jj][i], dW[jj], vis);
          kF[i].add(fmaf((float)Gk[i + 1], vis, pp * dW[i]));
        } else {
          kF[i].add_prod(pp, dW[i]);
        }
      }
      float dvv = 0.f;
#pragma unroll
      for (int kk = 0; kk < D; ++kk) {
#pragma unroll
        for (int nu = 0; nu < D; ++nu) kdu[kk][nu].add_prod((float)bU[nu] - (float)aU[nu], dW[kk]);
        dvv = fmaf((float)bV[kk] - (float)aV[kk], dW[kk], dvv);
      }
      kdv.add(dvv);
    } else {
      const double rr = sqrt(d2);
      if (!(rr > 0.0)) return;
      const double f = spline_dw(rr * ih) / rr;
      double dW[3];
#pragma unroll
      for (int q = 0; q < D; ++q) dW[q] = (xa[q] - xb[q]) * f;
      const double pp = aPP + (double)bpp;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        if (VISC) {
          double vis = 0.0;
#pragma unroll
          for (int jj = 0; jj < D; ++jj) vis = fma(aA[jj][i] + (double)bA[jj][i], dW[jj], vis);
          F[i] += fma(Gk[i + 1], vis, pp * dW[i]);
        } else {
          F[i] = fma(pp, dW[i], F[i]);
        }
      }
#pragma unroll
      for (int kk = 0; kk < D; ++kk) {
#pragma unroll
        for (int nu = 0; nu < D; ++nu) du[kk][nu] = fma((double)bU[nu] - aU[nu], dW[kk], du[kk][nu]);
        dv = fma((double)bV[kk] - aV[kk], dW[kk], dv);
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
    const double r = sqrt(d2);
    const double f = spline_dw(r * ih) / r;
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

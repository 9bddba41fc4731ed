// Device equation of state: tabulated 4D (T, muB, muS, muQ) EoS with an
// online inverter (damped FP64 Newton on the quadrilinear interpolant) and the
// analytic massless u, d, s + gluon gas as the backup EoS; closed-form
// conformal EoS.  Paper: "Equation of state", "EoS inverter" (online inverter
// with the backup-EoS chain), "Modified EoS ..." appendix for the conformal
// family.  Units fm^-1.
//
// Table columns are dimensionless (s/T^3, n_q/T^3, p/T^4, c_s^2, (dp/de)_n) and
// stored node-major, 8 doubles per node, so that one corner of the 16-corner
// stencil is one 64-byte line and the four Newton columns are one 32-byte load.
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace ccake {

#define CCAKE_PI 3.14159265358979323846

struct Thermo {
  double T, mu[3], p, e, s, n[3], cs2, kappa;
  int in_table, iters, ok;
};

// flavour charges (B, S, Q) of u, d, s
__device__ __forceinline__ double flav(int f, int q) {
  const double c[3][3] = {{1.0 / 3.0, 0.0, 2.0 / 3.0}, {1.0 / 3.0, 0.0, -1.0 / 3.0}, {1.0 / 3.0, -1.0, -1.0 / 3.0}};
  return c[f][q];
}

// massless gas: p = a_g T^4 + sum_f (mu_f^2 T^2 / 2 + mu_f^4 / (4 pi^2)), a_g = 19 pi^2 / 36
__device__ inline void gas_eval(double T, const double mu[3], double* p, double sn[4], double J[4][4]) {
  const double ag = 19.0 * CCAKE_PI * CCAKE_PI / 36.0;
  const double ipi2 = 1.0 / (CCAKE_PI * CCAKE_PI);
  double mf[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) mf[f] = flav(f, 0) * mu[0] + flav(f, 1) * mu[1] + flav(f, 2) * mu[2];
  double T2 = T * T;
  double pp = ag * T2 * T2, ss = 4.0 * ag * T2 * T, nf[3];
  double jtt = 12.0 * ag * T2;
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    double m2 = mf[f] * mf[f];
    pp += 0.5 * m2 * T2 + 0.25 * ipi2 * m2 * m2;
    ss += m2 * T;
    nf[f] = mf[f] * T2 + mf[f] * m2 * ipi2;
    jtt += m2;
  }
  if (p) *p = pp;
  sn[0] = ss;
#pragma unroll
  for (int q = 0; q < 3; ++q) sn[1 + q] = flav(0, q) * nf[0] + flav(1, q) * nf[1] + flav(2, q) * nf[2];
  if (J) {
    J[0][0] = jtt;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double d = 0.0;
#pragma unroll
      for (int f = 0; f < 3; ++f) d += 2.0 * mf[f] * T * flav(f, q);
      J[0][1 + q] = d;
      J[1 + q][0] = d;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        double c = 0.0;
#pragma unroll
        for (int f = 0; f < 3; ++f) c += flav(f, q) * flav(f, r) * (T2 + 3.0 * mf[f] * mf[f] * ipi2);
        J[1 + q][1 + r] = c;
      }
    }
  }
}

__device__ __forceinline__ void tab_locate(const EosDev& e, const double x[4], int i0[4], double f[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double u = (x[k] - e.lo[k]) / e.d[k];
    int i = (int)floor(u);
    i = i < 0 ? 0 : (i > e.n[k] - 2 ? e.n[k] - 2 : i);
    i0[k] = i;
    f[k] = u - (double)i;
  }
}

// Quadrilinear interpolant of the four Newton columns (and optionally p/T^4)
// with its gradient in (T, mu).  Returns values v[0..3] = (s, nB, nS, nQ)/T^3
// and v[4] = p/T^4 when want_p.
__device__ inline void tab_interp(const EosDev& e, const double x[4], double v[5], double g[5][4], bool want_p) {
  int i0[4];
  double f[4];
  tab_locate(e, x, i0, f);
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    v[c] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) g[c][k] = 0.0;
  }
  const int n1 = e.n[1], n2 = e.n[2], n3 = e.n[3];
  for (int corner = 0; corner < 16; ++corner) {
    const int b0 = (corner >> 3) & 1, b1 = (corner >> 2) & 1, b2 = (corner >> 1) & 1, b3 = corner & 1;
    const int64_t node = (((int64_t)(i0[0] + b0) * n1 + (i0[1] + b1)) * n2 + (i0[2] + b2)) * n3 + (i0[3] + b3);
    const double* base = e.tab + node * TC_STRIDE;
    const double4 sv = *reinterpret_cast<const double4*>(base);
    const double pv = want_p ? base[TC_P] : 0.0;
    const double w0 = b0 ? f[0] : 1.0 - f[0], w1 = b1 ? f[1] : 1.0 - f[1];
    const double w2 = b2 ? f[2] : 1.0 - f[2], w3 = b3 ? f[3] : 1.0 - f[3];
    const double s0 = (b0 ? 1.0 : -1.0) / e.d[0], s1 = (b1 ? 1.0 : -1.0) / e.d[1];
    const double s2 = (b2 ? 1.0 : -1.0) / e.d[2], s3 = (b3 ? 1.0 : -1.0) / e.d[3];
    const double w = w0 * w1 * w2 * w3;
    const double dw[4] = {s0 * w1 * w2 * w3, w0 * s1 * w2 * w3, w0 * w1 * s2 * w3, w0 * w1 * w2 * s3};
    const double cv[5] = {sv.x, sv.y, sv.z, sv.w, pv};
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      v[c] += w * cv[c];
#pragma unroll
      for (int k = 0; k < 4; ++k) g[c][k] += dw[k] * cv[c];
    }
  }
}

// scalar columns (p/T^4, cs2, kappa) at x
__device__ inline void tab_scalars(const EosDev& e, const double x[4], double* ip, double* cs2, double* kap) {
  int i0[4];
  double f[4];
  tab_locate(e, x, i0, f);
  double a = 0.0, b = 0.0, c = 0.0;
  const int n1 = e.n[1], n2 = e.n[2], n3 = e.n[3];
  for (int corner = 0; corner < 16; ++corner) {
    const int b0 = (corner >> 3) & 1, b1 = (corner >> 2) & 1, b2 = (corner >> 1) & 1, b3 = corner & 1;
    const int64_t node = (((int64_t)(i0[0] + b0) * n1 + (i0[1] + b1)) * n2 + (i0[2] + b2)) * n3 + (i0[3] + b3);
    const double* base = e.tab + node * TC_STRIDE;
    const double w = (b0 ? f[0] : 1.0 - f[0]) * (b1 ? f[1] : 1.0 - f[1]) * (b2 ? f[2] : 1.0 - f[2]) *
                     (b3 ? f[3] : 1.0 - f[3]);
    a += w * base[TC_P];
    b += w * base[TC_CS2];
    c += w * base[TC_KAP];
  }
  *ip = a;
  *cs2 = b;
  *kap = c;
}

// Scaled residual of the inversion.  mode 0: (s, n) targets scaled by s0;
// mode 1: e scaled by e0, n scaled by e0^(3/4).
__device__ inline void inv_resid(const EosDev& e, bool use_table, int mode, const double tgt[4],
                                 const double x[4], double r[4], double J[4][4]) {
  double sn[4], Jsn[4][4], p = 0.0, gp[4] = {0.0, 0.0, 0.0, 0.0};
  const double T = x[0];
  if (use_table) {
    double v[5], g[5][4];
    tab_interp(e, x, v, g, mode == 1);
    const double T2 = T * T, T3 = T2 * T;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sn[c] = T3 * v[c];
      Jsn[c][0] = 3.0 * T2 * v[c] + T3 * g[c][0];
#pragma unroll
      for (int k = 1; k < 4; ++k) Jsn[c][k] = T3 * g[c][k];
    }
    if (mode == 1) {
      p = T3 * T * v[4];
      gp[0] = 4.0 * T3 * v[4] + T3 * T * g[4][0];
#pragma unroll
      for (int k = 1; k < 4; ++k) gp[k] = T3 * T * g[4][k];
    }
  } else {
    gas_eval(T, x + 1, &p, sn, Jsn);
#pragma unroll
    for (int k = 0; k < 4; ++k) gp[k] = sn[k];
  }
  if (mode == 0) {
    const double inv = 1.0 / tgt[0];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      r[c] = (sn[c] - tgt[c]) * inv;
#pragma unroll
      for (int k = 0; k < 4; ++k) J[c][k] = Jsn[c][k] * inv;
    }
  } else {
    const double en = x[0] * sn[0] + x[1] * sn[1] + x[2] * sn[2] + x[3] * sn[3] - p;
    const double inv = 1.0 / tgt[0], invn = 1.0 / pow(tgt[0], 0.75);
    r[0] = (en - tgt[0]) * inv;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double ge = x[0] * Jsn[0][k] + x[1] * Jsn[1][k] + x[2] * Jsn[2][k] + x[3] * Jsn[3][k] - gp[k];
      ge += sn[k];  // d(T s)/dT = s + ..., d(mu_q n_q)/dmu_q = n_q + ...
      J[0][k] = ge * inv;
    }
#pragma unroll
    for (int c = 1; c < 4; ++c) {
      r[c] = (sn[c] - tgt[c]) * invn;
#pragma unroll
      for (int k = 0; k < 4; ++k) J[c][k] = Jsn[c][k] * invn;
    }
  }
}

// NU x NU (NU = 1 or 4) solve by Gaussian elimination with partial pivoting;
// all indices are compile-time constants (row exchanges are selects), so the
// system stays in registers.
template <int NU>
__device__ inline bool lsolve(double A[4][4], double b[4], double x[4]) {
#pragma unroll
  for (int col = 0; col < NU; ++col) {
    int piv = col;
    double best = fabs(A[col][col]);
#pragma unroll
    for (int r = col + 1; r < NU; ++r) {
      const double v = fabs(A[r][col]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
    if (!(best > 0.0) || !isfinite(best)) return false;
#pragma unroll
    for (int r = col + 1; r < NU; ++r) {
      const bool sw = piv == r;
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        const double a = A[col][j], c = A[r][j];
        A[col][j] = sw ? c : a;
        A[r][j] = sw ? a : c;
      }
      const double a = b[col], c = b[r];
      b[col] = sw ? c : a;
      b[r] = sw ? a : c;
    }
#pragma unroll
    for (int r = col + 1; r < NU; ++r) {
      const double fct = A[r][col] / A[col][col];
#pragma unroll
      for (int j = col; j < NU; ++j) A[r][j] -= fct * A[col][j];
      b[r] -= fct * b[col];
    }
  }
#pragma unroll
  for (int i = NU - 1; i >= 0; --i) {
    double acc = b[i];
#pragma unroll
    for (int j = i + 1; j < NU; ++j) acc -= A[i][j] * x[j];
    x[i] = acc / A[i][i];
  }
  return true;
}

template <int NU>
__device__ __forceinline__ double maxnorm(const double r[4]) {
  double m = 0.0;
#pragma unroll
  for (int k = 0; k < NU; ++k) {
    const double a = fabs(r[k]);
    m = (a <= m) ? m : a;  // propagates NaN
  }
  return m;
}

// Damped Newton: full step halved until the max-norm of the scaled residual
// decreases; the table solve keeps iterates inside the table axes.  Unknowns
// (T, muB, muS, muQ), or T alone without charges.
template <int NQ>
__device__ inline bool newton(const EosDev& e, bool use_table, int mode, const double tgt[4], double x[4],
                              int max_iter, int* iters) {
  constexpr int NU = NQ > 0 ? 4 : 1;
  double r[4], J[4][4];
  inv_resid(e, use_table, mode, tgt, x, r, J);
  double nr = maxnorm<NU>(r);
  int it = 0;
  for (; it < max_iter; ++it) {
    if (nr <= e.tol) break;
    double rhs[4] = {-r[0], -r[1], -r[2], -r[3]}, dx[4] = {0.0, 0.0, 0.0, 0.0};
    if (!lsolve<NU>(J, rhs, dx)) break;
    double lam = 1.0, xt[4], rt[4], Jt[4][4], nrt = 0.0;
    bool acc = false;
    for (int hv = 0; hv < 40; ++hv) {
#pragma unroll
      for (int k = 0; k < 4; ++k) xt[k] = x[k] + (k < NU ? lam * dx[k] : 0.0);
      if (xt[0] <= 0.0) xt[0] = 0.5 * x[0];
      if (use_table) {
#pragma unroll
        for (int k = 0; k < 4; ++k) xt[k] = fmin(fmax(xt[k], e.lo[k]), e.hi[k]);
      }
      inv_resid(e, use_table, mode, tgt, xt, rt, Jt);
      nrt = maxnorm<NU>(rt);
      if (nrt < nr) {
        acc = true;
        break;
      }
      lam *= 0.5;
    }
    if (!acc) break;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[k] = xt[k];
      r[k] = rt[k];
#pragma unroll
      for (int j = 0; j < 4; ++j) J[k][j] = Jt[k][j];
    }
    nr = nrt;
  }
  *iters += it;
  return nr <= e.tol;
}


__device__ __forceinline__ bool in_axes(const EosDev& e, const double x[4]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 4; ++k) ok = ok && (x[k] >= e.lo[k]) && (x[k] <= e.hi[k]);
  return ok;
}

__device__ inline void thermo_fill(const EosDev& e, bool table, double T, const double mu[3], Thermo& th) {
  th.T = T;
  if (e.kind == EOS_CONFORMAL) {
    th.mu[0] = th.mu[1] = th.mu[2] = 0.0;
    th.e = e.fstar * T * T * T * T;
    th.p = th.e / 3.0;
    th.s = 4.0 * e.fstar * T * T * T / 3.0;
    th.n[0] = th.n[1] = th.n[2] = 0.0;
    th.cs2 = 1.0 / 3.0;
    th.kappa = 1.0 / 3.0;
    return;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) th.mu[q] = mu[q];
  if (table) {
    const double x[4] = {T, mu[0], mu[1], mu[2]};
    double v[5], g[5][4], ip, cs2, kap;
    tab_interp(e, x, v, g, false);
    tab_scalars(e, x, &ip, &cs2, &kap);
    const double T3 = T * T * T;
    th.s = T3 * v[0];
#pragma unroll
    for (int q = 0; q < 3; ++q) th.n[q] = T3 * v[1 + q];
    th.p = T3 * T * ip;
    th.e = T * th.s + mu[0] * th.n[0] + mu[1] * th.n[1] + mu[2] * th.n[2] - th.p;
    th.cs2 = cs2;
    th.kappa = kap;
    return;
  }
  double sn[4];
  gas_eval(T, mu, &th.p, sn, nullptr);
  th.s = sn[0];
#pragma unroll
  for (int q = 0; q < 3; ++q) th.n[q] = sn[1 + q];
  th.e = 3.0 * th.p;
  th.cs2 = 1.0 / 3.0;
  th.kappa = 1.0 / 3.0;
}

// Invert (s or e, nB, nS, nQ) -> (T, mu).  The analytic gas is solved first
// (from the warm start when given); if its root lies inside the table axes the
// table interpolant is solved from that root and accepted when it converges
// inside; otherwise the gas is the backup.  Conformal: closed form.
template <int NQ>
__device__ inline void eos_invert(const EosDev& e, int mode, const double in[4], const double* warm, Thermo& th) {
  th.iters = 0;
  th.in_table = 0;
  th.ok = 1;
  const double zero[3] = {0.0, 0.0, 0.0};
  if (e.kind == EOS_CONFORMAL) {
    const double T = mode == 0 ? cbrt(3.0 * in[0] / (4.0 * e.fstar)) : pow(in[0] / e.fstar, 0.25);
    thermo_fill(e, false, T, zero, th);
    return;
  }
  const double ag = 19.0 * CCAKE_PI * CCAKE_PI / 36.0;
  double tgt[4] = {in[0], NQ > 0 ? in[1] : 0.0, NQ > 0 ? in[2] : 0.0, NQ > 0 ? in[3] : 0.0};
  double x[4];
  if (warm && warm[0] > 0.0 && isfinite(warm[0]) && isfinite(warm[1]) && isfinite(warm[2]) && isfinite(warm[3])) {
    x[0] = warm[0];
    x[1] = NQ > 0 ? warm[1] : 0.0;
    x[2] = NQ > 0 ? warm[2] : 0.0;
    x[3] = NQ > 0 ? warm[3] : 0.0;
  } else {
    x[0] = mode == 0 ? cbrt(in[0] / (4.0 * ag)) : pow(in[0] / (3.0 * ag), 0.25);
    x[1] = x[2] = x[3] = 0.0;
  }
  bool ok = newton<NQ>(e, false, mode, tgt, x, e.max_iter * 4, &th.iters);
  if (e.kind == EOS_TABLE && ok && in_axes(e, x)) {
    double xt[4] = {x[0], x[1], x[2], x[3]};
    bool okt = newton<NQ>(e, true, mode, tgt, xt, e.max_iter, &th.iters);
    if (okt && in_axes(e, xt)) {
      thermo_fill(e, true, xt[0], xt + 1, th);
      th.in_table = 1;
      return;
    }
  }
  th.ok = ok ? 1 : 0;
  thermo_fill(e, false, x[0], x + 1, th);
}


}  // namespace ccake

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
  int in_table, iters, evals, ok;  // evals: residual evaluations (halvings included)
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

// Reciprocal of a (finite, nonzero) by the hardware estimate refined with
// two Newton-Raphson steps r <- r (2 - a r), to within a few ulp: for the
// pivots of the Newton solves, where it replaces a correctly rounded
// division (a long dependent chain) at no cost to the converged roots.
__device__ __forceinline__ double fast_rcp(double a) {
  double r = __builtin_amdgcn_rcp(a);
  double e = fma(-a, r, 1.0);
  r = fma(r, e, r);
  e = fma(-a, r, 1.0);
  return fma(r, e, r);
}

// Cell of x and its fractional position; node0 is the node index of the
// lower corner.  The cell index is clamped so that extrapolation off the axes
// uses the boundary cell.
__device__ __forceinline__ int32_t tab_locate(const EosDev& e, const double x[4], double f[4]) {
  int32_t node = 0;  // the table holds fewer than 2^31 nodes
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double u = (x[k] - e.lo[k]) * e.inv_d[k];
    int i = (int)floor(u);
    i = i < 0 ? 0 : (i > e.n[k] - 2 ? e.n[k] - 2 : i);
    f[k] = u - (double)i;
    node = node * e.n[k] + i;
  }
  return node;
}

// Quadrilinear interpolant of NC consecutive columns starting at column C0,
// and with GRAD its gradient in (T, mu).  The 16 corner loads are issued
// together and the multilinear form is evaluated axis by axis (last axis
// first), carrying the partial derivatives of the already-contracted axes:
// the same polynomial as the sum over corners of weight products, with about
// a third of the arithmetic.
template <int C0, int NC, bool GRAD>
__device__ inline void tab_interp(const EosDev& e, const double x[4], double v[NC], double g[NC][4]) {
  double f[4];
  const int32_t node0 = tab_locate(e, x, f);
  // corner offsets of axes 0..2 (the same for every lane)
  const int32_t s2 = e.n[3], s1 = e.n[2] * s2, s0 = e.n[1] * s1;
  // axis 3: lerp the pairs (b3 = 0, 1), which are adjacent nodes
  double a[8][NC], a3[8][NC];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int32_t node = node0 + ((m & 4) ? s0 : 0) + ((m & 2) ? s1 : 0) + ((m & 1) ? s2 : 0);
    const double* p0 = e.tab + (uint64_t)(uint32_t)node * TC_STRIDE + C0;
    const double* p1 = p0 + TC_STRIDE;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double lo = p0[c], hi = p1[c];
      a3[m][c] = hi - lo;
      a[m][c] = lo + f[3] * a3[m][c];
    }
  }
  // axis 2
  double b[4][NC], b3[4][NC], b2[4][NC];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      b2[q][c] = a[2 * q + 1][c] - a[2 * q][c];
      b[q][c] = a[2 * q][c] + f[2] * b2[q][c];
      if (GRAD) b3[q][c] = a3[2 * q][c] + f[2] * (a3[2 * q + 1][c] - a3[2 * q][c]);
    }
  // axis 1
  double c0v[2][NC], c3[2][NC], c2[2][NC], c1[2][NC];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      c1[r][c] = b[2 * r + 1][c] - b[2 * r][c];
      c0v[r][c] = b[2 * r][c] + f[1] * c1[r][c];
      if (GRAD) {
        c3[r][c] = b3[2 * r][c] + f[1] * (b3[2 * r + 1][c] - b3[2 * r][c]);
        c2[r][c] = b2[2 * r][c] + f[1] * (b2[2 * r + 1][c] - b2[2 * r][c]);
      }
    }
  // axis 0
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double d0 = c0v[1][c] - c0v[0][c];
    v[c] = c0v[0][c] + f[0] * d0;
    if (GRAD) {
      g[c][0] = d0 * e.inv_d[0];
      g[c][1] = (c1[0][c] + f[0] * (c1[1][c] - c1[0][c])) * e.inv_d[1];
      g[c][2] = (c2[0][c] + f[0] * (c2[1][c] - c2[0][c])) * e.inv_d[2];
      g[c][3] = (c3[0][c] + f[0] * (c3[1][c] - c3[0][c])) * e.inv_d[3];
    }
  }
}

// Scaled residual of the inversion and its Jacobian; sn receives (s, n) at x.
// mode 0: (s, n) targets scaled by s0; mode 1: e scaled by e0, n scaled by
// e0^(3/4).
__device__ inline void inv_resid(const EosDev& e, bool use_table, int mode, const double tgt[4],
                                 const double x[4], double r[4], double J[4][4], double sn[4]) {
  double Jsn[4][4], p = 0.0, gp[4] = {0.0, 0.0, 0.0, 0.0};
  const double T = x[0];
  if (use_table) {
    double v[5], g[5][4];
    if (mode == 1)
      tab_interp<0, 5, true>(e, x, v, g);
    else
      tab_interp<0, 4, true>(e, x, v, g);
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
  double ipv[4];  // reciprocal pivots
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
    ipv[col] = fast_rcp(A[col][col]);
#pragma unroll
    for (int r = col + 1; r < NU; ++r) {
      const double fct = A[r][col] * ipv[col];
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
    x[i] = acc * ipv[i];
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
// decreases.  Unknowns (T, muB, muS, muQ), or T alone without charges.  Table
// iterates are not confined to the axes (the interpolant continues linearly
// from the boundary cells), so a root outside the axes is found as such and
// rejected by the caller rather than stalling against the boundary.
template <int NQ>
__device__ inline bool newton(const EosDev& e, bool use_table, int mode, const double tgt[4], double x[4],
                              int max_iter, int* iters, double sn[4], int* evals) {
  constexpr int NU = NQ > 0 ? 4 : 1;
  double r[4], J[4][4];
  inv_resid(e, use_table, mode, tgt, x, r, J, sn);
  int nev = 1;
  double nr = maxnorm<NU>(r);
  int it = 0;
  for (; it < max_iter; ++it) {
    if (nr <= e.tol) break;
    double rhs[4] = {-r[0], -r[1], -r[2], -r[3]}, dx[4] = {0.0, 0.0, 0.0, 0.0};
    if (!lsolve<NU>(J, rhs, dx)) break;
    double lam = 1.0, xt[4], rt[4], Jt[4][4], snt[4], nrt = 0.0;
    bool acc = false;
    for (int hv = 0; hv < 40; ++hv) {
#pragma unroll
      for (int k = 0; k < 4; ++k) xt[k] = x[k] + (k < NU ? lam * dx[k] : 0.0);
      if (xt[0] <= 0.0) xt[0] = 0.5 * x[0];
      inv_resid(e, use_table, mode, tgt, xt, rt, Jt, snt);
      ++nev;
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
      sn[k] = snt[k];
#pragma unroll
      for (int j = 0; j < 4; ++j) J[k][j] = Jt[k][j];
    }
    nr = nrt;
  }
  *iters += it;
  *evals += nev;
  return nr <= e.tol;
}


__device__ __forceinline__ bool in_axes(const EosDev& e, const double x[4]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 4; ++k) ok = ok && (x[k] >= e.lo[k]) && (x[k] <= e.hi[k]);
  return ok;
}

// Thermodynamics at (T, mu).  For the table, sn_tab may carry (s, n) at this
// point from the solve (the interpolant's values there); the remaining
// columns are interpolated.
__device__ inline void thermo_fill(const EosDev& e, bool table, double T, const double mu[3], Thermo& th,
                                   const double* sn_tab = nullptr) {
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
    const double T3 = T * T * T;
    if (sn_tab) {
      th.s = sn_tab[0];
#pragma unroll
      for (int q = 0; q < 3; ++q) th.n[q] = sn_tab[1 + q];
    } else {
      double v[4];
      tab_interp<TC_S, 4, false>(e, x, v, nullptr);
      th.s = T3 * v[0];
#pragma unroll
      for (int q = 0; q < 3; ++q) th.n[q] = T3 * v[1 + q];
    }
    double w[3];
    tab_interp<TC_P, 3, false>(e, x, w, nullptr);
    th.p = T3 * T * w[0];
    th.e = T * th.s + mu[0] * th.n[0] + mu[1] * th.n[1] + mu[2] * th.n[2] - th.p;
    th.cs2 = w[1];
    th.kappa = w[2];
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

__device__ __forceinline__ bool finite4(const double* x) {
  return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(x[3]);
}

// Invert (s or e, nB, nS, nQ) -> (T, mu).  The analytic gas is solved first;
// if its root lies inside the table axes the table interpolant is solved and
// accepted when it converges inside; otherwise the gas is the backup.
// Conformal: closed form.
// Warm start (warm[NWARM_EOS] or null): the gas solve starts from the last gas
// root; the table solve starts from the last table root moved by the change
// of the gas root since then (the two roots differ by the interpolation
// error, which varies slowly), else from the gas root.  Both solves converge
// to the same roots from any start inside their basins; the starts only save
// iterations.  warm_out (or null) receives the new record.
template <int NQ>
__device__ inline void eos_invert(const EosDev& e, int mode, const double in[4], const double* warm, Thermo& th,
                                  double* warm_out = nullptr) {
  th.iters = 0;
  th.evals = 0;
  th.in_table = 0;
  th.ok = 1;
  const double zero[3] = {0.0, 0.0, 0.0};
  if (e.kind == EOS_CONFORMAL) {
    const double T = mode == 0 ? cbrt(3.0 * in[0] / (4.0 * e.fstar)) : pow(in[0] / e.fstar, 0.25);
    thermo_fill(e, false, T, zero, th);
    if (warm_out) {
      warm_out[W_GT] = T;
      warm_out[W_GMUB] = warm_out[W_GMUS] = warm_out[W_GMUQ] = 0.0;
      warm_out[W_TT] = warm_out[W_TMUB] = warm_out[W_TMUS] = warm_out[W_TMUQ] = 0.0;
    }
    return;
  }
  const double ag = 19.0 * CCAKE_PI * CCAKE_PI / 36.0;
  double tgt[4] = {in[0], NQ > 0 ? in[1] : 0.0, NQ > 0 ? in[2] : 0.0, NQ > 0 ? in[3] : 0.0};
  const bool warm_gas = warm && warm[W_GT] > 0.0 && finite4(warm + W_GT);
  double x[4];
  if (warm_gas) {
    x[0] = warm[W_GT];
    x[1] = NQ > 0 ? warm[W_GMUB] : 0.0;
    x[2] = NQ > 0 ? warm[W_GMUS] : 0.0;
    x[3] = NQ > 0 ? warm[W_GMUQ] : 0.0;
  } else {
    x[0] = mode == 0 ? cbrt(in[0] / (4.0 * ag)) : pow(in[0] / (3.0 * ag), 0.25);
    x[1] = x[2] = x[3] = 0.0;
  }
  double sn[4];
  bool ok = newton<NQ>(e, false, mode, tgt, x, e.max_iter * 4, &th.iters, sn, &th.evals);
  if (warm_out) {
#pragma unroll
    for (int k = 0; k < 4; ++k) warm_out[W_GT + k] = x[k];
    warm_out[W_TT] = warm_out[W_TMUB] = warm_out[W_TMUS] = warm_out[W_TMUQ] = 0.0;
  }
  if (e.kind == EOS_TABLE && ok && in_axes(e, x)) {
    double xt[4] = {x[0], x[1], x[2], x[3]};
    if (warm_gas && warm[W_TT] > 0.0 && finite4(warm + W_TT)) {
      double xs[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) xs[k] = warm[W_TT + k] + (x[k] - warm[W_GT + k]);
      if (xs[0] > 0.0 && in_axes(e, xs)) {
#pragma unroll
        for (int k = 0; k < 4; ++k) xt[k] = NQ > 0 || k == 0 ? xs[k] : 0.0;
      }
    }
    bool okt = newton<NQ>(e, true, mode, tgt, xt, e.max_iter, &th.iters, sn, &th.evals);
    if (okt && in_axes(e, xt)) {
      thermo_fill(e, true, xt[0], xt + 1, th, sn);
      th.in_table = 1;
      if (warm_out) {
#pragma unroll
        for (int k = 0; k < 4; ++k) warm_out[W_TT + k] = xt[k];
      }
      return;
    }
  }
  th.ok = ok ? 1 : 0;
  thermo_fill(e, false, x[0], x + 1, th);
}


// ---------------------------------------------------------------------------
// Offline inverter ("EoS inverter", offline option).  The node values are the
// online inversions of the node coordinates (built once by k_inv_build); a
// lookup interpolates every stored quantity multilinearly in (s, x_B, x_S,
// x_Q), x_q = n_q / s, linear in s inside a decade segment.  The point counts
// as a table point when every corner node with a weight above 1e-9 came from
// the table (so a point on a node face is decided by that face alone, whatever
// the rounding of its coordinates).  Returns false (th untouched) off the grid.

// 10^d by repeated multiplication (small d)
__device__ __forceinline__ double pow10_int(int d) {
  double p = 1.0;
  const int a = d < 0 ? -d : d;
  for (int k = 0; k < a; ++k) p *= 10.0;
  return d >= 0 ? p : 1.0 / p;
}

__host__ __device__ inline double inv_s_node(const InvDev& v, int64_t g) {
#pragma clang fp contract(off)
  const int64_t last = (int64_t)(v.d1 - v.d0) * v.P;
  int d = v.d1, m = 0;
  if (g < last) {
    d = v.d0 + (int)(g / v.P);
    m = (int)(g % v.P);
  }
  double p = 1.0;
  const int a = d < 0 ? -d : d;
  for (int k = 0; k < a; ++k) p *= 10.0;
  p = d >= 0 ? p : 1.0 / p;
  return g < last ? p * (1.0 + 9.0 * m / v.P) : p;
}

template <int NQ>
__device__ inline bool inv_lookup(const InvDev& v, const double in[4], Thermo& th) {
#pragma clang fp contract(off)
  const double s = in[0];
  if (!(s >= inv_s_node(v, 0) && s <= inv_s_node(v, v.ns - 1))) return false;
  int d = v.d0;
  while (d + 1 < v.d1 && s >= pow10_int(d + 1)) ++d;
  int m = (int)floor((s / pow10_int(d) - 1.0) * v.P / 9.0);
  m = m < 0 ? 0 : (m > v.P - 1 ? v.P - 1 : m);
  const int64_t g = (int64_t)(d - v.d0) * v.P + m;
  const double s0 = inv_s_node(v, g), s1 = inv_s_node(v, g + 1);
  constexpr int ND = NQ > 0 ? 4 : 1;
  double f[4] = {(s - s0) / (s1 - s0), 0.0, 0.0, 0.0};
  int64_t k[4] = {g, 0, 0, 0};
  int64_t ext[4] = {v.ns, 1, 1, 1};
  if (NQ > 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double x = in[1 + q] / s;
      const double u = (x - v.xlo[q]) / (v.xhi[q] - v.xlo[q]) * (v.nx[q] - 1);
      if (!(u >= 0.0 && u <= v.nx[q] - 1)) return false;
      int64_t kk = (int64_t)floor(u);
      kk = kk > v.nx[q] - 2 ? v.nx[q] - 2 : kk;
      k[1 + q] = kk;
      f[1 + q] = u - kk;
      ext[1 + q] = v.nx[q];
    }
  }
  double acc[IV_STRIDE];
#pragma unroll
  for (int c = 0; c < IV_STRIDE; ++c) acc[c] = 0.0;
  bool all_table = true;
#pragma unroll
  for (int c = 0; c < (1 << ND); ++c) {
    double w = 1.0;
    int64_t idx = 0;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      const int bit = (c >> (ND - 1 - a)) & 1;
      w *= bit ? f[a] : 1.0 - f[a];
      idx = idx * ext[a] + k[a] + bit;
    }
    const double* o = v.val + idx * IV_STRIDE;
#pragma unroll
    for (int q = 0; q < IV_STRIDE; ++q) acc[q] += w * o[q];
    if (w > 1e-9 && !(o[IV_TAB] > 0.5)) all_table = false;
  }
  th.T = acc[IV_T];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    th.mu[q] = NQ > 0 ? acc[IV_MUB + q] : 0.0;
    th.n[q] = NQ > 0 ? in[1 + q] : 0.0;
  }
  th.p = acc[IV_P];
  th.e = acc[IV_E];
  th.s = s;
  th.cs2 = acc[IV_CS2];
  th.kappa = acc[IV_KAP];
  th.in_table = all_table ? 1 : 0;
  th.iters = 0;
  th.evals = 0;
  th.ok = 1;
  return true;
}

}  // namespace ccake

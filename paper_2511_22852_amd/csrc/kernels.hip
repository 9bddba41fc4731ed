// Support kernels of the SPH library (gfx950): time advance, initialisation
// from intensive densities, pair export, state (un)sorting, per-event totals
// and the standalone EoS inversion.  The binning is in binning.hip and the
// Runge-Kutta stage in stage.hip.
#include <hip/hip_runtime.h>

#include "common.h"
#include "eos_device.h"
#include "kernels.h"
#include "sph_device.h"

namespace ccake {

__global__ void k_advance(BatchDev b) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b.max_events || !b.evt[e].active) return;
  b.evt[e].t_prev = b.evt[e].t;
  b.evt[e].t += b.evt[e].dt;
}

// Initialisation with m_b = 1 ("SPH interpretation of a fluid element"):
// sigma*_a = sum_b W_ab, S_a = s_a gamma_a sqrt(-g) / sigma*_a, N_a likewise,
// Pi = pi = 0 (sorted order; only_event >= 0 restricts to one event)
template <int D, int NQ>
__global__ void __launch_bounds__(128) k_init(BatchDev b, Params prm, EosDev eos, int dens_kind,
                                              const double* __restrict__ dens, int64_t nslots, int only_event) {
  const int64_t j = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0 || (only_event >= 0 && e != only_event)) return;
  const EventDev& E = b.evt[e];
  const double t = E.t;
  const int64_t cap = b.cap;
  const double* Y = b.Ys;
  const double h = prm.h, ih = 1.0 / h, r2max = (2.0 * h) * (2.0 * h);
  const double xa[3] = {row(Y, cap, R_X1, j), row(Y, cap, R_X2, j), D == 3 ? row(Y, cap, R_X3, j) : 0.0};
  double ss = 0.0;
  for_each_row<D>(b, E, b.keys[j], xa, prm.cell_edge, [&](int32_t lo, int32_t hi) {
    for (int32_t k = lo; k < hi; ++k) {
      const double xb[3] = {row(Y, cap, R_X1, k), row(Y, cap, R_X2, k), D == 3 ? row(Y, cap, R_X3, k) : 0.0};
      const double d2 = dist2<D>(xa, xb);
      if (d2 < r2max) ss += spline_w(sqrt(d2) * ih);
    }
  });
  ss *= sigma_d<D>(h);
  const double G3 = metric_G3(prm, t);
  const double u1 = row(Y, cap, R_U1, j), u2 = row(Y, cap, R_U2, j), u3 = D == 3 ? row(Y, cap, R_U3, j) : 0.0;
  const double gam = sqrt(1.0 + u1 * u1 + u2 * u2 + G3 * u3 * u3);
  const int64_t ii = b.ids[j];
  const int64_t n = E.n;
  const double in[4] = {dens[ii], dens[n + ii], dens[2 * n + ii], dens[3 * n + ii]};
  double s = in[0];
  if (dens_kind == 1) {
    Thermo th;
    eos_invert<NQ>(eos, 1, in, nullptr, th);
    if (!th.ok) atomicAdd(&b.evt[e].noconv, 1u);
    s = th.s;
  }
  const double fac = gam * sqrt_g(prm, t) / ss;
  b.Ys[(int64_t)R_S * cap + j] = s * fac;
  for (int q = 0; q < 3; ++q) b.Ys[(int64_t)(R_NB + q) * cap + j] = q < NQ ? in[1 + q] * fac : 0.0;
  for (int r = R_B; r <= R_P33; ++r) b.Ys[(int64_t)r * cap + j] = 0.0;
  for (int w = 0; w < NWARM; ++w) b.warms[(int64_t)w * cap + j] = 0.0;
}

// pair export (original ids) of one event; counts all, writes at most cap
template <int D>
__global__ void __launch_bounds__(256) k_pairs(BatchDev b, Params prm, int e, int64_t* counter, int64_t cap_pairs,
                                               int32_t* pa, int32_t* pb) {
  const EventDev& E = b.evt[e];
  const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (jj >= E.n) return;
  const int64_t j = E.p_base + jj;
  const int64_t cap = b.cap;
  const double* Y = b.Ys;
  const double h = prm.h, r2max = (2.0 * h) * (2.0 * h);
  const double xa[3] = {row(Y, cap, R_X1, j), row(Y, cap, R_X2, j), D == 3 ? row(Y, cap, R_X3, j) : 0.0};
  for_each_row<D>(b, E, b.keys[j], xa, prm.cell_edge, [&](int32_t lo, int32_t hi) {
    for (int32_t k = lo; k < hi; ++k) {
      const double xb[3] = {row(Y, cap, R_X1, k), row(Y, cap, R_X2, k), D == 3 ? row(Y, cap, R_X3, k) : 0.0};
      if (dist2<D>(xa, xb) < r2max) {
        const int64_t slot = (int64_t)atomicAdd((unsigned long long*)counter, 1ull);
        if (slot < cap_pairs) {
          pa[slot] = b.ids[j];
          pb[slot] = b.ids[k];
        }
      }
    }
  });
}

// state rows of one event in the caller's order
__global__ void __launch_bounds__(256) k_unsort(BatchDev b, int e, uint32_t rowmask, double* out) {
  const EventDev& E = b.evt[e];
  const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (jj >= E.n) return;
  const int64_t j = E.p_base + jj;
  const int64_t ii = b.id[j];
  for (int r = 0; r < NROW; ++r)
    out[(int64_t)r * E.n + ii] = (rowmask & (1u << r)) ? b.Y0[(int64_t)r * b.cap + j] : 0.0;
}

// state rows of one event from the caller's order into its home slots (ids = identity)
__global__ void __launch_bounds__(256) k_upload(BatchDev b, int e, const double* in, int nrows_given) {
  const EventDev& E = b.evt[e];
  const int64_t ii = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ii >= E.n) return;
  const int64_t j = E.p_base + ii;
  for (int r = 0; r < NROW; ++r) b.Y0[(int64_t)r * b.cap + j] = r < nrows_given ? in[(int64_t)r * E.n + ii] : 0.0;
  for (int w = 0; w < NWARM; ++w) b.warm[(int64_t)w * b.cap + j] = 0.0;
  b.id[j] = (int32_t)ii;
}

// Per-event totals (S, NB, NS, NQ, E, M1, M2, M3), fixed-order reduction, from
// the sorted state Ys and the thermodynamic record of the same evaluation:
// E = sum sqrt(-g) T^00 / sigma*, M_i = sum sqrt(-g) G_i T^0i / sigma*
// ("Exact conservation": the conserved energy and momentum in Cartesian runs)
__global__ void __launch_bounds__(256) k_totals(BatchDev b, Params prm, double* out) {
  const int e = blockIdx.x;
  const EventDev& E = b.evt[e];
  __shared__ double red[8][256];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (E.active) {
    const int64_t cap = b.cap;
    const double t = E.t;
    const double G3 = metric_G3(prm, t), sqg = sqrt_g(prm, t);
    const double Gk[4] = {0.0, 1.0, 1.0, G3};
    for (int64_t jj = threadIdx.x; jj < E.n; jj += blockDim.x) {
      const int64_t j = E.p_base + jj;
      const double* Y = b.Ys;
      acc[0] += row(Y, cap, R_S, j);
      double u[4] = {0.0, row(Y, cap, R_U1, j), row(Y, cap, R_U2, j), prm.dim == 3 ? row(Y, cap, R_U3, j) : 0.0};
      const double gam = sqrt(1.0 + u[1] * u[1] + u[2] * u[2] + G3 * u[3] * u[3]);
      u[0] = gam;
      // charge of a particle: N_q, plus sqrt(-g) J^0_q / sigma* = (G_k u^k V^k_q) / gamma^2 with diffusion
      for (int q = 0; q < 3; ++q) {
        double Nq = row(Y, cap, R_NB + q, j);
        if (prm.diffusion) {
          double X = 0.0;
          for (int k = 0; k < prm.dim; ++k) X += Gk[1 + k] * u[1 + k] * row(Y, cap, R_JB1 + 3 * q + k, j);
          Nq += X / (gam * gam);
        }
        acc[1 + q] += Nq;
      }
      const double ss = b.th[(int64_t)T_SIGSTAR * cap + j];
      const double sigma = ss / (gam * sqg);
      const double p = b.th[(int64_t)T_P * cap + j], w = b.th[(int64_t)T_E * cap + j] + p;
      const double Pi = prm.viscous ? b.th[(int64_t)T_PI * cap + j] : 0.0;
      double pi[4][4];
      for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) pi[m][n] = 0.0;
      if (prm.viscous) {
        pi[1][1] = sigma * row(Y, cap, R_P11, j);
        pi[1][2] = pi[2][1] = sigma * row(Y, cap, R_P12, j);
        pi[2][2] = sigma * row(Y, cap, R_P22, j);
        pi[3][3] = sigma * row(Y, cap, R_P33, j);
        if (prm.dim == 3) {
          pi[1][3] = pi[3][1] = sigma * row(Y, cap, R_P13, j);
          pi[2][3] = pi[3][2] = sigma * row(Y, cap, R_P23, j);
        }
        for (int i = 1; i < 4; ++i) {
          double a = 0.0;
          for (int k = 1; k < 4; ++k) a += Gk[k] * u[k] * pi[k][i];
          pi[0][i] = pi[i][0] = a / gam;
        }
        double a = 0.0;
        for (int i = 1; i < 4; ++i) a += Gk[i] * u[i] * pi[0][i];
        pi[0][0] = a / gam;
      }
      acc[4] += sqg * ((w + Pi) * gam * gam - (p + Pi) + pi[0][0]) / ss;
      for (int i = 1; i <= 3; ++i) acc[4 + i] += sqg * Gk[i] * ((w + Pi) * gam * u[i] + pi[0][i]) / ss;
    }
  }
  for (int k = 0; k < 8; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 8; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 8; ++k) out[e * 8 + k] = red[k][0];
}

template <int NQ>
__global__ void __launch_bounds__(128) k_eos_invert(EosDev eos, int mode, int64_t n, const double* in, double* out,
                                                    int32_t* in_table, uint32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v[4] = {in[i], in[n + i], in[2 * n + i], in[3 * n + i]};
  Thermo th;
  eos_invert<NQ>(eos, mode, v, nullptr, th);
  out[i] = th.T;
  for (int q = 0; q < 3; ++q) out[(1 + q) * n + i] = th.mu[q];
  if (in_table) in_table[i] = th.in_table;
  if (!th.ok && bad) atomicAdd(bad, 1u);
}

// Offline table: one thread per node inverts the node's (s, n) online (cold
// start) with the forward EoS and stores the thermodynamics.
template <int NQ>
__global__ void __launch_bounds__(128) k_inv_build(EosDev eos, InvDev v, double* val, int64_t nodes,
                                                   uint32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nodes) return;
  const int64_t nc = NQ > 0 ? (int64_t)v.nx[0] * v.nx[1] * v.nx[2] : 1;
  const int64_t g = i / nc;
  int64_t r = i % nc;
  double in[4] = {inv_s_node(v, g), 0.0, 0.0, 0.0};
  if (NQ > 0) {
    int k[3];
    k[2] = (int)(r % v.nx[2]);
    r /= v.nx[2];
    k[1] = (int)(r % v.nx[1]);
    k[0] = (int)(r / v.nx[1]);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double x = v.xlo[q] + (v.xhi[q] - v.xlo[q]) * k[q] / (v.nx[q] - 1);
      in[1 + q] = x * in[0];
    }
  }
  eos.inv.val = nullptr;  // the forward EoS inverts the nodes
  Thermo th;
  eos_invert<NQ>(eos, 0, in, nullptr, th);
  double* o = val + i * IV_STRIDE;
  o[IV_T] = th.T;
#pragma unroll
  for (int q = 0; q < 3; ++q) o[IV_MUB + q] = th.mu[q];
  o[IV_P] = th.p;
  o[IV_E] = th.e;
  o[IV_CS2] = th.cs2;
  o[IV_KAP] = th.kappa;
  o[IV_TAB] = th.in_table ? 1.0 : 0.0;
  if (!th.ok) atomicAdd(bad, 1u);
}

// Offline lookups of n points (s, nB, nS, nQ) = in [4][n]: out [9][n] = T,
// muB, muS, muQ, p, e, cs2, kappa, in_table; inside[i] = 1 on the grid.  Off
// the grid: online inversion when fallback is set, else NaN.
template <int NQ>
__global__ void __launch_bounds__(128) k_inv_eval(EosDev eos, int fallback, int64_t n, const double* in,
                                                  double* out, int32_t* inside) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v[4] = {in[i], in[n + i], in[2 * n + i], in[3 * n + i]};
  Thermo th;
  const bool on = eos.inv.val && inv_lookup<NQ>(eos.inv, v, th);
  inside[i] = on ? 1 : 0;
  if (!on) {
    if (!fallback) {
      for (int q = 0; q < IV_STRIDE; ++q) out[q * n + i] = NAN;
      return;
    }
    eos_invert<NQ>(eos, 0, v, nullptr, th);
  }
  out[IV_T * n + i] = th.T;
  for (int q = 0; q < 3; ++q) out[(IV_MUB + q) * n + i] = th.mu[q];
  out[IV_P * n + i] = th.p;
  out[IV_E * n + i] = th.e;
  out[IV_CS2 * n + i] = th.cs2;
  out[IV_KAP * n + i] = th.kappa;
  out[IV_TAB * n + i] = th.in_table;
}

// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_inv_build(const EosDev& eos, const InvDev& v, double* val, int64_t nodes, uint32_t* bad,
                            hipStream_t s) {
  if (nodes <= 0) return hipSuccess;
  if (v.ncharge)
    hipLaunchKernelGGL(k_inv_build<3>, dim3(blocks_for(nodes, 128)), dim3(128), 0, s, eos, v, val, nodes, bad);
  else
    hipLaunchKernelGGL(k_inv_build<0>, dim3(blocks_for(nodes, 128)), dim3(128), 0, s, eos, v, val, nodes, bad);
  return hipGetLastError();
}

hipError_t launch_inv_eval(const EosDev& eos, int fallback, int64_t n, const double* in, double* out,
                           int32_t* inside, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (eos.inv.ncharge)
    hipLaunchKernelGGL(k_inv_eval<3>, dim3(blocks_for(n, 128)), dim3(128), 0, s, eos, fallback, n, in, out, inside);
  else
    hipLaunchKernelGGL(k_inv_eval<0>, dim3(blocks_for(n, 128)), dim3(128), 0, s, eos, fallback, n, in, out, inside);
  return hipGetLastError();
}

hipError_t launch_advance(const BatchDev& b, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(blocks_for(b.max_events, 64)), dim3(64), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_init(const BatchDev& b, const Params& prm, const EosDev& eos, int dens_kind, const double* dens,
                       int64_t nslots, hipStream_t s, int only_event) {
  const unsigned g = blocks_for(nslots, 128);
  if (g == 0) return hipSuccess;
  const int key = (prm.dim == 3 ? 2 : 0) + (prm.ncharge ? 1 : 0);
  switch (key) {
    case 0:
      hipLaunchKernelGGL((k_init<2, 0>), dim3(g), dim3(128), 0, s, b, prm, eos, dens_kind, dens, nslots, only_event);
      break;
    case 1:
      hipLaunchKernelGGL((k_init<2, 3>), dim3(g), dim3(128), 0, s, b, prm, eos, dens_kind, dens, nslots, only_event);
      break;
    case 2:
      hipLaunchKernelGGL((k_init<3, 0>), dim3(g), dim3(128), 0, s, b, prm, eos, dens_kind, dens, nslots, only_event);
      break;
    case 3:
      hipLaunchKernelGGL((k_init<3, 3>), dim3(g), dim3(128), 0, s, b, prm, eos, dens_kind, dens, nslots, only_event);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_pairs(const BatchDev& b, const Params& prm, int e, int64_t n, int64_t* counter, int64_t cap,
                        int32_t* pa, int32_t* pb, hipStream_t s) {
  const unsigned g = blocks_for(n, 256);
  if (g == 0) return hipSuccess;
  if (prm.dim == 3)
    hipLaunchKernelGGL(k_pairs<3>, dim3(g), dim3(256), 0, s, b, prm, e, counter, cap, pa, pb);
  else
    hipLaunchKernelGGL(k_pairs<2>, dim3(g), dim3(256), 0, s, b, prm, e, counter, cap, pa, pb);
  return hipGetLastError();
}

hipError_t launch_unsort(const BatchDev& b, int e, int64_t n, uint32_t rowmask, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unsort, dim3(blocks_for(n, 256)), dim3(256), 0, s, b, e, rowmask, out);
  return hipGetLastError();
}

hipError_t launch_upload(const BatchDev& b, int e, int64_t n, const double* in, int nrows, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_upload, dim3(blocks_for(n, 256)), dim3(256), 0, s, b, e, in, nrows);
  return hipGetLastError();
}

hipError_t launch_totals(const BatchDev& b, const Params& prm, int nevents, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_totals, dim3(nevents), dim3(256), 0, s, b, prm, out);
  return hipGetLastError();
}

hipError_t launch_eos_invert(const EosDev& eos, int mode, int nq, int64_t n, const double* in, double* out,
                             int32_t* in_table, uint32_t* bad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (nq)
    hipLaunchKernelGGL(k_eos_invert<3>, dim3(blocks_for(n, 128)), dim3(128), 0, s, eos, mode, n, in, out, in_table,
                       bad);
  else
    hipLaunchKernelGGL(k_eos_invert<0>, dim3(blocks_for(n, 128)), dim3(128), 0, s, eos, mode, n, in, out, in_table,
                       bad);
  return hipGetLastError();
}

}  // namespace ccake

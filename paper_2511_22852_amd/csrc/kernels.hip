// HIP kernels (gfx950) for one Runge-Kutta stage of relativistic viscous SPH.
//
// Every kernel works on a batch: the particles of all resident events sit in
// one slot range, each event in a contiguous sub-range with its own cell
// grid, time and error counters (EventDev).  A single simulation is a batch
// of one event; the serving loop runs many events through the same launches.
//
// Per step:  k_bbox -> k_count -> k_scan -> k_scatter -> k_cellsort ->
//            k_permute -> [k_pass1 -> k_pass2] x 2 Heun stages -> k_advance.
// The cell grid is built once per step with an edge of at least 2h + skin,
// which keeps every stage-2 pair inside the 3^D neighbour block (particles
// move at most dt * max(1, 1/tau) per stage).
#include <hip/hip_runtime.h>

#include "common.h"
#include "eom_device.h"
#include "eos_device.h"
#include "kernels.h"

namespace ccake {

// ---------------------------------------------------------------------------
// cubic-spline kernel ("Kernel function"): W = sigma_d w(q); grad_a W_ab =
// (sigma_d/h) w'(q) (x_a - x_b)/r, zero at r = 0
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ double sigma_d(double h) {
  return D == 2 ? 10.0 / (7.0 * CCAKE_PI * h * h) : 1.0 / (CCAKE_PI * h * h * h);
}

__device__ __forceinline__ double spline_w(double q) {
  if (q <= 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
  if (q <= 2.0) {
    double t = 2.0 - q;
    return 0.25 * t * t * t;
  }
  return 0.0;
}

__device__ __forceinline__ double spline_dw(double q) {
  if (q <= 1.0) return -3.0 * q + 2.25 * q * q;
  if (q <= 2.0) {
    double t = 2.0 - q;
    return -0.75 * t * t;
  }
  return 0.0;
}

__device__ __forceinline__ float spline_wf(float q) {
  if (q <= 1.0f) return 1.0f - 1.5f * q * q + 0.75f * q * q * q;
  if (q <= 2.0f) {
    float t = 2.0f - q;
    return 0.25f * t * t * t;
  }
  return 0.0f;
}

__device__ __forceinline__ float spline_dwf(float q) {
  if (q <= 1.0f) return -3.0f * q + 2.25f * q * q;
  if (q <= 2.0f) {
    float t = 2.0f - q;
    return -0.75f * t * t;
  }
  return 0.0f;
}

// compensated (Kahan) accumulation in FP32
struct Kahan {
  float s, c;
  __device__ __forceinline__ void add(float x) {
    float y = x - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
  }
};

// squared distance, accumulated axis by axis with separately rounded
// products and sums (FMA contraction off) so that the pair relation is
// reproducible bit for bit
template <int D>
__device__ __forceinline__ double dist2(const double xa[3], const double xb[3]) {
#pragma clang fp contract(off)
  double dx = xa[0] - xb[0];
  double d2 = dx * dx;
#pragma unroll
  for (int k = 1; k < D; ++k) {
    double dk = xa[k] - xb[k];
    d2 = d2 + dk * dk;
  }
  return d2;
}

__device__ __forceinline__ double row(const double* Y, int64_t cap, int r, int64_t i) { return Y[(int64_t)r * cap + i]; }

// neighbour block of a particle: 3^(D-1) contiguous slot ranges (x-rows of cells)
template <int D>
struct Block {
  int32_t lo[9], hi[9];
  int nr;
};

template <int D>
__device__ __forceinline__ void neighbour_block(const BatchDev& b, const EventDev& E, int32_t key, Block<D>& blk) {
  const int nx = E.nc[0], ny = E.nc[1], nz = D == 3 ? E.nc[2] : 1;
  const int ix = key % nx;
  const int iy = (key / nx) % ny;
  const int iz = D == 3 ? key / (nx * ny) : 0;
  const int x0 = ix > 0 ? ix - 1 : 0, x1 = ix + 1 < nx ? ix + 1 : nx - 1;
  blk.nr = 0;
  const int32_t* cs = b.cell_start + E.c_base;
  for (int z = (D == 3 ? iz - 1 : 0); z <= (D == 3 ? iz + 1 : 0); ++z) {
    if (z < 0 || z >= nz) continue;
    for (int y = iy - 1; y <= iy + 1; ++y) {
      if (y < 0 || y >= ny) continue;
      const int c = (z * ny + y) * nx;
      blk.lo[blk.nr] = cs[c + x0];
      blk.hi[blk.nr] = cs[c + x1 + 1];
      ++blk.nr;
    }
  }
}

// ---------------------------------------------------------------------------
// binning: per-event bounding box and grid, counting sort by (cell, id)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_bbox(BatchDev b, Params prm, int dim) {
  const int e = blockIdx.x;
  EventDev* E = b.evt + e;
  if (!E->active) return;
  __shared__ double smin[3][256], smax[3][256];
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = threadIdx.x; i < E->n; i += blockDim.x) {
    for (int k = 0; k < dim; ++k) {
      double x = row(b.Y0, b.cap, R_X1 + k, E->p_base + i);
      lo[k] = fmin(lo[k], x);
      hi[k] = fmax(hi[k], x);
    }
  }
  for (int k = 0; k < 3; ++k) {
    smin[k][threadIdx.x] = lo[k];
    smax[k][threadIdx.x] = hi[k];
  }
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) {
        smin[k][threadIdx.x] = fmin(smin[k][threadIdx.x], smin[k][threadIdx.x + s]);
        smax[k][threadIdx.x] = fmax(smax[k][threadIdx.x], smax[k][threadIdx.x + s]);
      }
    __syncthreads();
  }
  __shared__ int64_t s_ncell;
  if (threadIdx.x == 0) {
    double edge = prm.cell_edge;
    int64_t nc[3] = {1, 1, 1}, tot = 1;
    bool finite = true;
    for (int k = 0; k < dim; ++k) finite = finite && isfinite(smin[k][0]) && isfinite(smax[k][0]);
    if (!finite || E->n == 0) {
      for (int k = 0; k < 3; ++k) {
        smin[k][0] = 0.0;
        smax[k][0] = 0.0;
      }
      if (!finite) E->capacity_err += 1;
    }
    // coarsen the grid (never below the cutoff) until it fits the capacity
    for (int it = 0; it < 64; ++it) {
      tot = 1;
      for (int k = 0; k < dim; ++k) {
        nc[k] = (int64_t)floor((smax[k][0] - smin[k][0]) / edge) + 1;
        tot *= nc[k];
      }
      if (tot + 1 <= E->c_cap) break;
      edge *= 1.25;
    }
    if (tot + 1 > E->c_cap) {
      // cannot happen for finite coordinates; fall back to one cell (exact, slow)
      E->capacity_err += 1;
      for (int k = 0; k < 3; ++k) nc[k] = 1;
      tot = 1;
    }
    for (int k = 0; k < 3; ++k) {
      E->lo[k] = smin[k][0];
      E->nc[k] = (int32_t)nc[k];
    }
    E->edge = edge;
    s_ncell = tot;
  }
  __syncthreads();
  const int64_t ncell = s_ncell;
  for (int64_t c = threadIdx.x; c < ncell; c += blockDim.x) b.cell_fill[E->c_base + c] = 0;
}

__global__ void __launch_bounds__(256) k_count(BatchDev b, int dim, int64_t nslots) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslots) return;
  const int e = b.ev[i];
  if (e < 0) return;
  const EventDev& E = b.evt[e];
  int32_t key = 0, stride = 1;
  for (int k = 0; k < dim; ++k) {
    double u = (row(b.Y0, b.cap, R_X1 + k, i) - E.lo[k]) / E.edge;
    int c = (int)floor(u);
    c = c < 0 ? 0 : (c >= E.nc[k] ? E.nc[k] - 1 : c);
    key += c * stride;
    stride *= E.nc[k];
  }
  b.key[i] = key;
  atomicAdd(&b.cell_fill[E.c_base + key], 1);
}

// exclusive scan of the cell counts of one event (one 1024-thread block per event)
__global__ void __launch_bounds__(1024) k_scan(BatchDev b, int dim) {
  const int e = blockIdx.x;
  const EventDev& E = b.evt[e];
  if (!E.active) return;
  int64_t ncell = 1;
  for (int k = 0; k < dim; ++k) ncell *= E.nc[k];
  __shared__ int32_t part[1024];
  const int T = blockDim.x;
  const int64_t chunk = (ncell + T - 1) / T;
  const int64_t c0 = threadIdx.x * chunk, c1 = min(ncell, c0 + chunk);
  int32_t* cf = b.cell_fill + E.c_base;
  int32_t* cs = b.cell_start + E.c_base;
  int32_t sum = 0;
  for (int64_t c = c0; c < c1; ++c) sum += cf[c];
  part[threadIdx.x] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 1024 partial sums
  for (int off = 1; off < T; off <<= 1) {
    int32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int32_t run = (int32_t)E.p_base + (threadIdx.x > 0 ? part[threadIdx.x - 1] : 0);
  for (int64_t c = c0; c < c1; ++c) {
    int32_t cnt = cf[c];
    cs[c] = run;
    cf[c] = run;  // becomes the scatter cursor
    run += cnt;
  }
  if (threadIdx.x == T - 1) cs[ncell] = (int32_t)(E.p_base + E.n);
}

__global__ void __launch_bounds__(256) k_scatter(BatchDev b, int64_t nslots) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslots) return;
  const int e = b.ev[i];
  if (e < 0) return;
  const int32_t slot = atomicAdd(&b.cell_fill[b.evt[e].c_base + b.key[i]], 1);
  b.perm[slot] = (int32_t)i;
}

// order each cell by original id (insertion sort; cells hold tens of particles)
__global__ void __launch_bounds__(256) k_cellsort(BatchDev b, int dim) {
  const int e = blockIdx.y;
  const EventDev& E = b.evt[e];
  if (!E.active) return;
  int64_t ncell = 1;
  for (int k = 0; k < dim; ++k) ncell *= E.nc[k];
  const int32_t* cs = b.cell_start + E.c_base;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = cs[c], t = cs[c + 1];
    for (int32_t i = s + 1; i < t; ++i) {
      const int32_t p = b.perm[i];
      const int32_t pid = b.id[p];
      int32_t j = i - 1;
      while (j >= s && b.id[b.perm[j]] > pid) {
        b.perm[j + 1] = b.perm[j];
        --j;
      }
      b.perm[j + 1] = p;
    }
  }
}

__global__ void __launch_bounds__(256) k_permute(BatchDev b, int64_t nslots, uint32_t rowmask) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslots || b.ev[j] < 0) return;
  const int64_t src = b.perm[j];
  for (int r = 0; r < NROW; ++r)
    if (rowmask & (1u << r)) b.Ys[(int64_t)r * b.cap + j] = b.Y0[(int64_t)r * b.cap + src];
  for (int w = 0; w < NWARM; ++w) b.warms[(int64_t)w * b.cap + j] = b.warm[(int64_t)w * b.cap + src];
  b.ids[j] = b.id[src];
  b.keys[j] = b.key[src];
}

// sorted -> home (after an initialisation or a state upload)
__global__ void __launch_bounds__(256) k_commit(BatchDev b, int64_t nslots, uint32_t rowmask) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslots || b.ev[j] < 0) return;
  for (int r = 0; r < NROW; ++r)
    if (rowmask & (1u << r)) b.Y0[(int64_t)r * b.cap + j] = b.Ys[(int64_t)r * b.cap + j];
  for (int w = 0; w < NWARM; ++w) b.warm[(int64_t)w * b.cap + j] = b.warms[(int64_t)w * b.cap + j];
  b.id[j] = b.ids[j];
}

// ---------------------------------------------------------------------------
// geometry helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double metric_G3(const Params& prm, double t) { return prm.hyperbolic ? t * t : 1.0; }
__device__ __forceinline__ double sqrt_g(const Params& prm, double t) { return prm.hyperbolic ? t : 1.0; }

// ---------------------------------------------------------------------------
// pass 1: density sums, EoS inversion, transport coefficients, records
// ---------------------------------------------------------------------------
template <int D, bool VISC, bool MIXED>
__global__ void __launch_bounds__(256) k_pass1(BatchDev b, Params prm, EosDev eos, const double* __restrict__ Y,
                                               int stage, int64_t nslots, double* aux) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0) return;
  const EventDev& E = b.evt[e];
  const double t = E.t + stage * E.dt;
  const int64_t cap = b.cap;
  const double h = prm.h;
  const double r2max = (2.0 * h) * (2.0 * h);
  const double ih = 1.0 / h;
  const double xa[3] = {row(Y, cap, R_X1, j), row(Y, cap, R_X2, j), D == 3 ? row(Y, cap, R_X3, j) : 0.0};
  const bool smoothed = prm.density_mode == 0;
  const int nq = prm.ncharge;

  Block<D> blk;
  neighbour_block<D>(b, E, b.keys[j], blk);
  double ss = 0.0, st = 0.0, sn[3] = {0.0, 0.0, 0.0};
  Kahan ks{0.f, 0.f}, kt{0.f, 0.f}, kn[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
  int nnb = 0;
  for (int r = 0; r < blk.nr; ++r) {
    for (int32_t k = blk.lo[r]; k < blk.hi[r]; ++k) {
      const double xb[3] = {row(Y, cap, R_X1, k), row(Y, cap, R_X2, k), D == 3 ? row(Y, cap, R_X3, k) : 0.0};
      const double d2 = dist2<D>(xa, xb);
      if (!(d2 < r2max)) continue;
      ++nnb;
      if (MIXED) {
        const float W = spline_wf(sqrtf((float)d2) * (float)ih);
        ks.add(W);
        if (smoothed) {
          kt.add((float)row(Y, cap, R_S, k) * W);
          for (int q = 0; q < nq; ++q) kn[q].add((float)row(Y, cap, R_NB + q, k) * W);
        }
      } else {
        const double W = spline_w(sqrt(d2) * ih);
        ss += W;
        if (smoothed) {
          st += row(Y, cap, R_S, k) * W;
          for (int q = 0; q < nq; ++q) sn[q] += row(Y, cap, R_NB + q, k) * W;
        }
      }
    }
  }
  const double sd = sigma_d<D>(h);
  if (MIXED) {
    ss = (double)ks.s;
    st = (double)kt.s;
    for (int q = 0; q < 3; ++q) sn[q] = (double)kn[q].s;
  }
  ss *= sd;
  st *= sd;
  for (int q = 0; q < 3; ++q) sn[q] *= sd;

  // lab frame -> rest frame
  const double G3 = metric_G3(prm, t);
  double u[4] = {0.0, row(Y, cap, R_U1, j), row(Y, cap, R_U2, j), D == 3 ? row(Y, cap, R_U3, j) : 0.0};
  const double gam = sqrt(1.0 + u[1] * u[1] + u[2] * u[2] + G3 * u[3] * u[3]);
  u[0] = gam;
  const double norm = gam * sqrt_g(prm, t);
  const double sigma = ss / norm;
  double dens[4];
  if (smoothed) {
    dens[0] = st / norm;
    for (int q = 0; q < 3; ++q) dens[1 + q] = q < nq ? sn[q] / norm : 0.0;
  } else {
    dens[0] = row(Y, cap, R_S, j) * sigma;
    for (int q = 0; q < 3; ++q) dens[1 + q] = q < nq ? row(Y, cap, R_NB + q, j) * sigma : 0.0;
  }

  // EoS inversion (s, n) -> (T, mu), warm-started from the particle's last root
  double warm[4];
  for (int w = 0; w < 4; ++w) warm[w] = b.warms[(int64_t)w * cap + j];
  Thermo th;
  eos_invert(eos, 0, nq, dens, warm, th);
  b.warms[(int64_t)W_T * cap + j] = th.T;
  for (int q = 0; q < 3; ++q) b.warms[(int64_t)(W_MUB + q) * cap + j] = th.mu[q];
  if (!th.ok) atomicAdd(&b.evt[e].noconv, 1u);
  if (!th.in_table && eos.kind == EOS_TABLE) atomicAdd(&b.evt[e].backup, 1u);
  atomicAdd(&b.evt[e].newton_iters, (uint32_t)th.iters);

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

  // thermodynamic record of the particle itself
  double* T_ = b.th;
  T_[(int64_t)T_SIGSTAR * cap + j] = ss;
  T_[(int64_t)T_T * cap + j] = th.T;
  for (int q = 0; q < 3; ++q) T_[(int64_t)(T_MUB + q) * cap + j] = th.mu[q];
  T_[(int64_t)T_P * cap + j] = th.p;
  T_[(int64_t)T_E * cap + j] = th.e;
  T_[(int64_t)T_CS2 * cap + j] = th.cs2;
  T_[(int64_t)T_KAP * cap + j] = th.kappa;
  T_[(int64_t)T_PI * cap + j] = Pi;
  T_[(int64_t)T_ETA * cap + j] = eta;
  T_[(int64_t)T_ZETA * cap + j] = zeta;
  T_[(int64_t)T_TAUPI * cap + j] = taupi;
  T_[(int64_t)T_TAUPIB * cap + j] = tauPi;
  T_[(int64_t)T_S * cap + j] = dens[0];
  for (int q = 0; q < 3; ++q) T_[(int64_t)(T_NB + q) * cap + j] = dens[1 + q];
  T_[(int64_t)T_NNB * cap + j] = (double)nnb + (th.in_table ? 0.5 : 0.0);

  // neighbour record for pass 2
  const double is2 = 1.0 / (ss * ss);
  double rec[NREC];
  rec[Q_PP] = (th.p + Pi) * is2;
#pragma unroll
  for (int jj = 1; jj < 4; ++jj)
#pragma unroll
    for (int ii = 1; ii < 4; ++ii) rec[Q_A11 + (jj - 1) * 3 + (ii - 1)] = (pi[jj][ii] - (u[jj] / gam) * pi[0][ii]) * is2;
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    rec[Q_U1 + k - 1] = u[k];
    rec[Q_V1 + k - 1] = u[k] / gam;
  }
  for (int r = 0; r < NREC; ++r) {
    if (!VISC && r >= Q_A11 && r <= Q_A33) continue;
    if (MIXED)
      b.recf[(int64_t)r * cap + j] = (float)rec[r];
    else
      b.rec[(int64_t)r * cap + j] = rec[r];
  }
  if (aux) {
    const int64_t ii = b.ids[j];
    const int64_t n = E.n;
    double* A = aux;  // [NAUXROW][n] in original order of the event
    A[X_SIGSTAR * n + ii] = ss;
    A[X_S * n + ii] = dens[0];
    for (int q = 0; q < 3; ++q) A[(X_NB + q) * n + ii] = dens[1 + q];
    A[X_T * n + ii] = th.T;
    for (int q = 0; q < 3; ++q) A[(X_MUB + q) * n + ii] = th.mu[q];
    A[X_P * n + ii] = th.p;
    A[X_E * n + ii] = th.e;
    A[X_CS2 * n + ii] = th.cs2;
    A[X_INTABLE * n + ii] = th.in_table;
    A[X_GAMMA * n + ii] = gam;
    A[X_NNB * n + ii] = nnb;
  }
}

// ---------------------------------------------------------------------------
// pass 2: gradient sums, local EoM solve, Heun update
//   mode 0: Y1 = Ys + dt f(Ys)
//   mode 1: Y0 = (Ys + Y1 + dt f(Y1)) / 2, carry ids and warm starts home
//   mode 2: write f(Y) and diagnostics in original order (no update)
// ---------------------------------------------------------------------------
template <int D, bool VISC, bool MIXED>
__global__ void __launch_bounds__(256) k_pass2(BatchDev b, Params prm, const double* __restrict__ Y, int stage,
                                               int mode, int64_t nslots, double* fout, double* aux) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0) return;
  const EventDev& E = b.evt[e];
  const double t = E.t + stage * E.dt;
  const int64_t cap = b.cap;
  const double h = prm.h;
  const double r2max = (2.0 * h) * (2.0 * h);
  const double ih = 1.0 / h;
  const double xa[3] = {row(Y, cap, R_X1, j), row(Y, cap, R_X2, j), D == 3 ? row(Y, cap, R_X3, j) : 0.0};
  const double G3 = metric_G3(prm, t);
  const double Gk[4] = {0.0, 1.0, 1.0, G3};

  // own record
  double ra[NREC];
  for (int r = 0; r < NREC; ++r) {
    if (!VISC && r >= Q_A11 && r <= Q_A33) {
      ra[r] = 0.0;
      continue;
    }
    ra[r] = MIXED ? (double)b.recf[(int64_t)r * cap + j] : b.rec[(int64_t)r * cap + j];
  }
  const double sigstar = b.th[(int64_t)T_SIGSTAR * cap + j];

  Block<D> blk;
  neighbour_block<D>(b, E, b.keys[j], blk);
  double F[4] = {0.0, 0.0, 0.0, 0.0}, du[4][4], divv = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < 4; ++n) du[k][n] = 0.0;
  Kahan kF[4], kdu[4][4], kdv;
  if (MIXED) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      kF[k] = Kahan{0.f, 0.f};
#pragma unroll
      for (int n = 0; n < 4; ++n) kdu[k][n] = Kahan{0.f, 0.f};
    }
    kdv = Kahan{0.f, 0.f};
  }
  const double fsd = sigma_d<D>(h) * ih;  // sigma_d / h
  float rfa[NREC];
  if (MIXED)
    for (int r = 0; r < NREC; ++r) rfa[r] = (float)ra[r];
  for (int r = 0; r < blk.nr; ++r) {
    for (int32_t k = blk.lo[r]; k < blk.hi[r]; ++k) {
      const double xb[3] = {row(Y, cap, R_X1, k), row(Y, cap, R_X2, k), D == 3 ? row(Y, cap, R_X3, k) : 0.0};
      const double d2 = dist2<D>(xa, xb);
      if (!(d2 < r2max)) continue;
      if (MIXED) {
        const float rr = sqrtf((float)d2);
        if (rr <= 0.0f) continue;
        const float f = spline_dwf(rr * (float)ih) / rr;
        float dW[4] = {0.f, (float)(xa[0] - xb[0]) * f, (float)(xa[1] - xb[1]) * f,
                       D == 3 ? (float)(xa[2] - xb[2]) * f : 0.f};
        float rb[NREC];
        for (int q = 0; q < NREC; ++q) {
          if (!VISC && q >= Q_A11 && q <= Q_A33) {
            rb[q] = 0.f;
            continue;
          }
          rb[q] = b.recf[(int64_t)q * cap + k];
        }
        const float pp = rfa[Q_PP] + rb[Q_PP];
#pragma unroll
        for (int i = 1; i <= D; ++i) {
          float val = pp * dW[i];
          if (VISC) {
            float vis = 0.f;
#pragma unroll
            for (int jj = 1; jj <= D; ++jj) {
              const int q = Q_A11 + (jj - 1) * 3 + (i - 1);
              vis += (rfa[q] + rb[q]) * dW[jj];
            }
            val += (float)Gk[i] * vis;
          }
          kF[i].add(val);
        }
        float dv = 0.f;
#pragma unroll
        for (int kk = 1; kk <= D; ++kk) {
#pragma unroll
          for (int nu = 1; nu <= D; ++nu) kdu[kk][nu].add((rb[Q_U1 + nu - 1] - rfa[Q_U1 + nu - 1]) * dW[kk]);
          dv += (rb[Q_V1 + kk - 1] - rfa[Q_V1 + kk - 1]) * dW[kk];
        }
        kdv.add(dv);
      } else {
        const double rr = sqrt(d2);
        if (rr <= 0.0) continue;
        const double f = spline_dw(rr * ih) / rr;
        const double dW[4] = {0.0, (xa[0] - xb[0]) * f, (xa[1] - xb[1]) * f, D == 3 ? (xa[2] - xb[2]) * f : 0.0};
        double rb[NREC];
        for (int q = 0; q < NREC; ++q) {
          if (!VISC && q >= Q_A11 && q <= Q_A33) {
            rb[q] = 0.0;
            continue;
          }
          rb[q] = b.rec[(int64_t)q * cap + k];
        }
        const double pp = ra[Q_PP] + rb[Q_PP];
#pragma unroll
        for (int i = 1; i <= D; ++i) {
          double val = pp * dW[i];
          if (VISC) {
            double vis = 0.0;
#pragma unroll
            for (int jj = 1; jj <= D; ++jj) {
              const int q = Q_A11 + (jj - 1) * 3 + (i - 1);
              vis += (ra[q] + rb[q]) * dW[jj];
            }
            val += Gk[i] * vis;
          }
          F[i] += val;
        }
#pragma unroll
        for (int kk = 1; kk <= D; ++kk) {
#pragma unroll
          for (int nu = 1; nu <= D; ++nu) du[kk][nu] += (rb[Q_U1 + nu - 1] - ra[Q_U1 + nu - 1]) * dW[kk];
          divv += (rb[Q_V1 + kk - 1] - ra[Q_V1 + kk - 1]) * dW[kk];
        }
      }
    }
  }
  if (MIXED) {
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      F[k] = (double)kF[k].s;
#pragma unroll
      for (int n = 1; n < 4; ++n) du[k][n] = (double)kdu[k][n].s;
    }
    divv = (double)kdv.s;
  }
  // restore the kernel normalisation sigma_d / h
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    F[k] *= fsd;
#pragma unroll
    for (int n = 1; n < 4; ++n) du[k][n] *= fsd / sigstar;
  }
  divv *= fsd / sigstar;

  // local equation of motion
  EomIn in;
  in.t = t;
  in.u[0] = 0.0;
  for (int k = 1; k < 4; ++k) in.u[k] = k <= D ? row(Y, cap, R_U1 + k - 1, j) : 0.0;
  const double gam = sqrt(1.0 + in.u[1] * in.u[1] + in.u[2] * in.u[2] + G3 * in.u[3] * in.u[3]);
  in.u[0] = gam;
  for (int k = 0; k < 4; ++k) in.v[k] = in.u[k] / gam;
  for (int k = 1; k < 4; ++k) {
    double acc = 0.0;
    for (int n = 1; n < 4; ++n) {
      in.dudx[k][n] = du[k][n];
      acc += Gk[n] * in.u[n] * du[k][n];
    }
    in.dudx[k][0] = acc / gam;
  }
  for (int n = 0; n < 4; ++n) in.dudx[0][n] = 0.0;
  in.divv = divv;
  for (int k = 0; k < 4; ++k) in.F[k] = F[k];
  const double sqg = sqrt_g(prm, t);
  in.sigma = sigstar / (gam * sqg);
  const double* T_ = b.th;
  in.w = T_[(int64_t)T_E * cap + j] + T_[(int64_t)T_P * cap + j];
  in.Pi = T_[(int64_t)T_PI * cap + j];
  in.T = T_[(int64_t)T_T * cap + j];
  in.cs2 = T_[(int64_t)T_CS2 * cap + j];
  in.kappa = T_[(int64_t)T_KAP * cap + j];
  in.eta = T_[(int64_t)T_ETA * cap + j];
  in.zeta = T_[(int64_t)T_ZETA * cap + j];
  in.taupi = T_[(int64_t)T_TAUPI * cap + j];
  in.tauPi = T_[(int64_t)T_TAUPIB * cap + j];
  for (int m = 0; m < 4; ++m)
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
    for (int i = 1; i < 4; ++i) {
      double acc = 0.0;
      for (int k = 1; k < 4; ++k) acc += Gk[k] * in.u[k] * in.pi[k][i];
      in.pi[0][i] = in.pi[i][0] = acc / gam;
    }
    double acc = 0.0;
    for (int i = 1; i < 4; ++i) acc += Gk[i] * in.u[i] * in.pi[0][i];
    in.pi[0][0] = acc / gam;
  }
  EomOut o;
  eom_solve<D, VISC>(prm, in, o);

  // rates of the 17 state rows
  double f[NROW];
  for (int r = 0; r < NROW; ++r) f[r] = 0.0;
  for (int k = 1; k <= D; ++k) {
    f[R_X1 + k - 1] = in.v[k];
    f[R_U1 + k - 1] = o.a[k];
  }
  f[R_S] = o.dS;
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

  const double dt = E.dt;
  bool finite = true;
  if (mode == 2) {
    const int64_t ii = b.ids[j];
    const int64_t n = E.n;
    for (int r = 0; r < NROW; ++r) fout[(int64_t)r * n + ii] = f[r];
    if (aux) {
      aux[X_THETA * n + ii] = o.theta;
      for (int k = 1; k <= 3; ++k) aux[(X_F1 + k - 1) * n + ii] = F[k];
    }
    return;
  }
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
    for (int w = 0; w < NWARM; ++w) b.warm[(int64_t)w * cap + j] = b.warms[(int64_t)w * cap + j];
  }
  if (!finite) {
    atomicAdd(&b.evt[e].nonfinite, 1u);
    atomicMin(&b.evt[e].first_bad, b.ids[j]);
  }
}

__global__ void k_advance(BatchDev b) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b.max_events || !b.evt[e].active) return;
  b.evt[e].t += b.evt[e].dt;
}

__global__ void k_reset_stage_counters(BatchDev b) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b.max_events) return;
  b.evt[e].backup = 0;
  b.evt[e].newton_iters = 0;
}

// initialisation: S = s gamma sqrt(-g) / sigma*, N likewise (sorted order)
template <int D>
__global__ void __launch_bounds__(256) k_init(BatchDev b, Params prm, EosDev eos, int dens_kind,
                                              const double* __restrict__ dens, int64_t nslots, int only_event) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0 || (only_event >= 0 && e != only_event)) return;
  const EventDev& E = b.evt[e];
  const double t = E.t;
  const int64_t cap = b.cap;
  const double* Y = b.Ys;
  const double h = prm.h, ih = 1.0 / h, r2max = (2.0 * h) * (2.0 * h);
  const double xa[3] = {row(Y, cap, R_X1, j), row(Y, cap, R_X2, j), D == 3 ? row(Y, cap, R_X3, j) : 0.0};
  Block<D> blk;
  neighbour_block<D>(b, E, b.keys[j], blk);
  double ss = 0.0;
  for (int r = 0; r < blk.nr; ++r)
    for (int32_t k = blk.lo[r]; k < blk.hi[r]; ++k) {
      const double xb[3] = {row(Y, cap, R_X1, k), row(Y, cap, R_X2, k), D == 3 ? row(Y, cap, R_X3, k) : 0.0};
      const double d2 = dist2<D>(xa, xb);
      if (d2 < r2max) ss += spline_w(sqrt(d2) * ih);
    }
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
    eos_invert(eos, 1, prm.ncharge, in, nullptr, th);
    if (!th.ok) atomicAdd(&b.evt[e].noconv, 1u);
    s = th.s;
  }
  const double fac = gam * sqrt_g(prm, t) / ss;
  b.Ys[(int64_t)R_S * cap + j] = s * fac;
  for (int q = 0; q < 3; ++q) b.Ys[(int64_t)(R_NB + q) * cap + j] = q < prm.ncharge ? in[1 + q] * fac : 0.0;
  for (int r = R_B; r <= R_P33; ++r) b.Ys[(int64_t)r * cap + j] = 0.0;
  for (int w = 0; w < NWARM; ++w) b.warms[(int64_t)w * cap + j] = 0.0;
}

// debug: pair lists (original ids) of one event; counts first, then fills
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
  Block<D> blk;
  neighbour_block<D>(b, E, b.keys[j], blk);
  for (int r = 0; r < blk.nr; ++r)
    for (int32_t k = blk.lo[r]; k < blk.hi[r]; ++k) {
      const double xb[3] = {row(Y, cap, R_X1, k), row(Y, cap, R_X2, k), D == 3 ? row(Y, cap, R_X3, k) : 0.0};
      if (dist2<D>(xa, xb) < r2max) {
        const int64_t slot = atomicAdd((unsigned long long*)counter, 1ull);
        if (slot < cap_pairs) {
          pa[slot] = b.ids[j];
          pb[slot] = b.ids[k];
        }
      }
    }
}

// state rows of one event in original order
__global__ void __launch_bounds__(256) k_unsort(BatchDev b, int e, uint32_t rowmask, double* out) {
  const EventDev& E = b.evt[e];
  const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (jj >= E.n) return;
  const int64_t j = E.p_base + jj;
  const int64_t ii = b.id[j];
  for (int r = 0; r < NROW; ++r) out[(int64_t)r * E.n + ii] = (rowmask & (1u << r)) ? b.Y0[(int64_t)r * b.cap + j] : 0.0;
}

// state rows of one event from original order into the home slots (ids = identity)
__global__ void __launch_bounds__(256) k_upload(BatchDev b, int e, const double* in, int nrows_given) {
  const EventDev& E = b.evt[e];
  const int64_t ii = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ii >= E.n) return;
  const int64_t j = E.p_base + ii;
  for (int r = 0; r < NROW; ++r) b.Y0[(int64_t)r * b.cap + j] = r < nrows_given ? in[(int64_t)r * E.n + ii] : 0.0;
  for (int w = 0; w < NWARM; ++w) b.warm[(int64_t)w * b.cap + j] = 0.0;
  b.id[j] = (int32_t)ii;
}

// per-event totals: S, NB, NS, NQ, E, M1, M2, M3 (fixed-order reduction)
// E = sum sqrt(-g) T^00 / sigma*, M_i = sum sqrt(-g) G_i T^0i / sigma*, using
// the sorted state Ys and the pass-1 record of the same evaluation
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
      for (int q = 0; q < 3; ++q) acc[1 + q] += row(Y, cap, R_NB + q, j);
      double u[4] = {0.0, row(Y, cap, R_U1, j), row(Y, cap, R_U2, j), prm.dim == 3 ? row(Y, cap, R_U3, j) : 0.0};
      const double gam = sqrt(1.0 + u[1] * u[1] + u[2] * u[2] + G3 * u[3] * u[3]);
      u[0] = gam;
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

// standalone batch inversion (ccake_eos_invert)
__global__ void __launch_bounds__(256) k_eos_invert(EosDev eos, int mode, int nq, int64_t n, const double* in,
                                                    double* out, int32_t* in_table, uint32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v[4] = {in[i], in[n + i], in[2 * n + i], in[3 * n + i]};
  Thermo th;
  eos_invert(eos, mode, nq, v, nullptr, th);
  out[i] = th.T;
  for (int q = 0; q < 3; ++q) out[(1 + q) * n + i] = th.mu[q];
  if (in_table) in_table[i] = th.in_table;
  if (!th.ok && bad) atomicAdd(bad, 1u);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_bin(const BatchDev& b, const Params& prm, int nevents, int64_t nslots, uint32_t rowmask,
                      hipStream_t s, const hipEvent_t* marks) {
  if (nslots <= 0 || nevents <= 0) return hipSuccess;
  if (marks) (void)hipEventRecord(marks[0], s);
  hipLaunchKernelGGL(k_bbox, dim3(nevents), dim3(256), 0, s, b, prm, prm.dim);
  hipLaunchKernelGGL(k_count, dim3(blocks_for(nslots, 256)), dim3(256), 0, s, b, prm.dim, nslots);
  hipLaunchKernelGGL(k_scan, dim3(nevents), dim3(1024), 0, s, b, prm.dim);
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(nslots, 256)), dim3(256), 0, s, b, nslots);
  hipLaunchKernelGGL(k_cellsort, dim3(8, nevents), dim3(256), 0, s, b, prm.dim);
  hipLaunchKernelGGL(k_permute, dim3(blocks_for(nslots, 256)), dim3(256), 0, s, b, nslots, rowmask);
  if (marks) (void)hipEventRecord(marks[1], s);
  return hipGetLastError();
}

template <int D, bool VISC, bool MIXED>
static void launch_passes_t(const BatchDev& b, const Params& prm, const EosDev& eos, int64_t nslots, int which,
                            double* fout, double* aux, hipStream_t s, const hipEvent_t* marks) {
  const unsigned g = blocks_for(nslots, 256);
  if (which == 0) {  // full Heun step
    if (marks) (void)hipEventRecord(marks[0], s);
    hipLaunchKernelGGL((k_pass1<D, VISC, MIXED>), dim3(g), dim3(256), 0, s, b, prm, eos, b.Ys, 0, nslots,
                       (double*)nullptr);
    if (marks) (void)hipEventRecord(marks[1], s);
    hipLaunchKernelGGL((k_pass2<D, VISC, MIXED>), dim3(g), dim3(256), 0, s, b, prm, b.Ys, 0, 0, nslots,
                       (double*)nullptr, (double*)nullptr);
    if (marks) (void)hipEventRecord(marks[2], s);
    hipLaunchKernelGGL((k_pass1<D, VISC, MIXED>), dim3(g), dim3(256), 0, s, b, prm, eos, b.Y1, 1, nslots,
                       (double*)nullptr);
    if (marks) (void)hipEventRecord(marks[3], s);
    hipLaunchKernelGGL((k_pass2<D, VISC, MIXED>), dim3(g), dim3(256), 0, s, b, prm, b.Y1, 1, 1, nslots,
                       (double*)nullptr, (double*)nullptr);
    if (marks) (void)hipEventRecord(marks[4], s);
  } else if (which == 1) {  // right-hand side only, at the sorted state
    hipLaunchKernelGGL((k_pass1<D, VISC, MIXED>), dim3(g), dim3(256), 0, s, b, prm, eos, b.Ys, 0, nslots, aux);
    if (fout)
      hipLaunchKernelGGL((k_pass2<D, VISC, MIXED>), dim3(g), dim3(256), 0, s, b, prm, b.Ys, 0, 2, nslots, fout,
                         aux);
  }
}

hipError_t launch_passes(const BatchDev& b, const Params& prm, const EosDev& eos, int64_t nslots, int which,
                         double* fout, double* aux, hipStream_t s, const hipEvent_t* marks) {
  if (nslots <= 0) return hipSuccess;
  const int key = (prm.dim == 3 ? 4 : 0) + (prm.viscous ? 2 : 0) + (prm.mixed ? 1 : 0);
  switch (key) {
    case 0: launch_passes_t<2, false, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 1: launch_passes_t<2, false, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 2: launch_passes_t<2, true, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 3: launch_passes_t<2, true, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 4: launch_passes_t<3, false, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 5: launch_passes_t<3, false, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 6: launch_passes_t<3, true, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 7: launch_passes_t<3, true, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
  }
  return hipGetLastError();
}

hipError_t launch_advance(const BatchDev& b, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(blocks_for(b.max_events, 64)), dim3(64), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_reset_stage_counters(const BatchDev& b, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_stage_counters, dim3(blocks_for(b.max_events, 64)), dim3(64), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_init(const BatchDev& b, const Params& prm, const EosDev& eos, int dens_kind, const double* dens,
                       int64_t nslots, hipStream_t s, int only_event) {
  const unsigned g = blocks_for(nslots, 256);
  if (g == 0) return hipSuccess;
  if (prm.dim == 3)
    hipLaunchKernelGGL(k_init<3>, dim3(g), dim3(256), 0, s, b, prm, eos, dens_kind, dens, nslots, only_event);
  else
    hipLaunchKernelGGL(k_init<2>, dim3(g), dim3(256), 0, s, b, prm, eos, dens_kind, dens, nslots, only_event);
  return hipGetLastError();
}

hipError_t launch_commit(const BatchDev& b, int64_t nslots, uint32_t rowmask, hipStream_t s) {
  hipLaunchKernelGGL(k_commit, dim3(blocks_for(nslots, 256)), dim3(256), 0, s, b, nslots, rowmask);
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
  hipLaunchKernelGGL(k_eos_invert, dim3(blocks_for(n, 256)), dim3(256), 0, s, eos, mode, nq, n, in, out, in_table,
                     bad);
  return hipGetLastError();
}

}  // namespace ccake

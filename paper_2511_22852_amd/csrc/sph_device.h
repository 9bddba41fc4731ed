// Device helpers shared by the binning and stage kernels: the cubic-spline
// kernel of the paper ("Kernel function"), the exact pair test, compensated
// FP32 accumulation, and the neighbour block of a particle's cell.
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace ccake {

#ifndef CCAKE_PI
#define CCAKE_PI 3.14159265358979323846
#endif

// W = sigma_d w(q), q = r/h: sigma_2 = 10/(7 pi h^2), sigma_3 = 1/(pi h^3)
template <int D>
__device__ __forceinline__ double sigma_d(double h) {
  return D == 2 ? 10.0 / (7.0 * CCAKE_PI * h * h) : 1.0 / (CCAKE_PI * h * h * h);
}

// w(q) = 1 - 3/2 q^2 + 3/4 q^3 (q <= 1), (2 - q)^3 / 4 (1 < q <= 2), 0 beyond.
// Both pieces are evaluated and one is selected (no divergent branches).  The
// polynomials are written in Horner form with explicit fused multiply-adds and
// contraction off elsewhere, so every caller rounds them the same way.
__device__ __forceinline__ double spline_w(double q) {
#pragma clang fp contract(off)
  const double t = 2.0 - q;
  const double inner = fma(q * q, fma(0.75, q, -1.5), 1.0);
  const double outer = (0.25 * t) * (t * t);
  return q <= 1.0 ? inner : (q <= 2.0 ? outer : 0.0);
}

// w'(q) = -3 q + 9/4 q^2 (q <= 1), -3/4 (2 - q)^2 (1 < q <= 2), 0 beyond
__device__ __forceinline__ double spline_dw(double q) {
#pragma clang fp contract(off)
  const double t = 2.0 - q;
  const double inner = q * fma(2.25, q, -3.0);
  const double outer = (-0.75 * t) * t;
  return q <= 1.0 ? inner : (q <= 2.0 ? outer : 0.0);
}

__device__ __forceinline__ float spline_wf(float q) {
#pragma clang fp contract(off)
  const float t = 2.0f - q;
  const float inner = fmaf(q * q, fmaf(0.75f, q, -1.5f), 1.0f);
  const float outer = (0.25f * t) * (t * t);
  return q <= 1.0f ? inner : (q <= 2.0f ? outer : 0.0f);
}

__device__ __forceinline__ float spline_dwf(float q) {
#pragma clang fp contract(off)
  const float t = 2.0f - q;
  const float inner = q * fmaf(2.25f, q, -3.0f);
  const float outer = (-0.75f * t) * t;
  return q <= 1.0f ? inner : (q <= 2.0f ? outer : 0.0f);
}

// Hardware square root and reciprocal square root (about 1 ulp; the FP32
// pair sums carry their own compensated error budget)
__device__ __forceinline__ float fast_sqrtf(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rsqf(float x) { return __builtin_amdgcn_rsqf(x); }

// FP64 reciprocal square root of x > 0: the hardware estimate refined by two
// Newton-Raphson steps y <- y (3 - x y^2) / 2 (each doubles the correct
// bits), to within a few ulp; the FP64 pair sums use r = x y and 1/r = y in
// place of a correctly rounded square root and division (per-term
// differences of a few ulp, far below the parity tolerance of the sums).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x * y;
  y = fma(y, fma(-h, y, 0.5), y);
  h = 0.5 * x * y;
  return fma(y, fma(-h, y, 0.5), y);
}

// Compensated (Kahan) FP32 accumulator; value = s - c.
struct Kahan {
  float s, c;
  __device__ __forceinline__ void add(float x) {
#pragma clang fp contract(off)
    float y = x - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  // add the product a*b, rounded once together with the compensation
  __device__ __forceinline__ void add_prod(float a, float b) {
#pragma clang fp contract(off)
    float y = fmaf(a, b, -c);
    float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ __forceinline__ double value() const { return (double)s - (double)c; }
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

// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// block index.  The hardware index is mapped to a logical one that gives
// every XCD one contiguous share of the cell-sorted particles, so the
// neighbourhoods it reads stay in its own L2: in the plain order every L2
// fetches the whole working set (measured: 12% faster on the FP64
// 1.2 M-particle 3D event; on the 40k-particle 2D event the neighbour-tile
// kernels fetch less from HBM and the step is 0.3% faster).  Bijective.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblocks) {
  const int64_t x = b % NUM_XCD, k = b / NUM_XCD;
  const int64_t q = nblocks / NUM_XCD, r = nblocks % NUM_XCD;
  return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ double row(const double* Y, int64_t cap, int r, int64_t i) {
  return Y[(int64_t)r * cap + i];
}

__device__ __forceinline__ double metric_G3(const Params& prm, double t) { return prm.hyperbolic ? t * t : 1.0; }
__device__ __forceinline__ double sqrt_g(const Params& prm, double t) { return prm.hyperbolic ? t : 1.0; }

// Adds per-lane EoS counters to the event records with one atomic per wave
// when all particles of the wave belong to one event (the common case).
// Every lane of the wave must call it; lanes without a particle pass e = -1.
__device__ inline void wave_count_eos(EventDev* evt, int e, uint32_t backup, uint32_t iters, uint32_t noconv) {
  const unsigned long long m = __ballot(e >= 0);
  if (m == 0) return;
  const int src = __ffsll((unsigned long long)m) - 1;
  const int e0 = __shfl(e, src, 64);
  if (__all(e < 0 || e == e0)) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      backup += __shfl_xor(backup, off, 64);
      iters += __shfl_xor(iters, off, 64);
      noconv += __shfl_xor(noconv, off, 64);
    }
    if ((int)(threadIdx.x & 63) == src) {
      if (backup) atomicAdd(&evt[e0].backup, backup);
      if (iters) atomicAdd(&evt[e0].newton_iters, iters);
      if (noconv) atomicAdd(&evt[e0].noconv, noconv);
    }
  } else if (e >= 0) {
    if (backup) atomicAdd(&evt[e].backup, backup);
    if (iters) atomicAdd(&evt[e].newton_iters, iters);
    if (noconv) atomicAdd(&evt[e].noconv, noconv);
  }
}

// Distance from v to the interval [c0, c0 + e] (zero inside).
__device__ __forceinline__ double interval_gap(double v, double c0, double e) {
  const double below = c0 - v, above = v - (c0 + e);
  return below > 0.0 ? below : (above > 0.0 ? above : 0.0);
}

// Candidate slot ranges of a particle at xa whose binning cell is key: the
// x-rows of cells within subcells(D) cells in y (and z), each row trimmed to the
// cells that intersect the ball of radius reach around xa.  Cells of a row
// are contiguous in slot order (x is the fastest axis of the key), so each
// row is one range [lo, hi).  reach must cover the kernel support plus the
// displacement allowed since binning (the skin); the exact pair test is made
// on every candidate, so the trimming only has to be conservative, which the
// relative margin on reach guarantees against rounding.  f(lo, hi) is called
// for every non-empty row in increasing slot order.
template <int D, class F>
__device__ __forceinline__ void for_each_row(const BatchDev& b, const EventDev& E, int32_t key, const double xa[3],
                                             double reach, F&& f) {
  const int nx = E.nc[0], ny = E.nc[1], nz = D == 3 ? E.nc[2] : 1;
  const int ix = key % nx;
  const int iy = (key / nx) % ny;
  const int iz = D == 3 ? key / (nx * ny) : 0;
  const double e = E.edge, ie = 1.0 / e;
  const double R = reach * (1.0 + 1e-9);
  const double R2 = R * R;
  const int32_t* cs = b.cell_start + E.c_base;
  constexpr int SUB = subcells(D);
  for (int dz = (D == 3 ? -SUB : 0); dz <= (D == 3 ? SUB : 0); ++dz) {
    const int z = iz + dz;
    if (z < 0 || z >= nz) continue;
    const double gz = D == 3 ? interval_gap(xa[2], E.lo[2] + z * e, e) : 0.0;
    for (int dy = -SUB; dy <= SUB; ++dy) {
      const int y = iy + dy;
      if (y < 0 || y >= ny) continue;
      const double gy = interval_gap(xa[1], E.lo[1] + y * e, e);
      const double r2 = R2 - gy * gy - gz * gz;
      if (!(r2 >= 0.0)) continue;
      const double rx = sqrt(r2) * (1.0 + 1e-9);
      int x0 = (int)floor((xa[0] - rx - E.lo[0]) * ie), x1 = (int)floor((xa[0] + rx - E.lo[0]) * ie);
      x0 = max(x0, max(ix - SUB, 0));
      x1 = min(x1, min(ix + SUB, nx - 1));
      if (x0 > x1) continue;
      const int c = (z * ny + y) * nx;
      f(cs[c + x0], cs[c + x1 + 1]);
    }
  }
}

// Team version of for_each_row, with the rows kept in LDS and trimmed in x^1
// to the particle, not just to cells.  Cells are sorted by x^1 inside (and
// ordered by x^1 along a row), so the binning-time coordinates xbin of a
// row's slots increase along it.  A candidate b in row (y, z) can be within
// the support now only if |xbin_b - x_a| <= rx (rx from the row's gap to x_a
// with reach = support + skin: b moved at most half the skin since
// binning), so the row is cut to the slots whose xbin lies in
// [x_a - rx, x_a + rx]; only its first and last cells need a search (binary,
// all searches of a lane interleaved, so they cost one round of dependent
// loads per halving).  Row r of the block (r = (dz + S)(2S + 1) + dy + S) is
// set up by lane r mod L; its slot range is stored at lo[r], hi[r] (empty
// rows as lo = hi).  The team then walks the concatenation of its rows with
// RowCursor below.
template <int D>
struct RowBlock {
  static constexpr int SUB = subcells(D);
  static constexpr int W = 2 * SUB + 1;
  static constexpr int ROWS = D == 3 ? W * W : W;
};

template <int D, int L>
__device__ __forceinline__ void team_rows(const BatchDev& b, const EventDev& E, int32_t key, const double xa[3],
                                          double reach, int lane, int32_t* __restrict__ lo,
                                          int32_t* __restrict__ hi) {
  constexpr int W = RowBlock<D>::W;
  constexpr int ROWS = RowBlock<D>::ROWS;
  constexpr int PER = (ROWS + L - 1) / L;
  const int nx = E.nc[0], ny = E.nc[1], nz = D == 3 ? E.nc[2] : 1;
  const int ix = key % nx;
  const int iy = (key / nx) % ny;
  const int iz = D == 3 ? key / (nx * ny) : 0;
  const double e = E.edge, ie = 1.0 / e;
  const double R = reach * (1.0 + 1e-9);
  const double R2 = R * R;
  const int32_t* cs = b.cell_start + E.c_base;
  // per row of this lane: first cell [s0, e0), last cell [s1, e1), x^1 interval
  int32_t s0[PER], e0[PER], s1[PER], e1[PER];
  double xl[PER], xh[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int r = lane + q * L;
    s0[q] = e0[q] = s1[q] = e1[q] = 0;
    xl[q] = xh[q] = 0.0;
    if (r >= ROWS) continue;
    const int dz = D == 3 ? r / W - RowBlock<D>::SUB : 0, dy = r % W - RowBlock<D>::SUB;
    const int z = iz + dz, y = iy + dy;
    if (z < 0 || z >= nz || y < 0 || y >= ny) continue;
    const double gz = D == 3 ? interval_gap(xa[2], E.lo[2] + z * e, e) : 0.0;
    const double gy = interval_gap(xa[1], E.lo[1] + y * e, e);
    const double r2 = R2 - gy * gy - gz * gz;
    if (!(r2 >= 0.0)) continue;
    const double rx = sqrt(r2) * (1.0 + 1e-9);
    int x0 = (int)floor((xa[0] - rx - E.lo[0]) * ie), x1 = (int)floor((xa[0] + rx - E.lo[0]) * ie);
    x0 = max(x0, max(ix - RowBlock<D>::SUB, 0));
    x1 = min(x1, min(ix + RowBlock<D>::SUB, nx - 1));
    if (x0 > x1) continue;
    const int c = (z * ny + y) * nx;
    s0[q] = cs[c + x0];
    e0[q] = cs[c + x0 + 1];
    s1[q] = cs[c + x1];
    e1[q] = cs[c + x1 + 1];
    xl[q] = xa[0] - rx;
    xh[q] = xa[0] + rx;
  }
  // lower bound of xl in the first cell, upper bound of xh in the last cell
  int32_t f0[PER], n0[PER], f1[PER], n1[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    f0[q] = s0[q];
    n0[q] = e0[q] - s0[q];
    f1[q] = s1[q];
    n1[q] = e1[q] - s1[q];
  }
  for (;;) {
    bool more = false;
#pragma unroll
    for (int q = 0; q < PER; ++q) more = more || n0[q] > 0 || n1[q] > 0;
    if (!more) break;
    double v0[PER], v1[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {  // probes of finished searches read a valid slot and are ignored
      v0[q] = b.xbin[n0[q] > 0 ? f0[q] + (n0[q] >> 1) : 0];
      v1[q] = b.xbin[n1[q] > 0 ? f1[q] + (n1[q] >> 1) : 0];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      if (n0[q] > 0) {
        const int32_t half = n0[q] >> 1;
        if (v0[q] < xl[q]) {
          f0[q] += half + 1;
          n0[q] -= half + 1;
        } else {
          n0[q] = half;
        }
      }
      if (n1[q] > 0) {
        const int32_t half = n1[q] >> 1;
        if (v1[q] <= xh[q]) {
          f1[q] += half + 1;
          n1[q] -= half + 1;
        } else {
          n1[q] = half;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int r = lane + q * L;
    if (r < ROWS) {
      lo[r] = f0[q];
      hi[r] = f1[q];
    }
  }
  // the rows are read back by other lanes of the same wave
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row cache: the density pass stores the team's row bounds of particle j
// (lanes r, r + L, ... write rows r, r + L, ...); later passes read them back
// into their LDS rows instead of searching again.
template <int D, int L>
__device__ __forceinline__ void rows_keep(const BatchDev& b, int64_t j, int lane, const int32_t* lo,
                                           const int32_t* hi) {
  static_assert(2 * RowBlock<D>::ROWS <= ROW_CACHE, "row cache too small");
  for (int r = lane; r < RowBlock<D>::ROWS; r += L) {
    b.rows[(int64_t)(2 * r) * b.cap + j] = lo[r];
    b.rows[(int64_t)(2 * r + 1) * b.cap + j] = hi[r];
  }
}

template <int D, int L>
__device__ __forceinline__ void rows_load(const BatchDev& b, int64_t j, int lane, int32_t* __restrict__ lo,
                                          int32_t* __restrict__ hi) {
  static_assert(2 * RowBlock<D>::ROWS <= ROW_CACHE, "row cache too small");
  for (int r = lane; r < RowBlock<D>::ROWS; r += L) {
    lo[r] = b.rows[(int64_t)(2 * r) * b.cap + j];
    hi[r] = b.rows[(int64_t)(2 * r + 1) * b.cap + j];
  }
  // the rows are read back by other lanes of the same wave
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Walk of one lane of a team over the concatenation of the team's rows: the
// lane takes positions lane, lane + L, lane + 2L, ... of that sequence, so
// that the L lanes together visit every candidate exactly once, each lane in
// increasing slot order.  A step past the end of a row continues in the next
// non-empty row with the overshoot carried.
template <int L, int ROWS>
struct RowCursor {
  const int32_t* lo;
  const int32_t* hi;
  int r;
  int32_t k, h;

  __device__ __forceinline__ void start(const int32_t* lo_, const int32_t* hi_, int lane) {
    lo = lo_;
    hi = hi_;
    r = 0;
    k = lo[0] + lane;
    h = hi[0];
    settle();
  }
  __device__ __forceinline__ void settle() {
    while (k >= h && r + 1 < ROWS) {
      ++r;
      const int32_t over = k - h;
      k = lo[r] + over;
      h = hi[r];
    }
  }
  __device__ __forceinline__ bool valid() const { return k < h; }
  __device__ __forceinline__ int32_t next() {
    const int32_t c = k;
    k += L;
    settle();
    return c;
  }
};

}  // namespace ccake

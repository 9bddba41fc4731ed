// Cell binning of a batch of events: per-event bounding box and grid (cell
// edge >= 2h + skin, the kernel support of "Kernel function" plus the skin
// that keeps stage-2 pairs inside the block), counting sort of the particles
// by cell, then by (x^1, original id) inside each cell.  This is the uniform-grid neighbour
// binning the paper takes from Cabana's VerletList, rebuilt as
//   k_bbox   min/max per event: a few blocks per event reduce its slots, then
//            one atomic per axis and block on order-preserving integer images
//            of the coordinates
//   k_grid   one thread per event: grid origin, cells per axis, reset of the box
//   k_count  particle -> cell key, atomic count per cell
//   k_scan   one block per event: exclusive scan of the counts
//   k_scatter particle -> slot of its cell (arbitrary order within the cell)
//   k_cellsort one wave per cell: rank by (x^1, original id), so the order
//            inside a cell is deterministic and every x-row of cells is
//            sorted by x^1; clears the counts for the next binning
//   k_permute gather of the state, warm starts, ids and keys into cell order,
//            and the binning-time x^1 of every slot
//   k_rows   every slot's neighbour rows, cut to the x^1 interval its
//            particle can reach before the next binning
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "sph_device.h"

namespace ccake {

// k_bbox: blocks (x, e) reduce slices of `per` x 256 slots of event e (an
// event's slots are contiguous), BBOX_BATCH per thread at a time with the
// loads of a batch issued together; one atomic per axis and block on the
// event's box, so an event sees at most gridDim.x atomics per address
constexpr int BBOX_BATCH = 8;

__global__ void __launch_bounds__(256) k_bbox(BatchDev b, int dim, int per) {
  __shared__ double s_lo[4][3], s_hi[4][3];
  const int e = blockIdx.y;
  const EventDev& E = b.evt[e];
  if (!E.active || !E.rebin) return;
  const int64_t first = (int64_t)blockIdx.x * blockDim.x * per;
  if (first >= E.n) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n = E.n, p0 = E.p_base;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int q0 = 0; q0 < per; q0 += BBOX_BATCH) {
    double x[BBOX_BATCH][3];
    bool v[BBOX_BATCH];
#pragma unroll
    for (int u = 0; u < BBOX_BATCH; ++u) {
      const int64_t i = first + (int64_t)(q0 + u) * blockDim.x + threadIdx.x;
      v[u] = q0 + u < per && i < n;
#pragma unroll
      for (int k = 0; k < 3; ++k) x[u][k] = (v[u] && k < dim) ? row(b.Y0, b.cap, R_X1 + k, p0 + i) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < BBOX_BATCH; ++u)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (v[u] && k < dim && isfinite(x[u][k])) {
          lo[k] = fmin(lo[k], x[u][k]);
          hi[k] = fmax(hi[k], x[u][k]);
        }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      lo[k] = fmin(lo[k], __shfl_xor(lo[k], off, 64));
      hi[k] = fmax(hi[k], __shfl_xor(hi[k], off, 64));
    }
  }
  if (lane == 0) {
    for (int k = 0; k < 3; ++k) {
      s_lo[w][k] = lo[k];
      s_hi[w][k] = hi[k];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (int)(blockDim.x >> 6);
    for (int k = 0; k < dim; ++k) {
      double l = s_lo[0][k], h = s_hi[0][k];
      for (int a = 1; a < nw; ++a) {
        l = fmin(l, s_lo[a][k]);
        h = fmax(h, s_hi[a][k]);
      }
      if (isfinite(l)) atomicMin(&b.evt[e].bb_min[k], ordered_bits(l));
      if (isfinite(h)) atomicMax(&b.evt[e].bb_max[k], ordered_bits(h));
    }
  }
}

__global__ void k_grid(BatchDev b, Params prm, int dim) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b.max_events) return;
  EventDev* E = b.evt + e;
  // per-step EoS counters start from zero (the stage kernels add to them)
  E->backup = 0;
  E->newton_iters = 0;
  if (!E->active || !E->rebin) return;
  double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
  bool empty = false;
  for (int k = 0; k < dim; ++k) {
    if (E->bb_min[k] == BB_EMPTY_MIN || E->bb_max[k] == BB_EMPTY_MAX) {
      empty = true;
    } else {
      lo[k] = from_ordered_bits(E->bb_min[k]);
      hi[k] = from_ordered_bits(E->bb_max[k]);
    }
    E->bb_min[k] = BB_EMPTY_MIN;
    E->bb_max[k] = BB_EMPTY_MAX;
  }
  if (empty) {
    for (int k = 0; k < 3; ++k) lo[k] = hi[k] = 0.0;
    if (E->n > 0) E->capacity_err += 1;  // every coordinate non-finite
  }
  double edge = prm.cell_edge / subcells(dim);
  int64_t nc[3] = {1, 1, 1};
  bool fits = false;
  // coarsen the grid (never below the cutoff) until it fits the capacity;
  // cell counts in FP64 so that no extent overflows an integer
  for (int it = 0; it < 64 && !fits; ++it) {
    double tot = 1.0;
    for (int k = 0; k < dim; ++k) tot *= floor((hi[k] - lo[k]) / edge) + 1.0;
    if (tot + 1.0 <= (double)E->c_cap) {
      fits = true;
    } else {
      edge *= 1.25;
    }
  }
  if (fits) {
    for (int k = 0; k < dim; ++k) nc[k] = (int64_t)floor((hi[k] - lo[k]) / edge) + 1;
  } else {
    // one cell that covers the whole event: the pair sums stay complete
    // (every particle is a candidate of every other), the event is flagged
    E->capacity_err += 1;
    double ext = 0.0;
    for (int k = 0; k < dim; ++k) ext = fmax(ext, hi[k] - lo[k]);
    edge = ext + prm.cell_edge;
  }
  for (int k = 0; k < 3; ++k) {
    E->lo[k] = lo[k];
    E->nc[k] = (int32_t)nc[k];
  }
  E->edge = edge;
}

// Runs of equal (event, cell) among the lanes of a wave.  Particles arrive in
// the previous step's cell order, so runs are long and one atomic per run
// replaces one per particle.  Returns the lane of this lane's run head and the
// run length (for the head); lanes with tag < 0 form runs of their own.
__device__ __forceinline__ void wave_runs(int64_t tag, int lane, int* head, int* len) {
  const int64_t prev = __shfl_up(tag, 1, 64);
  const bool is_head = lane == 0 || tag < 0 || prev != tag;
  const unsigned long long heads = __ballot(is_head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  *head = 63 - __clzll((long long)(heads & upto));
  const unsigned long long after = heads & ~upto;
  const int next = after ? __ffsll((long long)after) - 1 : 64;
  *len = next - *head;
}

__global__ void __launch_bounds__(256) k_count(BatchDev b, int dim, int64_t nslots) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int e = i < nslots ? b.ev[i] : -1;
  if (e >= 0 && !b.evt[e].rebin) e = -1;
  int64_t tag = -1;
  int32_t cell = 0;
  if (e >= 0) {
    const EventDev& E = b.evt[e];
    int32_t key = 0, stride = 1;
    for (int k = 0; k < dim; ++k) {
      const double u = (row(b.Y0, b.cap, R_X1 + k, i) - E.lo[k]) / E.edge;
      int c = (int)floor(u);
      c = c < 0 ? 0 : (c >= E.nc[k] ? E.nc[k] - 1 : c);
      key += c * stride;
      stride *= E.nc[k];
    }
    b.key[i] = key;
    cell = E.c_base + key;
    tag = cell;
  }
  int head, len;
  wave_runs(tag, lane, &head, &len);
  if (e >= 0 && head == lane) atomicAdd(&b.cell_fill[cell], len);
}

// exclusive scan of the cell counts of one event (one 1024-thread block per
// event), over tiles of SCAN_TILE cells: each tile is loaded into LDS with
// coalesced loads, every thread scans SCAN_PER consecutive cells, and the
// per-thread totals are scanned across the block (waves by shuffles, then
// the wave totals)
constexpr int SCAN_T = 1024, SCAN_PER = 8, SCAN_TILE = SCAN_T * SCAN_PER;

__global__ void __launch_bounds__(1024) k_scan(BatchDev b, int dim) {
  const int e = blockIdx.x;
  const EventDev& E = b.evt[e];
  if (!E.active || !E.rebin) return;
  int64_t ncell = 1;
  for (int k = 0; k < dim; ++k) ncell *= E.nc[k];
  __shared__ int32_t s_c[SCAN_TILE];
  __shared__ int32_t s_w[SCAN_T / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int32_t* cf = b.cell_fill + E.c_base;
  int32_t* cs = b.cell_start + E.c_base;
  int32_t run = (int32_t)E.p_base;  // slot of the first cell of the tile
  for (int64_t t0 = 0; t0 < ncell; t0 += SCAN_TILE) {
    const int n = (int)min((int64_t)SCAN_TILE, ncell - t0);
    int32_t v[SCAN_PER];
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
      const int c = q * SCAN_T + t;
      v[q] = c < n ? cf[t0 + c] : 0;
    }
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) s_c[q * SCAN_T + t] = v[q];
    __syncthreads();
    int32_t mine[SCAN_PER], sum = 0;
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
      mine[q] = s_c[t * SCAN_PER + q];
      sum += mine[q];
    }
    // inclusive scan of the thread sums within the wave
    int32_t inc = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t y = __shfl_up(inc, off, 64);
      if (lane >= off) inc += y;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int a = 0; a < SCAN_T / 64; ++a) {
      const int32_t x = s_w[a];
      before += a < w ? x : 0;
      total += x;
    }
    int32_t r = run + before + inc - sum;
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
      const int64_t c = t0 + (int64_t)t * SCAN_PER + q;
      if (c < t0 + n) {
        cs[c] = r;
        cf[c] = r;  // becomes the scatter cursor
      }
      r += mine[q];
    }
    run += total;
    __syncthreads();  // s_c and s_w are reused by the next tile
  }
  if (threadIdx.x == 0) cs[ncell] = (int32_t)(E.p_base + E.n);
}

__global__ void __launch_bounds__(256) k_scatter(BatchDev b, int64_t nslots) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int e = i < nslots ? b.ev[i] : -1;
  if (e >= 0 && !b.evt[e].rebin) e = -1;
  const int32_t cell = e >= 0 ? b.evt[e].c_base + b.key[i] : 0;
  int head, len;
  wave_runs(e >= 0 ? (int64_t)cell : -1, lane, &head, &len);
  // the run head reserves len slots; the order inside a cell is fixed later
  int32_t base = 0;
  if (e >= 0 && head == lane) base = atomicAdd(&b.cell_fill[cell], len);
  base = __shfl(base, head, 64);
  if (e >= 0) b.perm[base + (lane - head)] = (int32_t)i;
}

// one wave per cell: the rank of each member is the number of members with a
// smaller (x^1 at binning, original id) key (ids are unique within an event)
constexpr int SORT_CAP = 1024;  // members per cell held in LDS by one wave
// sort key inside a cell: binning-time x^1 (total order on the bits), then id
struct CellKey {
  unsigned long long x;
  int32_t id;
  __device__ __forceinline__ bool operator<(const CellKey& o) const { return x < o.x || (x == o.x && id < o.id); }
};
__device__ __forceinline__ CellKey cell_key(const BatchDev& b, int32_t p) {
  return CellKey{ordered_bits(b.Y0[(int64_t)R_X1 * b.cap + p]), b.id[p]};
}

__global__ void __launch_bounds__(256) k_cellsort(BatchDev b, int dim) {
  __shared__ unsigned long long s_x[4][SORT_CAP];
  __shared__ int32_t s_id[4][SORT_CAP];
  __shared__ int32_t s_p[4][SORT_CAP];
  const int e = blockIdx.y;
  const EventDev& E = b.evt[e];
  if (!E.active || !E.rebin) return;
  int64_t ncell = 1;
  for (int k = 0; k < dim; ++k) ncell *= E.nc[k];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t* cs = b.cell_start + E.c_base;
  int32_t* cf = b.cell_fill + E.c_base;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t c = (int64_t)blockIdx.x * 4 + w; c < ncell; c += nwaves) {
    const int32_t s = cs[c], m = cs[c + 1] - s;
    if (lane == 0) cf[c] = 0;
    if (m <= 1) continue;
    if (m <= SORT_CAP) {
      for (int k = lane; k < m; k += 64) {
        const int32_t p = b.perm[s + k];
        const CellKey key = cell_key(b, p);
        s_p[w][k] = p;
        s_x[w][k] = key.x;
        s_id[w][k] = key.id;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      for (int k = lane; k < m; k += 64) {
        const CellKey mine{s_x[w][k], s_id[w][k]};
        int rank = 0;
        for (int q = 0; q < m; ++q) rank += CellKey{s_x[w][q], s_id[w][q]} < mine ? 1 : 0;
        b.perm[s + rank] = s_p[w][k];
      }
      __builtin_amdgcn_wave_barrier();
    } else if (!E.nonfinite) {
      // oversized cell (a degenerate grid): the lanes rank the members
      // against all others in global memory (m^2 / 64 comparisons per lane)
      // into the sorted-key array, which is free until the gather, then
      // copy back.  An event already flagged non-finite is left unsorted:
      // its results are void, and its positions may all share one cell.
      for (int k = lane; k < m; k += 64) {
        const int32_t p = b.perm[s + k];
        const CellKey mine = cell_key(b, p);
        int rank = 0;
        for (int q = 0; q < m; ++q) rank += cell_key(b, b.perm[s + q]) < mine ? 1 : 0;
        b.keys[s + rank] = p;
      }
      __threadfence();
      __builtin_amdgcn_wave_barrier();
      for (int k = lane; k < m; k += 64) b.perm[s + k] = b.keys[s + k];
      __threadfence();
      __builtin_amdgcn_wave_barrier();
    }
  }
}

__global__ void __launch_bounds__(256) k_permute(BatchDev b, int64_t nslots, uint32_t rowmask) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0) return;
  // events that keep their cells are already in cell order: plain copy
  const bool moved = b.evt[e].rebin != 0;
  const int64_t src = moved ? b.perm[j] : j;
  for (int r = 0; r < NROW; ++r)
    if (rowmask & (1u << r)) b.Ys[(int64_t)r * b.cap + j] = b.Y0[(int64_t)r * b.cap + src];
  for (int w = 0; w < NWARM; ++w) b.warms[(int64_t)w * b.cap + j] = b.warm[(int64_t)w * b.cap + src];
  b.ids[j] = b.id[src];
  if (moved) {
    b.keys[j] = b.key[src];
    b.xbin[j] = b.Y0[(int64_t)R_X1 * b.cap + src];
  }
}

// Neighbour rows of every slot of the events this step bins, at the
// binning-time positions (team_rows: a team of ROW_TEAM lanes per slot), for
// the pair kernels of every stage until the next binning.
constexpr int ROW_TEAM = 16;

template <int D>
__global__ void __launch_bounds__(256) k_rows(BatchDev b, Params prm, int64_t nslots) {
  constexpr int ROWS = RowBlock<D>::ROWS;
  constexpr int PER_BLOCK = 256 / ROW_TEAM;
  __shared__ int32_t s_lo[PER_BLOCK][ROWS], s_hi[PER_BLOCK][ROWS];
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = tid / ROW_TEAM;
  const int lane = (int)(tid % ROW_TEAM), team = (int)threadIdx.x / ROW_TEAM;
  // a team lies inside one wave and leaves as a whole
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0 || !b.evt[e].rebin) return;
  const EventDev& E = b.evt[e];
  const int64_t cap = b.cap;
  const double xa[3] = {row(b.Ys, cap, R_X1, j), row(b.Ys, cap, R_X2, j), D == 3 ? row(b.Ys, cap, R_X3, j) : 0.0};
  team_rows<D, ROW_TEAM>(b, E, b.keys[j], xa, prm.cell_edge, lane, s_lo[team], s_hi[team]);
  rows_keep<D, ROW_TEAM>(b, j, lane, s_lo[team], s_hi[team]);
}

// sorted -> home (after an initialisation)
__global__ void __launch_bounds__(256) k_commit(BatchDev b, int64_t nslots, uint32_t rowmask) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslots || b.ev[j] < 0) return;
  for (int r = 0; r < NROW; ++r)
    if (rowmask & (1u << r)) b.Y0[(int64_t)r * b.cap + j] = b.Ys[(int64_t)r * b.cap + j];
  for (int w = 0; w < NWARM; ++w) b.warm[(int64_t)w * b.cap + j] = b.warms[(int64_t)w * b.cap + j];
  b.id[j] = b.ids[j];
}

// Per-event rebinning schedule of a batch step: an event is binned when it
// is fresh or when twice its displacement bound since the last binning would
// exceed the skin after this step (the same rule a single simulation applies
// on the host).
__global__ void k_schedule(BatchDev b, double skin, int hyper3d) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b.max_events) return;
  EventDev* E = b.evt + e;
  if (!E->active) {
    E->rebin = 0;
    return;
  }
  const double vmax = hyper3d ? fmax(1.0, 1.0 / E->t) : 1.0;
  const double d = E->dt * vmax;
  const int rebin = E->need_bin || 2.0 * (E->disp + d) > skin;
  if (rebin) E->disp = 0.0;
  E->disp += d;
  E->need_bin = 0;
  E->rebin = rebin;
}

// only event e is binned by the next launch_bin (admission of a new event)
__global__ void k_bin_only(BatchDev b, int only) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b.max_events) return;
  b.evt[e].rebin = e == only ? 1 : 0;
}

static inline unsigned blocks_of(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_schedule(const BatchDev& b, double skin, bool hyper3d, hipStream_t s) {
  hipLaunchKernelGGL(k_schedule, dim3(blocks_of(b.max_events, 64)), dim3(64), 0, s, b, skin, hyper3d ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_bin_only(const BatchDev& b, int e, hipStream_t s) {
  hipLaunchKernelGGL(k_bin_only, dim3(blocks_of(b.max_events, 64)), dim3(64), 0, s, b, e);
  return hipGetLastError();
}

hipError_t launch_bin(const BatchDev& b, const Params& prm, int nevents, int64_t nslots, int64_t max_event_n,
                      uint32_t rowmask, hipStream_t s, const hipEvent_t* marks) {
  if (nslots <= 0 || nevents <= 0) return hipSuccess;
  if (marks) (void)hipEventRecord(marks[0], s);
  // about 16 blocks per event (at most 64 batches of slots per thread)
  const int64_t mx = std::max<int64_t>(1, std::min(max_event_n, nslots));
  const int per = (int)std::min<int64_t>(std::max<int64_t>((mx + 256 * 16 - 1) / (256 * 16), BBOX_BATCH), 64);
  hipLaunchKernelGGL(k_bbox, dim3(blocks_of(mx, 256 * per), nevents), dim3(256), 0, s, b, prm.dim, per);
  hipLaunchKernelGGL(k_grid, dim3(blocks_of(nevents, 64)), dim3(64), 0, s, b, prm, prm.dim);
  hipLaunchKernelGGL(k_count, dim3(blocks_of(nslots, 256)), dim3(256), 0, s, b, prm.dim, nslots);
  hipLaunchKernelGGL(k_scan, dim3(nevents), dim3(1024), 0, s, b, prm.dim);
  hipLaunchKernelGGL(k_scatter, dim3(blocks_of(nslots, 256)), dim3(256), 0, s, b, nslots);
  // enough waves for one cell each on a 40k-particle event, grid-stride beyond
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(512, nslots / (nevents * 64) + 1));
  hipLaunchKernelGGL(k_cellsort, dim3(gx, nevents), dim3(256), 0, s, b, prm.dim);
  hipLaunchKernelGGL(k_permute, dim3(blocks_of(nslots, 256)), dim3(256), 0, s, b, nslots, rowmask);
  if (prm.dim == 3)
    hipLaunchKernelGGL(k_rows<3>, dim3(blocks_of(nslots * ROW_TEAM, 256)), dim3(256), 0, s, b, prm, nslots);
  else
    hipLaunchKernelGGL(k_rows<2>, dim3(blocks_of(nslots * ROW_TEAM, 256)), dim3(256), 0, s, b, prm, nslots);
  if (marks) (void)hipEventRecord(marks[1], s);
  return hipGetLastError();
}

hipError_t launch_commit(const BatchDev& b, int64_t nslots, uint32_t rowmask, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_commit, dim3(blocks_of(nslots, 256)), dim3(256), 0, s, b, nslots, rowmask);
  return hipGetLastError();
}

}  // namespace ccake

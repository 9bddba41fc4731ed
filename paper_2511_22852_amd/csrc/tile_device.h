// Neighbour tiles of the pair kernels: each workgroup takes P = 256 / L
// consecutive slots (targets, one team of L lanes each), stages the union of
// their neighbour rows in LDS once, and lets every team walk its own
// candidates from LDS.
//
//   * Targets are sorted by cell, and inside an x-row of cells by
//     binning-time x^1, so the targets of a workgroup that share a cell row
//     (a "segment": same event, same cell row) have the same physical
//     neighbour rows, each cut to the x-interval its particle can reach.
//     The segment's halo in row r is the slot range [min lo_r, max hi_r) over
//     its targets: contiguous, because a row's slots are contiguous.
//   * The halos of all segments and rows are numbered consecutively (halo
//     index space); a target's candidate ranges are its row ranges shifted
//     into that space.  When the halo does not fit in the LDS buffers
//     (capacity C candidates) it is processed in chunks of C, and each team
//     walks the part of its ranges inside the chunk.
//   * The per-target row ranges come from the row cache that the binning
//     step fills (searched once per binning at binning-time positions); the
//     pair test at the current positions selects the pairs.
//
// The team sums are independent of the tiling: every candidate of a target
// is visited by the same lane in the same order whatever the chunking, since
// chunks cut the concatenated range sequence without reordering it and a
// lane's position in that sequence (lane, lane + L, ...) does not depend on
// where the chunk boundaries fall.
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"
#include "sph_device.h"

namespace ccake {

// LDS set-up arrays of one workgroup
template <int D, int P>
struct TileShared {
  static constexpr int ROWS = RowBlock<D>::ROWS;
  static constexpr int NENT = P * ROWS;  // (segment, row) entries, segment-major
  int32_t lo[P][ROWS], hi[P][ROWS];      // per target: halo-index range of each row
  int32_t glo[NENT], ghi[NENT];          // per entry: slot range (ghi <= glo: empty)
  int32_t base[NENT + 1];                // per entry: first halo index
  int32_t seg[P];                        // segment of each target (-1: none)
  int32_t cnt[P];                        // candidates of each target
  int32_t perm[P];                       // target of each team (walk order, with TeamSort)
  int64_t key[P];                        // segment key of each target
  int32_t nseg, total;
  int32_t wsum[4];                       // scan scratch (one per wave)
};

// The targets of workgroup t of the pair kernels: slots [j0, jend) of event
// e.  The workgroups of an event are consecutive, starting at its tile0, and
// each takes P slots counted from the event's first slot, so a particle's
// workgroup and its companions do not depend on where the event sits in a
// batch.  False when workgroup t has no targets.
template <int P>
__device__ __forceinline__ bool tile_targets(const BatchDev& b, int64_t t, int& e, int64_t& j0, int64_t& jend) {
  int m = 0;
  if (b.max_events > 1) {
    // last event whose first workgroup is at or before t
    int n = b.max_events;
    while (n > 1) {
      const int half = n >> 1;
      if ((int64_t)b.evt[m + half].tile0 <= t) {
        m += half;
        n -= half;
      } else {
        n = half;
      }
    }
  }
  const EventDev& E = b.evt[m];
  const int64_t rel = t - E.tile0;
  if (!E.active || rel < 0 || rel * P >= E.n) return false;
  e = m;
  j0 = E.p_base + rel * P;
  jend = E.p_base + E.n;
  return true;
}

// Segment key of slot j of event E: the global cell index of the first cell
// of its cell row (rows of different events never share a key), -1 for no
// target.  Every slot of an active event's range [p_base, p_base + n) holds
// one of its particles, so a tile's targets need no slot-to-event lookup.
__device__ __forceinline__ int64_t tile_segkey(const BatchDev& b, const EventDev& E, int64_t j, int64_t jend) {
  if (j >= jend) return -1;
  const int32_t key = b.keys[j];
  return (int64_t)E.c_base + key - key % E.nc[0];
}

// Teams take the workgroup's targets in order of decreasing candidate count
// (1) or in slot order (0), in 2+1D and 3+1D.  The ranking costs a barrier
// in the set-up: in 3+1D, where the workgroups queue up on each CU and the
// pair passes run at the issue limit, the lanes it saves pay for it; the
// 2+1D passes run in a single round of workgroups and wait on latency.
#ifndef CCAKE_TEAM_SORT2
#define CCAKE_TEAM_SORT2 0
#endif
#ifndef CCAKE_TEAM_SORT3
#define CCAKE_TEAM_SORT3 1
#endif
template <int D>
struct TeamSort {
  static constexpr bool ON = (D == 3 ? CCAKE_TEAM_SORT3 : CCAKE_TEAM_SORT2) != 0;
};

// Set-up of a tile of event ev0: segments, halos, halo bases and the targets'
// ranges in halo index space.  Every thread of the workgroup must call it.  Team t owns
// threads [t L, (t + 1) L); it sets up target j0 + t (if below jend) and then
// walks target j0 + perm[t] (with TeamSort<D>::ON; else target j0 + t), so
// that the teams of a wave, which run in lock step, walk candidate lists of
// similar length.  Returns the halo size.
template <int D, int L, int P>
__device__ __forceinline__ int32_t tile_setup(const BatchDev& b, int ev0, int64_t j0, int64_t jend,
                                              TileShared<D, P>& S) {
  constexpr int ROWS = RowBlock<D>::ROWS;
  constexpr int NENT = P * ROWS;
  const int tid = threadIdx.x, t = tid / L, lane = tid % L;
  const int64_t j = j0 + t;
  // the target's cached rows (slot ranges), loaded first so that their
  // latency overlaps the segment numbering; a slot beyond the event's last
  // has none
  constexpr int RL = (ROWS + L - 1) / L;
  int32_t rlo[RL], rhi[RL];
#pragma unroll
  for (int k = 0; k < RL; ++k) {
    const int r = lane + k * L;
    const bool ld = r < ROWS && j < jend;
    rlo[k] = ld ? b.rows[(int64_t)(2 * r) * b.cap + j] : 0;
    rhi[k] = ld ? b.rows[(int64_t)(2 * r + 1) * b.cap + j] : 0;
  }
  // 1. segment keys, then segment numbers by a prefix count of the boundaries
  if (lane == 0) S.key[t] = tile_segkey(b, b.evt[ev0], j, jend);
  for (int q = tid; q < NENT; q += 256) {
    S.glo[q] = INT32_MAX;
    S.ghi[q] = INT32_MIN;
  }
  __syncthreads();
  if (tid < 64) {
    const bool have = tid < P && S.key[tid] >= 0;
    const bool head = have && (tid == 0 || S.key[tid - 1] != S.key[tid]);
    const unsigned long long heads = __ballot(head);
    const unsigned long long below = tid == 0 ? 0ull : (heads & ((1ull << tid) - 1ull));
    const int s = __popcll(below) + (head ? 1 : 0) - 1;
    if (tid < P) S.seg[tid] = have ? s : -1;
    if (tid == 0) S.nseg = __popcll(heads);
  }
  __syncthreads();
  // 2. the segment halos
  const int sg = S.seg[t];
#pragma unroll
  for (int k = 0; k < RL; ++k) {
    const int r = lane + k * L;
    if (r >= ROWS) break;
    int32_t lo = 0, hi = 0;
    if (sg >= 0) {
      lo = rlo[k];
      hi = rhi[k];
      if (hi > lo) {
        atomicMin(&S.glo[sg * ROWS + r], lo);
        atomicMax(&S.ghi[sg * ROWS + r], hi);
      }
    }
    S.lo[t][r] = lo;
    S.hi[t][r] = hi;
  }
  __syncthreads();
  // 3. exclusive scan of the entry lengths (entries of nseg segments), each
  //    thread over a run of consecutive entries, then across the workgroup
  const int nent = S.nseg * ROWS;
  constexpr int PER = (NENT + 255) / 256;
  int32_t len[PER], sum = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid * PER + q;
    len[q] = (e < nent && S.ghi[e] > S.glo[e]) ? S.ghi[e] - S.glo[e] : 0;
    sum += len[q];
  }
  int32_t inc = sum;
  const int wl = tid & 63, w = tid >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(inc, off, 64);
    if (wl >= off) inc += y;
  }
  if (wl == 63) S.wsum[w] = inc;
  __syncthreads();
  int32_t before = 0, total = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    before += a < w ? S.wsum[a] : 0;
    total += S.wsum[a];
  }
  int32_t run = before + inc - sum;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid * PER + q;
    if (e < NENT) S.base[e] = run;
    run += len[q];
  }
  if (tid == 0) {
    S.base[NENT] = total;
    S.total = total;
  }
  __syncthreads();
  // 4. the target's ranges in halo index space
  for (int r = lane; r < ROWS; r += L) {
    const int32_t lo = S.lo[t][r], hi = S.hi[t][r];
    if (sg >= 0 && hi > lo) {
      const int e = sg * ROWS + r;
      S.lo[t][r] = lo - S.glo[e] + S.base[e];
      S.hi[t][r] = hi - S.glo[e] + S.base[e];
    } else {
      S.lo[t][r] = S.hi[t][r] = 0;
    }
  }
  __syncthreads();
  // 5. the walk order: targets ranked by candidate count, largest first (ties
  //    by slot); targets without a segment have none and come last
  if (TeamSort<D>::ON) {
    if (tid < P) {
      int32_t c = 0;
#pragma unroll
      for (int r = 0; r < ROWS; ++r) c += S.hi[tid][r] - S.lo[tid][r];
      S.cnt[tid] = c;
    }
    __syncthreads();
    if (tid < P) {
      const int32_t c = S.cnt[tid];
      int rank = 0;
      for (int u = 0; u < P; ++u) {
        const int32_t cu = S.cnt[u];
        rank += (cu > c || (cu == c && u < tid)) ? 1 : 0;
      }
      S.perm[rank] = tid;
    }
    __syncthreads();
  }
  return total;
}

// Slot of halo index x (x < total): the entry holding x is found from the
// hint e (an entry at or before it), and returned through e for the next,
// larger x.
template <int D, int P>
__device__ __forceinline__ int32_t tile_slot(const TileShared<D, P>& S, int32_t x, int& e) {
  while (S.base[e + 1] <= x) ++e;
  return S.glo[e] + (x - S.base[e]);
}

// Entry holding halo index x, by bisection over the nondecreasing bases.
template <int D, int P>
__device__ __forceinline__ int tile_entry(const TileShared<D, P>& S, int32_t x) {
  int a = 0, n = S.nseg * RowBlock<D>::ROWS;
  while (n > 1) {
    const int half = n >> 1;
    if (S.base[a + half] <= x) {
      a += half;
      n -= half;
    } else {
      n = half;
    }
  }
  return a;
}

// Walk of one lane over its team's ranges (halo index space), chunk by
// chunk: the lane takes positions lane, lane + L, lane + 2L, ... of the
// concatenation of the ranges (a step past the end of a range continues in
// the next non-empty one with the overshoot carried), and stops at the end
// of the current chunk [c0, c1); the next chunk continues from there.  The
// ranges increase with the row, so the walk's halo indices increase and a
// lane visits the same candidates in the same order whatever the chunking.
template <int L, int ROWS>
struct TileCursor {
  const int32_t* lo;
  const int32_t* hi;
  int32_t c0, c1;
  int r;
  int32_t k, h;

  __device__ __forceinline__ void start(const int32_t* lo_, const int32_t* hi_, int32_t pos) {
    lo = lo_;
    hi = hi_;
    c0 = 0;
    c1 = 0;
    r = 0;
    k = lo[0] + pos;
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
  // the next chunk; the walk stopped at or beyond the end of the previous one
  __device__ __forceinline__ void chunk(int32_t c0_, int32_t c1_) {
    c0 = c0_;
    c1 = c1_;
  }
  __device__ __forceinline__ bool valid() const { return k < h && k < c1; }
  // chunk-local index of the lane's next candidate
  __device__ __forceinline__ int32_t next() {
    const int32_t c = k - c0;
    k += L;
    settle();
    return c;
  }
};

// FP64 team sums through LDS for any number of values: lane k of the team
// stores its NV partials at buf[k * NV + v]; lane v adds value v (and v + L,
// v + 2L, ...) of the L lanes in lane order.  out[q] holds value lane + q L.
template <int L, int NV>
__device__ __forceinline__ void team_sums_lds_n(double* __restrict__ buf, int lane, const double (&v)[NV],
                                                double (&out)[(NV + L - 1) / L]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int q = 0; q < NV; ++q) buf[lane * NV + q] = v[q];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int q = 0; q < (NV + L - 1) / L; ++q) {
    const int vv = lane + q * L;
    double acc = 0.0;
    if (vv < NV) {
#pragma unroll
      for (int k = 0; k < L; ++k) acc += buf[k * NV + vv];
    }
    out[q] = acc;
  }
}

}  // namespace ccake

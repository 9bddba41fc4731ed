// One Runge-Kutta stage of the SPH update, as four kernels:
//
//   k_density  team of L lanes per particle: sigma*_a = sum_b W_ab and, for
//              the smoothed density form, s*_a = sum_b S_b W_ab and
//              n*_a = sum_b N_b W_ab ("SPH interpretation of a fluid element")
//   k_eos      one thread per particle: rest-frame densities, EoS inversion
//              (online inverter), transport coefficients, dissipative tensors,
//              the neighbour record of pass 2
//   k_grad     team of L lanes per particle: n = -1 force sums of p + Pi and
//              of the viscous tensor, n = 1 sums of d_k u^j and div v
//              ("Derivatives in relativistic SPH"); with BSQ diffusion also
//              d_k (mu/T) and the n = -1 flux sums of the currents
//   k_eom      one thread per particle: local M du/dx0 = F solve, relaxation
//              rates, Heun update
//
// The two pair kernels work on neighbour tiles (tile_device.h): a workgroup
// takes 256 / L consecutive slots, stages the union of their neighbour rows
// (positions and the operands of the sums) in LDS with coalesced loads, and
// each team of L lanes walks its own candidates from there, lane k taking
// every L-th candidate of the particle's rows, U at a time.  Rejected
// candidates add zero.  The lanes' partial sums are combined in a fixed
// order through LDS (lane v adds value v of the team's lanes in lane order),
// so the result is deterministic and independent of the batch.  In mixed
// precision the pair terms are formed and accumulated in FP32 with Kahan
// compensation per lane, and the lanes' partials are merged in FP64; the pair
// test itself is always the exact FP64 one.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "eom_device.h"
#include "eos_device.h"
#include "kernels.h"
#include "pair_device.h"
#include "sph_device.h"
#include "tile_device.h"

namespace ccake {

// lanes per particle in the pair loops (2D, 3D)
#ifndef CCAKE_TEAM2
#define CCAKE_TEAM2 8
#endif
#ifndef CCAKE_TEAM3
#define CCAKE_TEAM3 8
#endif
template <int D>
struct Team {
  static constexpr int L = D == 2 ? CCAKE_TEAM2 : CCAKE_TEAM3;
  static constexpr int P = 256 / L;  // particles per workgroup
  static_assert(L >= 4 && L <= 64 && (L & (L - 1)) == 0, "team of 4 to 64 lanes");
};
// candidates per lane in flight in the pair loops (2D, 3D)
#ifndef CCAKE_PAIR_U2
#define CCAKE_PAIR_U2 2
#endif
#ifndef CCAKE_PAIR_U3
#define CCAKE_PAIR_U3 2
#endif
template <int D>
struct PairU {
  static constexpr int U = D == 2 ? CCAKE_PAIR_U2 : CCAKE_PAIR_U3;
};
// LDS bytes of the staged candidates of a workgroup of the density and the
// gradient pass (2D, 3D); the chunk size follows from the bytes a candidate
// takes.  The 2D halos of a workgroup hold about 400 candidates.
#ifndef CCAKE_DENS_BYTES2
#define CCAKE_DENS_BYTES2 16384
#endif
#ifndef CCAKE_GRAD_BYTES2
#define CCAKE_GRAD_BYTES2 24576
#endif
#ifndef CCAKE_DENS_BYTES3
#define CCAKE_DENS_BYTES3 24576
#endif
#ifndef CCAKE_GRAD_BYTES3
#define CCAKE_GRAD_BYTES3 32768
#endif
template <int D>
struct TileBytes {
  static constexpr int DENS = D == 2 ? CCAKE_DENS_BYTES2 : CCAKE_DENS_BYTES3;
  static constexpr int GRAD = D == 2 ? CCAKE_GRAD_BYTES2 : CCAKE_GRAD_BYTES3;
};

// four operands of a candidate in LDS: one 16-byte load in FP32, two in FP64
template <bool MIXED>
struct Quad;
template <>
struct Quad<true> {
  float4 v;
  template <class T>
  __device__ __forceinline__ void put(T a0, T a1, T a2, T a3) {
    v = make_float4((float)a0, (float)a1, (float)a2, (float)a3);
  }
  __device__ __forceinline__ void get(float* o) const {
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};
template <>
struct Quad<false> {
  double2 a, b;
  template <class T>
  __device__ __forceinline__ void put(T a0, T a1, T a2, T a3) {
    a = make_double2((double)a0, (double)a1);
    b = make_double2((double)a2, (double)a3);
  }
  __device__ __forceinline__ void get(double* o) const {
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
  }
};

// LDS halo of a pair kernel: C candidates with their positions (x^1, x^2 as
// one 16-byte pair, x^3 apart), G quads of operands and, when SLOTS, their
// slots, C as many as fit in BUDGET bytes (a multiple of 64); the memory is
// reused for the team sums (NRED values per lane) after the last chunk.
template <int D, bool MIXED, int G, bool SLOTS, int NRED, int BUDGET>
struct Halo {
  static constexpr int PER = 16 + (D == 3 ? 8 : 0) + (int)sizeof(Quad<MIXED>) * G + (SLOTS ? 4 : 0);
  static constexpr int C = (BUDGET / PER) & ~63;
  static_assert(C >= 64, "LDS budget below 64 candidates");
  static constexpr size_t XY = 16 * (size_t)C;
  static constexpr size_t Z = D == 3 ? 8 * (size_t)C : 0;
  static constexpr size_t Q = sizeof(Quad<MIXED>) * (size_t)C * G;
  static constexpr size_t SL = SLOTS ? 4 * (size_t)C : 0;
  static constexpr size_t DATA = XY + Z + Q + SL;
  static constexpr size_t RED = 8 * (size_t)256 * NRED;
  static constexpr size_t BYTES = DATA > RED ? DATA : RED;
  char* m;
  __device__ __forceinline__ double2* xy() const { return (double2*)m; }
  __device__ __forceinline__ double* z() const { return (double*)(m + XY); }
  __device__ __forceinline__ Quad<MIXED>* q(int g) const { return (Quad<MIXED>*)(m + XY + Z) + (size_t)g * C; }
  __device__ __forceinline__ int32_t* slot() const { return (int32_t*)(m + XY + Z + Q); }
  __device__ __forceinline__ double* red() const { return (double*)m; }
};

// Cooperative load of the halo indices [c0, c1) into the LDS halo: thread
// i takes indices c0 + i, c0 + i + 256, ...; positions from the state Y,
// operands through operands(slot, quads) (G quads in the precision of the
// sums).
template <int D, bool MIXED, int G, bool SLOTS, int NRED, int BUDGET, int P, class F>
__device__ __forceinline__ void halo_load(const Halo<D, MIXED, G, SLOTS, NRED, BUDGET>& H, const TileShared<D, P>& S,
                                          const double* __restrict__ Y, int64_t cap, int32_t c0, int32_t c1,
                                          F&& operands) {
  int32_t x = c0 + (int32_t)threadIdx.x;
  if (x >= c1) return;
  int e = tile_entry(S, x);
  for (; x < c1; x += 256) {
    const int32_t sl = tile_slot(S, x, e);
    const int32_t i = x - c0;
    H.xy()[i] = make_double2(Y[(int64_t)R_X1 * cap + sl], Y[(int64_t)R_X2 * cap + sl]);
    if (D == 3) H.z()[i] = Y[(int64_t)R_X3 * cap + sl];
    operands(sl, &H.q(0)[i], (size_t)H.C);
    if (SLOTS) H.slot()[i] = sl;
  }
}

// Debug export of the pairs a pass accepts (original ids), or none.
struct PairExport {
  int64_t* counter;  // nullptr: no export
  int64_t cap;
  int32_t* a;
  int32_t* b;
};

// Takes this lane's next U candidates from the cursor (chunk-local LDS
// indices); missing ones point at index 0, a loaded candidate, and are
// flagged invalid.
template <int U, class Cursor>
__device__ __forceinline__ void take(Cursor& cur, int32_t k[U], bool v[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    v[u] = cur.valid();
    k[u] = 0;
    if (v[u]) k[u] = cur.next();
  }
}

// ---------------------------------------------------------------------------
// NS: smoothed scalars per neighbour (0 specific densities, 1 s*, 4 s* and n*);
// DBG: export the accepted pairs.  stage: the Heun stage (in 3+1D, stage 0
// also lists every candidate within the support plus twice a step's
// displacement bound, and the later pair passes of the step walk that skin
// list instead of the candidates)
template <int D, bool MIXED, int NS, bool DBG>
__global__ void __launch_bounds__(256) k_density(BatchDev b, Params prm, const double* __restrict__ Y, int stage,
                                                 PairExport px) {
  constexpr int L = Team<D>::L, P = Team<D>::P;
  constexpr int ROWS = RowBlock<D>::ROWS;
  constexpr int G = NS > 0 ? 1 : 0;
  using RT = typename std::conditional<MIXED, float, double>::type;
  using HaloT = Halo<D, MIXED, G, DBG, 6, TileBytes<D>::DENS>;
  constexpr int C = HaloT::C;
  __shared__ TileShared<D, P> S;
  __shared__ __align__(16) char s_mem[HaloT::BYTES];
  const HaloT H{s_mem};
  const int64_t cap = b.cap;
  int ev0;
  int64_t j0, jend;
  if (!tile_targets<P>(b, xcd_block(blockIdx.x, gridDim.x), ev0, j0, jend)) return;  // whole workgroup
  const int32_t total = tile_setup<D, L, P>(b, ev0, j0, jend, S);
  // team t walks target j0 + q (its partial sums go through the team's own
  // LDS region t)
  const int t = (int)threadIdx.x / L, lane = (int)threadIdx.x % L;
  const int q = TeamSort<D>::ON ? S.perm[t] : t;
  const int64_t j = j0 + q;
  const bool have = S.seg[q] >= 0;
  const double h = prm.h, ih = 1.0 / h, r2max = (2.0 * h) * (2.0 * h);
  double xa[3] = {0.0, 0.0, 0.0};
  if (have) {
#pragma unroll
    for (int k = 0; k < D; ++k) xa[k] = row(Y, cap, R_X1 + k, j);
  }
  DensAcc<MIXED, NS> A;
  A.init();
  TileCursor<L, ROWS> cur;
  cur.start(S.lo[q], S.hi[q], lane);
  constexpr int U = PairU<D>::U;
  // The target's skin list (3+1D), appended one ballot group at a time: the
  // team's lanes are bits [tsh, tsh + L) of a wave ballot, and a group goes
  // out in lane order; nskin counts the entries (the same on the team's
  // lanes while they walk).  Past the capacity the entries pile up on the
  // last one: such a list is marked unusable below.
  constexpr bool LIST = list_cap(D) > 0;
  static_assert(!LIST || L <= 32, "a team's ballot bits fit one 32-bit word");
  constexpr uint32_t TEAM_BITS = L == 32 ? ~0u : (1u << L) - 1u;
  const uint32_t tsh = (uint32_t)threadIdx.x & 63u & ~(uint32_t)(L - 1);
  const uint32_t below = (1u << lane) - 1u;
  uint16_t* const myskin = b.slist + (LIST ? (have ? j : j0) * list_cap(D) : 0);
  int32_t nskin = 0;
  // Skin list of stage 0: every candidate within 2h + 2d of the target,
  // d = dt max(1, 1/x0) the bound on a particle's displacement over a step
  // (its coordinate speeds are below 1, and below 1/x0 along eta in Milne
  // coordinates).  A pair within 2h at the stage-1 positions is within
  // 2h + 2d at the stage-0 ones, and the rows of the last binning hold every
  // such candidate (a binning is redone before twice the displacement bound
  // accumulated by the end of a step exceeds the skin).  The gradient pass of
  // stage 0 and both passes of stage 1 then test only these, with the same
  // pair test.
  const bool make_skin = LIST && !DBG && stage == 0;
  double r2skin = 0.0;
  if (make_skin) {
    const EventDev& E = b.evt[ev0];
    const double vmax = (prm.hyperbolic && D == 3) ? fmax(1.0, 1.0 / E.t) : 1.0;
    const double rs = 2.0 * h + 2.0 * E.dt * vmax;
    r2skin = rs * rs * (1.0 + 1e-9);
  }
  // stage 1: the target's skin list (-1: it did not fit; walk the candidates)
  const int32_t scnt = !(LIST && !DBG && stage == 1) ? -1 : have ? min(b.scnt[j], list_cap(D)) : 0;
  const bool from_skin = scnt >= 0;
  int32_t sp = 0;  // next skin-list entry
  // the sums over U candidates per lane (chunk-local halo indices k[u]; v[u]
  // marks the ones to test), with the skin-list appends
  auto add_pairs = [&](int32_t c0, const int32_t (&k)[U], const bool (&v)[U]) {
    double d2[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double2 p = H.xy()[k[u]];
      const double xb[3] = {p.x, p.y, D == 3 ? H.z()[k[u]] : 0.0};
      d2[u] = dist2<D>(xa, xb);
      ok[u] = v[u] && d2[u] < r2max;
    }
    RT sc[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      sc[u][0] = sc[u][1] = sc[u][2] = sc[u][3] = RT(0);
      if (G) H.q(0)[k[u]].get(sc[u]);
    }
    A.template add_block<U>(ok, d2, ih, sc);
    if (make_skin) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool sk = v[u] && d2[u] < r2skin;
        const uint32_t tb = (uint32_t)(__builtin_amdgcn_ballot_w64(sk) >> tsh);
        if (sk) {
          const int32_t at = nskin + __popc(tb & below);
          myskin[at < list_cap(D) ? at : list_cap(D) - 1] = (uint16_t)(c0 + k[u]);
        }
        nskin += __popc(tb & TEAM_BITS);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (DBG && ok[u]) {
        const int64_t at = (int64_t)atomicAdd((unsigned long long*)px.counter, 1ull);
        if (at < px.cap) {
          px.a[at] = b.ids[j];
          px.b[at] = b.ids[H.slot()[k[u]]];
        }
      }
    }
  };
  for (int32_t c0 = 0; c0 < total; c0 += C) {
    const int32_t c1 = total - c0 < C ? total : c0 + C;
    halo_load(H, S, Y, cap, c0, c1, [&](int32_t sl, Quad<MIXED>* q, size_t) {
      if (NS == 4)
        q->put(row(Y, cap, R_S, sl), row(Y, cap, R_NB, sl), row(Y, cap, R_NS, sl), row(Y, cap, R_NQ, sl));
      else if (NS == 1)
        q->put(row(Y, cap, R_S, sl), 0.0, 0.0, 0.0);
    });
    __syncthreads();
    if (from_skin) {
      // stage 1: the skin-list entries with halo index in [c0, c1), lane k
      // taking entries sp + k, sp + k + L, ...  Lanes enter a chunk of the
      // stage-0 walk at different phases, so the list is ordered group by
      // group only (entries L or more apart are in halo order): a lane's
      // first entry at or beyond c1 is followed only by larger ones, and
      // entries met again below c0 were taken in an earlier chunk.
      int32_t out = INT32_MAX;  // this lane's first entry at or beyond c1
      auto fetch = [&](int32_t (&xs)[U], int32_t i0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // unconditional loads (entry 0 stands in past the end), so that
          // the wait for them can leave the next pass's loads in flight
          const int32_t i = i0 + u * L;
          const int32_t v = myskin[i < scnt ? i : 0];
          xs[u] = i < scnt ? v : INT32_MAX;
        }
      };
      int32_t x[U];
      fetch(x, sp + lane);
      for (int32_t i0 = sp + lane;; i0 += L * U) {
        int32_t xn[U];
        fetch(xn, i0 + L * U);
        int32_t k[U];
        bool v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t i = i0 + u * L;
          v[u] = x[u] >= c0 && x[u] < c1;
          if (x[u] >= c1 && i < out) out = i;
          k[u] = v[u] ? x[u] - c0 : 0;
        }
        const bool end = out != INT32_MAX;
        if (end && !v[0]) break;
        add_pairs(c0, k, v);
        if (end) break;
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = xn[u];
      }
#pragma unroll
      for (int off = L / 2; off >= 1; off >>= 1) {
        const int32_t o = __shfl_xor(out, off, 64);
        out = o < out ? o : out;
      }
      sp = out;
    } else {
      cur.chunk(c0, c1);
      for (;;) {
        int32_t k[U];
        bool v[U];
        take<U>(cur, k, v);
        if (!v[0]) break;
        add_pairs(c0, k, v);
        if (!v[U - 1]) break;
      }
    }
    // the lists' lengths so far: the lane that walked longest has seen
    // every append of the chunk
#pragma unroll
    for (int off = LIST ? L / 2 : 0; off >= 1; off >>= 1) {
      const int32_t os = __shfl_xor(nskin, off, 64);
      nskin = os > nskin ? os : nskin;
    }
    A.flush();
    __syncthreads();
  }
  // -1 when the list overflows or its halo indices do not fit 16 bits
  if (make_skin && have && lane == 0) b.scnt[j] = (nskin <= list_cap(D) && total <= 65536) ? nskin : -1;
  // lanes v < 6 form row v of the density sums (sigma*, S, N_B, N_S, N_Q, count)
  double part[6], tot[(6 + L - 1) / L];
  A.partials(part);
  team_sums_lds_n<L, 6>(H.red() + (size_t)t * L * 6, lane, part, tot);
  if (have) {
#pragma unroll
    for (int q = 0; q < (6 + L - 1) / L; ++q) {
      const int v = lane + q * L;
      if (v < 6) b.dsum[(int64_t)(DS_SIG + v) * cap + j] = v == 5 ? tot[q] : tot[q] * sigma_d<D>(prm.h);
    }
  }
}

// own record and geometry of particle j for the gradient sums
template <int D, bool VISC, bool MIXED>
__device__ __forceinline__ void grad_setup(const BatchDev& b, const Params& prm, const double* __restrict__ Y,
                                           double t, int64_t j, GradAcc<D, VISC, MIXED>& A) {
  const int64_t cap = b.cap;
  const double G3 = metric_G3(prm, t);
  A.Gk[0] = 0.0;
  A.Gk[1] = 1.0;
  A.Gk[2] = 1.0;
  A.Gk[3] = G3;
  A.ih = 1.0 / prm.h;
  A.xa[0] = row(Y, cap, R_X1, j);
  A.xa[1] = row(Y, cap, R_X2, j);
  A.xa[2] = D == 3 ? row(Y, cap, R_X3, j) : 0.0;
  auto recv = [&](int q) -> double {
    return MIXED ? (double)b.recf[(int64_t)q * cap + j] : b.rec[(int64_t)q * cap + j];
  };
  A.aPP = recv(Q_PP);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    A.aU[k] = k < D ? recv(Q_U1 + k) : 0.0;
    A.aV[k] = k < D ? recv(Q_V1 + k) : 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) A.aA[k][i] = (VISC && k < D && i < D) ? recv(Q_A11 + k * 3 + i) : 0.0;
  }
  A.init();
}

// neighbour record of the gradient sums as staged in LDS: (p+Pi)/sigma*^2,
// u^1..u^D, v^1..v^D and, when viscous, A^{ji}/sigma*^2 at j*D + i
template <int D, bool VISC>
struct GradRec {
  static constexpr int N = 1 + 2 * D + (VISC ? D * D : 0);
  static constexpr int G = (N + 3) / 4;
  __device__ __forceinline__ static int source(int q) {  // its row of the pass-1 record
    return q == 0 ? Q_PP : q <= D ? Q_U1 + q - 1 : q <= 2 * D ? Q_V1 + q - 1 - D
                                                              : Q_A11 + ((q - 1 - 2 * D) / D) * 3 + (q - 1 - 2 * D) % D;
  }
};

// DIFF: also the BSQ diffusion sums (DiffAcc) over the same accepted pairs
// (1: without, 2: with the bulk-pressure gradient); their FP64 records are
// read from global memory by slot
template <int D, bool VISC, bool MIXED, int DIFF>
__global__ void __launch_bounds__(256) k_grad(BatchDev b, Params prm, const double* __restrict__ Y, int stage) {
  constexpr int L = Team<D>::L, P = Team<D>::P;
  constexpr int ROWS = RowBlock<D>::ROWS;
  using GA = GradAcc<D, VISC, MIXED>;
  using RT = typename GA::RT;
  using GR = GradRec<D, VISC>;
  constexpr int NP = GA::NP;
  using HaloT = Halo<D, MIXED, GR::G, DIFF != 0, NP, TileBytes<D>::GRAD>;
  constexpr int C = HaloT::C;
  __shared__ TileShared<D, P> S;
  __shared__ __align__(16) char s_mem[HaloT::BYTES];
  const HaloT H{s_mem};
  const int64_t cap = b.cap;
  int ev0;
  int64_t j0, jend;
  if (!tile_targets<P>(b, xcd_block(blockIdx.x, gridDim.x), ev0, j0, jend)) return;  // whole workgroup
  const int32_t total = tile_setup<D, L, P>(b, ev0, j0, jend, S);
  // team t walks target j0 + q (its partial sums go through the team's own
  // LDS region t)
  const int t = (int)threadIdx.x / L, lane = (int)threadIdx.x % L;
  const int q = TeamSort<D>::ON ? S.perm[t] : t;
  const int64_t j = j0 + q;
  const bool have = S.seg[q] >= 0;
  const double r2max = (2.0 * prm.h) * (2.0 * prm.h);
  GA A;
  DiffAcc<D, DIFF == 2> DA;
  if (have) {
    const EventDev& E = b.evt[ev0];
    grad_setup<D, VISC, MIXED>(b, prm, Y, E.t + stage * E.dt, j, A);
    if (DIFF) DA.init(b.drec, cap, j);
  } else {
    A.xa[0] = A.xa[1] = A.xa[2] = 0.0;
    A.ih = 1.0;
    A.init();
    if (DIFF) DA.init(b.drec, cap, j0);
  }
  TileCursor<L, ROWS> cur;
  cur.start(S.lo[q], S.hi[q], lane);
  constexpr int U = PairU<D>::U;
  // the target's skin list from the step's first density pass (-1: it did
  // not fit; walk the candidates instead), next entry lp
  constexpr bool LIST = list_cap(D) > 0;
  const int32_t cnt = !LIST ? -1 : have ? min(b.scnt[j], list_cap(D)) : 0;
  const bool listed = LIST && cnt >= 0;
  // (a lane without a target reads the list of the workgroup's first one)
  const uint16_t* const mylist = b.slist + (LIST ? (have ? j : j0) * list_cap(D) : 0);
  int32_t lp = 0;
  for (int32_t c0 = 0; c0 < total; c0 += C) {
    const int32_t c1 = total - c0 < C ? total : c0 + C;
    halo_load(H, S, Y, cap, c0, c1, [&](int32_t sl, Quad<MIXED>* q, size_t stride) {
      const RT* rb = MIXED ? (const RT*)b.recf : (const RT*)b.rec;
      auto op = [&](int i) -> RT { return i < GR::N ? rb[(int64_t)GR::source(i) * cap + sl] : RT(0); };
#pragma unroll
      for (int g = 0; g < GR::G; ++g) q[g * stride].put(op(4 * g), op(4 * g + 1), op(4 * g + 2), op(4 * g + 3));
    });
    __syncthreads();
    // the sums over U candidates per lane (chunk-local halo indices k[u],
    // pairs where okin[u], the target itself excluded)
    auto add_pairs = [&](const int32_t (&k)[U], const bool (&okin)[U]) {
      double xb[U][3], d2[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double2 p = H.xy()[k[u]];
        xb[u][0] = p.x;
        xb[u][1] = p.y;
        xb[u][2] = D == 3 ? H.z()[k[u]] : 0.0;
        d2[u] = dist2<D>(A.xa, xb[u]);
        // the pair test (the target itself has no gradient term)
        ok[u] = okin[u] && d2[u] < r2max && d2[u] > 0.0;
      }
      RT rec[U][4 * GR::G];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int g = 0; g < GR::G; ++g) H.q(g)[k[u]].get(rec[u] + 4 * g);
      A.template add_block<U>(ok, xb, d2, rec);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (DIFF && ok[u]) {
          double ab[3], Fb[3][3], Pb = 0.0;
          DiffAcc<D, DIFF == 2>::load(b.drec, cap, H.slot()[k[u]], ab, Fb, Pb);
          DA.add(A.xa, xb[u], d2[u], A.ih, ab, Fb, Pb);
        }
      }
    };
    if (listed) {
      // the target's skin-list entries with halo index in [c0, c1), each
      // with the pair test at this stage's positions: entries lp + lane,
      // lp + lane + L, ... of its list.  The density pass appends one ballot
      // group (at most L entries, lanes in lane order) at a time and its
      // lanes enter a chunk at different phases, so the list is ordered group
      // by group: entries L or more apart are in halo order.  A lane's first
      // entry at or beyond c1 is therefore followed only by larger ones, and
      // entries of the previous chunks met again below c0 are skipped.
      int32_t out = INT32_MAX;  // this lane's first entry at or beyond c1
      // the entries of a pass are loaded one pass ahead, so that their
      // latency hides behind the sums of the previous one
      auto fetch = [&](int32_t (&xs)[U], int32_t i0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // unconditional loads (entry 0 stands in past the end), so that
          // the wait for them can leave the next pass's loads in flight
          const int32_t i = i0 + u * L;
          const int32_t v = mylist[i < cnt ? i : 0];
          xs[u] = i < cnt ? v : INT32_MAX;
        }
      };
      int32_t x[U];
      fetch(x, lp + lane);
      for (int32_t i0 = lp + lane;; i0 += L * U) {
        int32_t xn[U];
        fetch(xn, i0 + L * U);
        int32_t k[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t i = i0 + u * L;
          ok[u] = x[u] >= c0 && x[u] < c1;
          if (x[u] >= c1 && i < out) out = i;
          k[u] = ok[u] ? x[u] - c0 : 0;
        }
        const bool end = out != INT32_MAX;
        if (end && !ok[0]) break;
        add_pairs(k, ok);
        if (end) break;
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = xn[u];
      }
      // the team's next chunk starts at the first entry any of its lanes
      // found at or beyond c1: every entry before it has been taken
#pragma unroll
      for (int off = L / 2; off >= 1; off >>= 1) {
        const int32_t o = __shfl_xor(out, off, 64);
        out = o < out ? o : out;
      }
      lp = out;
    } else {
      // more pairs than the list holds: the candidate walk with the pair test
      cur.chunk(c0, c1);
      for (;;) {
        int32_t k[U];
        bool v[U];
        take<U>(cur, k, v);
        if (!v[0]) break;
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double2 p = H.xy()[k[u]];
          const double xq[3] = {p.x, p.y, D == 3 ? H.z()[k[u]] : 0.0};
          const double dq = dist2<D>(A.xa, xq);
          ok[u] = v[u] && dq < r2max && dq > 0.0;
        }
        add_pairs(k, ok);
        if (!v[U - 1]) break;
      }
    }
    A.flush();
    __syncthreads();
  }
  // lane v forms gradient sums v, v + L, ...: F_i, d_k u^j (row-major), div v
  {
    constexpr int NQ = (NP + L - 1) / L;
    double part[NP], tot[NQ];
    A.partials(part);
    team_sums_lds_n<L, NP>(H.red() + (size_t)t * L * NP, lane, part, tot);
    if (have) {
      const double fsd = sigma_d<D>(prm.h) / prm.h;
      const double isg = fsd / b.th[(int64_t)T_SIGSTAR * cap + j];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int v = lane + q * L;
        if (v >= NP) continue;
        int rw;
        double scale = isg;
        if (v < D) {
          rw = GS_F1 + v;
          scale = fsd;
        } else if (v < NP - 1) {
          rw = GS_DU11 + ((v - D) / D) * 3 + (v - D) % D;
        } else {
          rw = GS_DIVV;
        }
        b.gsum[(int64_t)rw * cap + j] = tot[q] * scale;
      }
    }
  }
  if (DIFF) DA.template reduce<L>();
  if (DIFF && have && lane == 0) {
    const double fsd = sigma_d<D>(prm.h) / prm.h;
    DA.write(b.gsum, cap, j, fsd, fsd / b.th[(int64_t)T_SIGSTAR * cap + j]);
  }
}


// ---------------------------------------------------------------------------
// Freeze-out crossing of particle j at the start of a step ("Freeze-out
// hypersurface construction", eq. efo_surface): its energy density fell from
// >= e_fo at the previous step start to < e_fo now, and it has not crossed
// before.  The record gets the crossing time (e linear in x^0 between the two
// step starts), the position moved back to it along dx^i/dx^0 = u^i / u^0,
// and u^i, T, mu_q now; the update pass adds d sigma_mu (k_eom).
template <int D>
__device__ __forceinline__ void freezeout_crossing(const BatchDev& b, const Params& prm, const double* __restrict__ Y,
                                                   int64_t j, const EventDev& E, const Thermo& th, const double u[4],
                                                   double gam) {
  const int64_t cap = b.cap;
  const double ep = b.warms[(int64_t)W_EPREV * cap + j];
  const bool frozen = b.warms[(int64_t)W_FROZEN * cap + j] != 0.0;
  b.warms[(int64_t)W_EPREV * cap + j] = th.e;
  if (frozen || !(ep >= prm.e_fo && th.e < prm.e_fo)) return;
  b.warms[(int64_t)W_FROZEN * cap + j] = 1.0;
  const uint32_t at = atomicAdd(&b.fo_ctr[0], 1u);
  if (at >= (uint32_t)cap) return;  // each particle crosses once: cannot happen
  double* r = b.fo_rec + (int64_t)at * FO_NCOL;
  const double tfo = E.t - (E.t - E.t_prev) * (prm.e_fo - th.e) / (ep - th.e);
  r[FO_ID] = (double)b.ids[j];
  r[FO_T] = tfo;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[FO_X1 + k] = k < D ? row(Y, cap, R_X1 + k, j) - (E.t - tfo) * u[1 + k] / gam : 0.0;
    r[FO_U1 + k] = k < D ? u[1 + k] : 0.0;
  }
  r[FO_TEMP] = th.T;
#pragma unroll
  for (int q = 0; q < 3; ++q) r[FO_MUB + q] = th.mu[q];
#pragma unroll
  for (int m = 0; m < 4; ++m) r[FO_DS0 + m] = 0.0;
  b.fo_slot[at] = (int32_t)j;
  b.fo_mark[j] = (int32_t)at;
}

// fo: look for a freeze-out crossing (first stage of a step, surface on)
template <int D, bool VISC, bool MIXED, int NQ>
__device__ __forceinline__ void eos_particle(const BatchDev& b, const Params& prm, const EosDev& eos,
                                             const double* __restrict__ Y, int stage, int64_t j, int e, double* aux,
                                             bool fo, uint32_t& c_backup, uint32_t& c_iters, uint32_t& c_noconv) {
  const EventDev& E = b.evt[e];
  const int64_t cap = b.cap;
  const bool smoothed = prm.density_mode == 0;
  // every input of the particle, loaded together (one memory round trip
  // instead of a chain): sums, flow, densities (smoothed sums or the
  // particle's own S, N), dissipative state, warm start
  const double ss = b.dsum[(int64_t)DS_SIG * cap + j];
  double u[4] = {0.0, row(Y, cap, R_U1, j), row(Y, cap, R_U2, j), D == 3 ? row(Y, cap, R_U3, j) : 0.0};
  const double* dsrc = smoothed ? b.dsum + (int64_t)DS_S * cap : Y + (int64_t)R_S * cap;
  static_assert(DS_NB == DS_S + 1 && R_NB == R_S + 1, "S and N rows consecutive");
  double dv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) dv[q] = (q == 0 || NQ) ? dsrc[(int64_t)q * cap + j] : 0.0;
  double yv[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (VISC) {
    const int rv[7] = {R_B, R_P11, R_P12, R_P22, R_P33, R_P13, R_P23};
#pragma unroll
    for (int k = 0; k < (D == 3 ? 7 : 5); ++k) yv[k] = row(Y, cap, rv[k], j);
  }
  double warm[NWARM_EOS];
#pragma unroll
  for (int w = 0; w < NWARM_EOS; ++w) warm[w] = b.warms[(int64_t)w * cap + j];
  const double t = E.t + stage * E.dt;

  const double G3 = metric_G3(prm, t);
  const double g2 = 1.0 + u[1] * u[1] + u[2] * u[2] + G3 * u[3] * u[3];
  const double igam = rsqrt_nr(g2), gam = g2 * igam;
  u[0] = gam;
  const double norm = gam * sqrt_g(prm, t);
  // shared reciprocals (one division each instead of one per quotient)
  const double inorm = 1.0 / norm;
  const double sigma = ss * inorm;
  double dens[4];
  const double dscale = smoothed ? inorm : sigma;
#pragma unroll
  for (int q = 0; q < 4; ++q) dens[q] = dv[q] * dscale;

  // EoS inversion (s, n) -> (T, mu): the offline table when the EoS carries
  // one and (s, n) is on its grid, else online, warm-started from the
  // particle's last roots
  Thermo th;
  if (!(eos.inv.val && inv_lookup<NQ>(eos.inv, dens, th))) {
    double wnew[NWARM_EOS];
    eos_invert<NQ>(eos, 0, dens, warm, th, wnew);
#pragma unroll
    for (int w = 0; w < NWARM_EOS; ++w) b.warms[(int64_t)w * cap + j] = wnew[w];
  }
  c_noconv = th.ok ? 0u : 1u;
  c_backup = (!th.in_table && eos.kind == EOS_TABLE) ? 1u : 0u;
  c_iters = (uint32_t)th.iters;
  if (fo) freezeout_crossing<D>(b, prm, Y, j, E, th, u, gam);

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
    Pi = sigma * yv[0];
    pi[1][1] = sigma * yv[1];
    pi[1][2] = pi[2][1] = sigma * yv[2];
    pi[2][2] = sigma * yv[3];
    pi[3][3] = sigma * yv[4];
    if (D == 3) {
      pi[1][3] = pi[3][1] = sigma * yv[5];
      pi[2][3] = pi[3][2] = sigma * yv[6];
    }
    const double Gq[4] = {0.0, 1.0, 1.0, G3};
#pragma unroll
    for (int i = 1; i < 4; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 1; k < 4; ++k) acc += Gq[k] * u[k] * pi[k][i];
      pi[0][i] = pi[i][0] = acc * igam;
    }
  }

  double* T_ = b.th;
  T_[(int64_t)T_SIGSTAR * cap + j] = ss;
  T_[(int64_t)T_T * cap + j] = th.T;
  T_[(int64_t)T_P * cap + j] = th.p;
  T_[(int64_t)T_E * cap + j] = th.e;
  T_[(int64_t)T_CS2 * cap + j] = th.cs2;
  T_[(int64_t)T_KAP * cap + j] = th.kappa;
  if (NQ) {
#pragma unroll
    for (int q = 0; q < 3; ++q) T_[(int64_t)(T_MUB + q) * cap + j] = th.mu[q];
  }
  if (VISC) {
    T_[(int64_t)T_PI * cap + j] = Pi;
    T_[(int64_t)T_ETA * cap + j] = eta;
    T_[(int64_t)T_ZETA * cap + j] = zeta;
    T_[(int64_t)T_TAUPI * cap + j] = taupi;
    T_[(int64_t)T_TAUPIB * cap + j] = tauPi;
  }

  // neighbour record for the gradient sums
  const double is2 = 1.0 / (ss * ss);
  double rec[NREC];
  rec[Q_PP] = (th.p + Pi) * is2;
#pragma unroll
  for (int jj = 1; jj < 4; ++jj)
#pragma unroll
    for (int ii = 1; ii < 4; ++ii)
      rec[Q_A11 + (jj - 1) * 3 + (ii - 1)] = (pi[jj][ii] - (u[jj] * igam) * pi[0][ii]) * is2;
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    rec[Q_U1 + k - 1] = u[k];
    rec[Q_V1 + k - 1] = u[k] * igam;
  }
#pragma unroll
  for (int r = 0; r < NREC; ++r) {
    const bool used = r == Q_PP || (VISC && r >= Q_A11 && r <= Q_A33 && ((r - Q_A11) / 3) < D && ((r - Q_A11) % 3) < D) ||
                      (r >= Q_U1 && r < Q_U1 + D) || (r >= Q_V1 && r < Q_V1 + D);
    if (!used) continue;
    if (MIXED)
      b.recf[(int64_t)r * cap + j] = (float)rec[r];
    else
      b.rec[(int64_t)r * cap + j] = rec[r];
  }
  // record of the diffusion sums (FP64 in both precisions): alpha_q = mu_q/T and
  // F^k_q / sigma*^2 with F = J - v J^0, J^k = sigma V^k, J^0 = G_k u^k J^k / gamma
  if (NQ && prm.diffusion) {
    const double Gq[4] = {0.0, 1.0, 1.0, G3};
    const double iT = 1.0 / th.T;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double J[3], J0 = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        J[k] = k < D ? sigma * row(Y, cap, R_JB1 + 3 * q + k, j) : 0.0;
        J0 += Gq[1 + k] * u[1 + k] * J[k];
      }
      J0 *= igam;
      b.drec[(int64_t)(QD_AB + q) * cap + j] = th.mu[q] * iT;
      if (q == 0) b.drec[(int64_t)QD_PI * cap + j] = Pi;
#pragma unroll
      for (int k = 0; k < D; ++k)
        b.drec[(int64_t)(QD_FB1 + 3 * q + k) * cap + j] = (J[k] - (u[1 + k] * igam) * J0) * is2;
    }
  }
  if (aux) {
    const int64_t ii = b.ids[j];
    const int64_t n = E.n;
    aux[X_SIGSTAR * n + ii] = ss;
    aux[X_S * n + ii] = dens[0];
    for (int q = 0; q < 3; ++q) aux[(X_NB + q) * n + ii] = dens[1 + q];
    aux[X_T * n + ii] = th.T;
    for (int q = 0; q < 3; ++q) aux[(X_MUB + q) * n + ii] = th.mu[q];
    aux[X_P * n + ii] = th.p;
    aux[X_E * n + ii] = th.e;
    aux[X_CS2 * n + ii] = th.cs2;
    aux[X_INTABLE * n + ii] = th.in_table;
    aux[X_GAMMA * n + ii] = gam;
    aux[X_NNB * n + ii] = b.dsum[(int64_t)DS_NNB * cap + j];
    aux[X_NEWTON * n + ii] = th.iters;
    aux[X_EOS_EVALS * n + ii] = th.evals;
  }
}

template <int D, bool VISC, bool MIXED, int NQ>
__global__ void __launch_bounds__(128) k_eos(BatchDev b, Params prm, EosDev eos, const double* __restrict__ Y,
                                             int stage, int64_t nslots, double* aux, int fo) {
  const int64_t j = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  int e = -1;
  uint32_t c_backup = 0, c_iters = 0, c_noconv = 0;
  if (j < nslots) {
    e = b.ev[j];
    if (e >= 0)
      eos_particle<D, VISC, MIXED, NQ>(b, prm, eos, Y, stage, j, e, aux, fo != 0, c_backup, c_iters, c_noconv);
  }
  wave_count_eos(b.evt, e, c_backup, c_iters, c_noconv);
}


// Spatial gradient of the energy density for the freeze-out surface
// ("Freeze-out hypersurface construction"), n = 1 difference form like
// d_k u^j: d_i e_a = (1/sigma*_a) sum_b (e_b - e_a) d_i W_ab, at slot j.
template <int D>
__device__ inline void fo_grad_particle(const BatchDev& b, const Params& prm, const double* __restrict__ Y,
                                        int64_t j) {
  const int e = b.ev[j];
  if (e < 0) return;
  const EventDev& E = b.evt[e];
  const int64_t cap = b.cap;
  const double h = prm.h, ih = 1.0 / h, r2max = (2.0 * h) * (2.0 * h);
  const double xa[3] = {row(Y, cap, R_X1, j), row(Y, cap, R_X2, j), D == 3 ? row(Y, cap, R_X3, j) : 0.0};
  const double* Ev = b.th + (int64_t)T_E * cap;
  const double ea = Ev[j];
  double de[3] = {0.0, 0.0, 0.0};
  for_each_row<D>(b, E, b.keys[j], xa, prm.cell_edge, [&](int32_t lo, int32_t hi) {
    for (int32_t k = lo; k < hi; ++k) {
      const double xb[3] = {row(Y, cap, R_X1, k), row(Y, cap, R_X2, k), D == 3 ? row(Y, cap, R_X3, k) : 0.0};
      const double d2 = dist2<D>(xa, xb);
      if (!(d2 < r2max)) continue;
      const double r = sqrt(d2);
      if (!(r > 0.0)) continue;
      const double f = spline_dw(r * ih) / r * (Ev[k] - ea);
#pragma unroll
      for (int q = 0; q < D; ++q) de[q] += f * (xa[q] - xb[q]);
    }
  });
  const double isg = sigma_d<D>(h) / h / b.th[(int64_t)T_SIGSTAR * cap + j];
#pragma unroll
  for (int q = 0; q < 3; ++q) b.gsum[(int64_t)(GS_DE1 + q) * cap + j] = q < D ? de[q] * isg : 0.0;
}

// every particle (diagnostic evaluations)
template <int D>
__global__ void __launch_bounds__(128) k_fo_grad(BatchDev b, Params prm, const double* __restrict__ Y,
                                                 int64_t nslots) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nslots) fo_grad_particle<D>(b, prm, Y, j);
}

// the particles that crossed e_fo in this step (records [fo_ctr[1], fo_ctr[0]))
template <int D>
__global__ void __launch_bounds__(64) k_fo_grad_list(BatchDev b, Params prm, const double* __restrict__ Y) {
  const uint32_t lo = b.fo_ctr[1], hi = b.fo_ctr[0] < (uint32_t)b.cap ? b.fo_ctr[0] : (uint32_t)b.cap;
  for (uint32_t q = lo + blockIdx.x * blockDim.x + threadIdx.x; q < hi; q += gridDim.x * blockDim.x)
    fo_grad_particle<D>(b, prm, Y, b.fo_slot[q]);
}

// records found before this step: the first stage's crossings are appended after them
__global__ void k_fo_begin(BatchDev b) {
  if (blockIdx.x == 0 && threadIdx.x == 0) b.fo_ctr[1] = b.fo_ctr[0];
}

// Source densities I^mu, I_q at position x and time t: sum over the active
// sources of the rates times the normalised Gaussian around the moving
// centre, divided by sqrt(-g) (eq. conservation_source with the smeared
// deposition of the dynamical initialisation).
template <int D>
__device__ inline void source_density(const SourceSet& S, double t, double sqg, const double x[3], double I[4],
                                      double Iq[3]) {
  const int ns = S.n;
  for (int k = 0; k < ns; ++k) {
    const SourceDev& s = S.s[k];
    if (!(t >= s.t_on && t < s.t_off)) continue;
    double arg = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double dx = x[d] - (s.c0[d] + s.vel[d] * (t - s.t_on));
      arg += dx * dx * s.iw2[d];
    }
    const double g = s.norm * exp(-arg) / sqg;
#pragma unroll
    for (int m = 0; m < 4; ++m) I[m] += s.dpdt[m] * g;
#pragma unroll
    for (int q = 0; q < 3; ++q) Iq[q] += s.dndt[q] * g;
  }
}

// Freeze-out surface element at slot j ("Freeze-out hypersurface
// construction", eq. fonormal): d_0 e from D e = -(e + p + Pi) theta +
// pi:sigma + u.I with D = gamma d_0 + u^i d_i and the SPH gradient d_i e;
// n_mu = -d_mu e / sqrt(|d e . d e|), d sigma_mu = n_mu / (sigma |u.n|) (m = 1).
template <int D>
__device__ inline void surface_element(const BatchDev& b, int64_t j, const EomIn& in, const EomOut& o,
                                       const double Gk[4], double dmu[4], double dsl[4]) {
  const int64_t cap = b.cap;
  const double ee = b.th[(int64_t)T_E * cap + j], pp = b.th[(int64_t)T_P * cap + j];
  const double gm[4] = {1.0, -1.0, -1.0, -Gk[3]};
  const double giv[4] = {1.0, -1.0, -1.0, -1.0 / Gk[3]};
#pragma unroll
  for (int m = 0; m < 4; ++m) dmu[m] = 0.0;
#pragma unroll
  for (int q = 0; q < D; ++q) dmu[1 + q] = b.gsum[(int64_t)(GS_DE1 + q) * cap + j];
  double uI = 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m) uI += gm[m] * in.u[m] * in.I[m];
  const double De = -(ee + pp + in.Pi) * o.theta + o.pisig + uI;
  double adv = 0.0;
#pragma unroll
  for (int k = 1; k <= D; ++k) adv += in.u[k] * dmu[k];
  dmu[0] = (De - adv) / in.u[0];
  double nn = 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m) nn += giv[m] * dmu[m] * dmu[m];
  const double norm = sqrt(fabs(nn));
  double nl[4] = {0.0, 0.0, 0.0, 0.0}, un = 0.0;
  if (norm > 0.0) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      nl[m] = -dmu[m] / norm;
      un += in.u[m] * nl[m];
    }
  }
  const double dsig = (norm > 0.0 && fabs(un) > 0.0) ? 1.0 / (in.sigma * fabs(un)) : 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m) dsl[m] = dsig * nl[m];
}

// ---------------------------------------------------------------------------
//   mode 0: Y1 = Ys + dt f(Ys)
//   mode 1: Y0 = (Ys + Y1 + dt f(Y1)) / 2, carry ids and warm starts home
//   mode 2: write f(Y) and diagnostics in the caller's order (no update)
template <int D, bool VISC>
__global__ void __launch_bounds__(128) k_eom(BatchDev b, Params prm, const double* __restrict__ Y, int stage,
                                             int mode, int64_t nslots, double* fout, double* aux) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslots) return;
  const int e = b.ev[j];
  if (e < 0) return;
  const EventDev& E = b.evt[e];
  const double t = E.t + stage * E.dt;
  const int64_t cap = b.cap;
  const double G3 = metric_G3(prm, t);
  const double Gk[4] = {0.0, 1.0, 1.0, G3};
  const double sigstar = b.th[(int64_t)T_SIGSTAR * cap + j];

  EomIn in;
  in.t = t;
  in.u[0] = 0.0;
#pragma unroll
  for (int k = 1; k < 4; ++k) in.u[k] = k <= D ? row(Y, cap, R_U1 + k - 1, j) : 0.0;
  const double g2 = 1.0 + in.u[1] * in.u[1] + in.u[2] * in.u[2] + G3 * in.u[3] * in.u[3];
  const double igam = rsqrt_nr(g2), gam = g2 * igam;
  in.u[0] = gam;
#pragma unroll
  for (int k = 0; k < 4; ++k) in.v[k] = in.u[k] * igam;
#pragma unroll
  for (int n = 0; n < 4; ++n) in.dudx[0][n] = 0.0;
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int n = 1; n < 4; ++n) {
      const double v = (k <= D && n <= D) ? b.gsum[(int64_t)(GS_DU11 + (k - 1) * 3 + (n - 1)) * cap + j] : 0.0;
      in.dudx[k][n] = v;
      acc += Gk[n] * in.u[n] * v;
    }
    in.dudx[k][0] = acc * igam;
  }
  in.divv = b.gsum[(int64_t)GS_DIVV * cap + j];
  in.F[0] = 0.0;
#pragma unroll
  for (int k = 1; k < 4; ++k) in.F[k] = k <= D ? b.gsum[(int64_t)(GS_F1 + k - 1) * cap + j] : 0.0;
  const double sqg = sqrt_g(prm, t);
  in.sigma = sigstar / (gam * sqg);
  const double* T_ = b.th;
  in.w = T_[(int64_t)T_E * cap + j] + T_[(int64_t)T_P * cap + j];
  in.T = T_[(int64_t)T_T * cap + j];
  in.cs2 = T_[(int64_t)T_CS2 * cap + j];
  in.kappa = T_[(int64_t)T_KAP * cap + j];
  in.Pi = VISC ? T_[(int64_t)T_PI * cap + j] : 0.0;
  in.eta = VISC ? T_[(int64_t)T_ETA * cap + j] : 0.0;
  in.zeta = VISC ? T_[(int64_t)T_ZETA * cap + j] : 0.0;
  in.taupi = VISC ? T_[(int64_t)T_TAUPI * cap + j] : 1.0;
  in.tauPi = VISC ? T_[(int64_t)T_TAUPIB * cap + j] : 1.0;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
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
#pragma unroll
    for (int i = 1; i < 4; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 1; k < 4; ++k) acc += Gk[k] * in.u[k] * in.pi[k][i];
      in.pi[0][i] = in.pi[i][0] = acc * igam;
    }
    double acc = 0.0;
#pragma unroll
    for (int i = 1; i < 4; ++i) acc += Gk[i] * in.u[i] * in.pi[0][i];
    in.pi[0][0] = acc * igam;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) in.I[k] = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    in.Iq[q] = 0.0;
    in.mu[q] = 0.0;
  }
  // the chemical potentials enter only through the charge sources
  if (prm.src && prm.src->n > 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) in.mu[q] = q < prm.ncharge ? T_[(int64_t)(T_MUB + q) * cap + j] : 0.0;
    double x[3];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = row(Y, cap, R_X1 + k, j);
    source_density<D>(*prm.src, t, sqg, x, in.I, in.Iq);
    if (prm.ncharge == 0) in.Iq[0] = in.Iq[1] = in.Iq[2] = 0.0;
  }
  EomOut o;
  eom_solve<D, VISC>(prm, in, o);
  double dV[3][3], dNd[3] = {0.0, 0.0, 0.0};
  if (prm.diffusion) {
    double V[3][3], dal[3][3], dF[3], dPi[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      dF[q] = b.gsum[(int64_t)(GS_DJB + q) * cap + j];
      dPi[q] = q < D ? b.gsum[(int64_t)(GS_DPI1 + q) * cap + j] : 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        V[q][k] = k < D ? row(Y, cap, R_JB1 + 3 * q + k, j) : 0.0;
        dal[q][k] = k < D ? b.gsum[(int64_t)(GS_DAB1 + 3 * q + k) * cap + j] : 0.0;
      }
    }
    diffusion_rates<D>(prm, in, o, V, dal, dPi, dF, dV, dNd);
  }

  double f[NROW];
#pragma unroll
  for (int r = 0; r < NROW; ++r) f[r] = 0.0;
#pragma unroll
  for (int k = 1; k <= D; ++k) {
    f[R_X1 + k - 1] = in.v[k];
    f[R_U1 + k - 1] = o.a[k];
  }
  f[R_S] = o.dS;
#pragma unroll
  for (int q = 0; q < 3; ++q) f[R_NB + q] = q < prm.ncharge ? o.dN[q] : 0.0;
  if (prm.diffusion) {
    // the charge moved by diffusion, and the entropy it carries (R^S = -mu/T)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      f[R_NB + q] += dNd[q];
      f[R_S] -= T_[(int64_t)(T_MUB + q) * cap + j] * dNd[q] / in.T;
#pragma unroll
      for (int k = 0; k < D; ++k) f[R_JB1 + 3 * q + k] = dV[q][k];
    }
  }
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

  if (mode == 2) {
    const int64_t ii = b.ids[j];
    const int64_t n = E.n;
#pragma unroll
    for (int r = 0; r < NROW; ++r) fout[(int64_t)r * n + ii] = f[r];
    if (aux) {
      aux[X_THETA * n + ii] = o.theta;
#pragma unroll
      for (int k = 1; k <= 3; ++k) aux[(X_F1 + k - 1) * n + ii] = in.F[k];
      // Knudsen and inverse Reynolds numbers ("Particlization", eq. knudsen-reynolds)
      double kns = 0.0, res = 0.0, knb = 0.0, reb = 0.0;
      if (VISC) {
        const double p = T_[(int64_t)T_P * cap + j];
        const double gm[4] = {1.0, -1.0, -1.0, -Gk[3]};
        double pipi = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int k = 0; k < 4; ++k) pipi += in.pi[m][k] * gm[m] * gm[k] * in.pi[m][k];
        kns = in.taupi * sqrt(fabs(o.sigsig));
        res = sqrt(fabs(pipi)) / p;
        knb = in.tauPi * o.theta;
        reb = fabs(in.Pi) / p;
      }
      aux[X_KN_SHEAR * n + ii] = kns;
      aux[X_REINV_SHEAR * n + ii] = res;
      aux[X_KN_BULK * n + ii] = knb;
      aux[X_REINV_BULK * n + ii] = reb;
      double dmu[4], dsl[4];
      surface_element<D>(b, j, in, o, Gk, dmu, dsl);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        aux[(X_DE0 + m) * n + ii] = dmu[m];
        aux[(X_DSIG0 + m) * n + ii] = dsl[m];
      }
    }
    return;
  }
  if (mode == 0 && prm.e_fo > 0.0) {
    const int32_t at = b.fo_mark[j];
    if (at >= 0) {
      double dmu[4], dsl[4];
      surface_element<D>(b, j, in, o, Gk, dmu, dsl);
#pragma unroll
      for (int m = 0; m < 4; ++m) b.fo_rec[(int64_t)at * FO_NCOL + FO_DS0 + m] = dsl[m];
      b.fo_mark[j] = -1;
    }
  }
  const double dt = E.dt;
  bool finite = true;
#pragma unroll
  for (int r = 0; r < NROW; ++r) {
    const bool live = (r <= R_X1 + D - 1) || (r >= R_U1 && r <= R_U1 + D - 1) || r == R_S ||
                      (r >= R_NB && r < R_NB + prm.ncharge) ||
                      (VISC && (r == R_B || r == R_P11 || r == R_P12 || r == R_P22 || r == R_P33 ||
                                (D == 3 && (r == R_P13 || r == R_P23)))) ||
                      (prm.diffusion && r >= R_JB1 && ((r - R_JB1) % 3) < D);
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
  // (a step that keeps its binning already works on the home copies)
  if (mode == 1 && b.warms != b.warm) {
    b.id[j] = b.ids[j];
#pragma unroll
    for (int w = 0; w < NWARM; ++w) b.warm[(int64_t)w * cap + j] = b.warms[(int64_t)w * cap + j];
  }
  if (!finite) {
    atomicAdd(&b.evt[e].nonfinite, 1u);
    atomicMin(&b.evt[e].first_bad, b.ids[j]);
  }
}

// ---------------------------------------------------------------------------
static inline unsigned nblocks(int64_t threads, int bs) { return (unsigned)((threads + bs - 1) / bs); }

// Workgroups of the pair kernels: ceil(n / P) per event, at most one more
// per event than the slots need; surplus workgroups leave at once.
static inline unsigned pair_blocks(const BatchDev& b, int64_t nslots, int P) {
  return nblocks(nslots, P) + (b.max_events > 1 ? (unsigned)b.max_events : 0u);
}

// First workgroup of every event in the pair kernels' grid (ceil(n / P)
// workgroups per active event, none for the others): one workgroup scans the
// event table.  A single simulation keeps tile0 = 0 and needs no scan.
__global__ void __launch_bounds__(256) k_tiles(BatchDev b, int P) {
  __shared__ int32_t s_w[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int32_t run = 0;
  for (int base = 0; base < b.max_events; base += 256) {
    const int m = base + tid;
    int32_t nt = 0;
    if (m < b.max_events && b.evt[m].active) nt = (b.evt[m].n + P - 1) / P;
    int32_t inc = nt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t y = __shfl_up(inc, off, 64);
      if (lane >= off) inc += y;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    int32_t before = 0, total = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      before += a < w ? s_w[a] : 0;
      total += s_w[a];
    }
    if (m < b.max_events) b.evt[m].tile0 = run + before + inc - nt;
    run += total;
    __syncthreads();
  }
}

// A stage kernel launch.  With profiling events (ev = {start, stop}) the
// dispatch itself records them, so a group's time is its kernel's execution
// without the gaps between launches.
#define CCAKE_STAGE_LAUNCH(EV, KERNEL, GRID, BLOCK, ...)                                  \
  do {                                                                                    \
    if (EV)                                                                               \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, s, (EV)[0], (EV)[1], 0, __VA_ARGS__); \
    else                                                                                  \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, s, __VA_ARGS__);                         \
  } while (0)

// mk (profiling): 8 events, start and stop of the density, EoS, gradient and
// update kernels
template <int D, bool VISC, bool MIXED>
static void stage_t(const BatchDev& b, const Params& prm, const EosDev& eos, int64_t nslots, const double* Y,
                    int stage, int mode, double* fout, double* aux, bool rates, hipStream_t s,
                    const hipEvent_t* mk) {
  const unsigned gt = pair_blocks(b, nslots, Team<D>::P), gp = nblocks(nslots, 128);
  const PairExport none{nullptr, 0, nullptr, nullptr};
  const hipEvent_t* ed = mk ? mk + 0 : nullptr;
  const hipEvent_t* ee = mk ? mk + 2 : nullptr;
  const hipEvent_t* eg = mk ? mk + 4 : nullptr;
  const hipEvent_t* em = mk ? mk + 6 : nullptr;
  if (prm.density_mode != 0)
    CCAKE_STAGE_LAUNCH(ed, (k_density<D, MIXED, 0, false>), dim3(gt), dim3(256), b, prm, Y, stage, none);
  else if (prm.ncharge)
    CCAKE_STAGE_LAUNCH(ed, (k_density<D, MIXED, 4, false>), dim3(gt), dim3(256), b, prm, Y, stage, none);
  else
    CCAKE_STAGE_LAUNCH(ed, (k_density<D, MIXED, 1, false>), dim3(gt), dim3(256), b, prm, Y, stage, none);
  // the freeze-out surface is looked for at the step start of a step
  const int fo = (mode == 0 && prm.e_fo > 0.0) ? 1 : 0;
  if (fo) hipLaunchKernelGGL(k_fo_begin, dim3(1), dim3(64), 0, s, b);
  if (prm.ncharge)
    CCAKE_STAGE_LAUNCH(ee, (k_eos<D, VISC, MIXED, 3>), dim3(gp), dim3(128), b, prm, eos, Y, stage, nslots, aux, fo);
  else
    CCAKE_STAGE_LAUNCH(ee, (k_eos<D, VISC, MIXED, 0>), dim3(gp), dim3(128), b, prm, eos, Y, stage, nslots, aux, fo);
  if (!rates) return;
  // diffusion sums: 1 without, 2 with the bulk-pressure gradient
  if (prm.diffusion && (prm.d_JPi[0] != 0.0 || prm.d_JPi[1] != 0.0 || prm.d_JPi[2] != 0.0))
    CCAKE_STAGE_LAUNCH(eg, (k_grad<D, VISC, MIXED, 2>), dim3(gt), dim3(256), b, prm, Y, stage);
  else if (prm.diffusion)
    CCAKE_STAGE_LAUNCH(eg, (k_grad<D, VISC, MIXED, 1>), dim3(gt), dim3(256), b, prm, Y, stage);
  else
    CCAKE_STAGE_LAUNCH(eg, (k_grad<D, VISC, MIXED, 0>), dim3(gt), dim3(256), b, prm, Y, stage);
  // diagnostic evaluations only (never profiled)
  if (aux) hipLaunchKernelGGL((k_fo_grad<D>), dim3(gp), dim3(128), 0, s, b, prm, Y, nslots);
  if (fo) {
    const unsigned gl = nblocks(nslots, 64) < 512 ? nblocks(nslots, 64) : 512;
    hipLaunchKernelGGL((k_fo_grad_list<D>), dim3(gl), dim3(64), 0, s, b, prm, Y);
  }
  CCAKE_STAGE_LAUNCH(em, (k_eom<D, VISC>), dim3(gp), dim3(128), b, prm, Y, stage, mode, nslots, fout, aux);
}

template <int D, bool VISC, bool MIXED>
static void passes_t(const BatchDev& b, const Params& prm, const EosDev& eos, int64_t nslots, int which,
                     double* fout, double* aux, hipStream_t s, const hipEvent_t* marks) {
  if (b.max_events > 1) hipLaunchKernelGGL(k_tiles, dim3(1), dim3(256), 0, s, b, Team<D>::P);
  if (which == 0) {
    stage_t<D, VISC, MIXED>(b, prm, eos, nslots, b.Ys, 0, 0, nullptr, nullptr, true, s, marks);
    stage_t<D, VISC, MIXED>(b, prm, eos, nslots, b.Y1, 1, 1, nullptr, nullptr, true, s, marks ? marks + 8 : nullptr);
  } else {
    stage_t<D, VISC, MIXED>(b, prm, eos, nslots, b.Ys, 0, 2, fout, aux, fout != nullptr, s, nullptr);
  }
}

template <int D, bool MIXED>
static void pairs_cached_t(const BatchDev& b, const Params& prm, int64_t nslots, const PairExport& px,
                           hipStream_t s) {
  if (b.max_events > 1) hipLaunchKernelGGL(k_tiles, dim3(1), dim3(256), 0, s, b, Team<D>::P);
  const dim3 grid(pair_blocks(b, nslots, Team<D>::P));
  if (prm.density_mode != 0)
    hipLaunchKernelGGL((k_density<D, MIXED, 0, true>), grid, dim3(256), 0, s, b, prm, b.Ys, 0, px);
  else if (prm.ncharge)
    hipLaunchKernelGGL((k_density<D, MIXED, 4, true>), grid, dim3(256), 0, s, b, prm, b.Ys, 0, px);
  else
    hipLaunchKernelGGL((k_density<D, MIXED, 1, true>), grid, dim3(256), 0, s, b, prm, b.Ys, 0, px);
}

hipError_t launch_pairs_cached(const BatchDev& b, const Params& prm, int64_t nslots, int64_t* counter,
                               int64_t cap, int32_t* pa, int32_t* pb, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  const PairExport px{counter, cap, pa, pb};
  const int key = (prm.dim == 3 ? 2 : 0) + (prm.mixed ? 1 : 0);
  switch (key) {
    case 0: pairs_cached_t<2, false>(b, prm, nslots, px, s); break;
    case 1: pairs_cached_t<2, true>(b, prm, nslots, px, s); break;
    case 2: pairs_cached_t<3, false>(b, prm, nslots, px, s); break;
    case 3: pairs_cached_t<3, true>(b, prm, nslots, px, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_passes(const BatchDev& b, const Params& prm, const EosDev& eos, int64_t nslots, int which,
                         double* fout, double* aux, hipStream_t s, const hipEvent_t* marks) {
  if (nslots <= 0) return hipSuccess;
  const int key = (prm.dim == 3 ? 4 : 0) + (prm.viscous ? 2 : 0) + (prm.mixed ? 1 : 0);
  switch (key) {
    case 0: passes_t<2, false, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 1: passes_t<2, false, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 2: passes_t<2, true, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 3: passes_t<2, true, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 4: passes_t<3, false, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 5: passes_t<3, false, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 6: passes_t<3, true, false>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
    case 7: passes_t<3, true, true>(b, prm, eos, nslots, which, fout, aux, s, marks); break;
  }
  return hipGetLastError();
}

}  // namespace ccake

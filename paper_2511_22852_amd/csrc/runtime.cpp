// Host runtime of the C ABI declared in include/ccake.h: EoS objects, single
// simulations (a batch of one event) and the workspace layout.  The serving
// loop lives in server.cpp and drives the same launchers with many events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ccake.h"
#include "common.h"
#include "kernels.h"
#include "runtime.h"

using namespace ccake;

namespace ccake {

ccake_status fail(Handle* h, ccake_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h) h->err = buf;
  return code;
}

bool validate_config(const ccake_config* c, std::string* why) {
  if (!c) { *why = "config is NULL"; return false; }
  if (c->dim != 2 && c->dim != 3) { *why = "dim must be 2 or 3"; return false; }
  if (c->coords != CCAKE_CARTESIAN && c->coords != CCAKE_HYPERBOLIC) { *why = "coords must be 0 or 1"; return false; }
  if (c->ncharge != 0 && c->ncharge != 3) { *why = "ncharge must be 0 or 3"; return false; }
  if (c->precision != CCAKE_FP64 && c->precision != CCAKE_MIXED) { *why = "precision must be 0 or 1"; return false; }
  if (c->density_mode != 0 && c->density_mode != 1) { *why = "density_mode must be 0 or 1"; return false; }
  if (!(c->h > 0.0) || !std::isfinite(c->h)) { *why = "h must be positive"; return false; }
  if (!(c->skin >= 0.0)) { *why = "skin must be >= 0"; return false; }
  if (c->viscous) {
    if (!(c->eta_over_s > 0.0)) { *why = "viscous runs need eta_over_s > 0"; return false; }
    if (!(c->taupi_coeff > 0.0) || !(c->tauPi_ratio > 0.0)) { *why = "relaxation-time coefficients must be > 0"; return false; }
    if (!std::isfinite(c->c_pisig)) { *why = "c_pisig must be finite"; return false; }
  }
  if (c->diffusion != 0 && c->diffusion != 1) { *why = "diffusion must be 0 or 1"; return false; }
  if (c->diffusion) {
    if (c->ncharge != 3) { *why = "diffusion needs ncharge 3"; return false; }
    if (!(c->tauJ_coeff > 0.0) || !std::isfinite(c->tauJ_coeff)) { *why = "tauJ_coeff must be > 0"; return false; }
    if (!std::isfinite(c->c_JJ)) { *why = "c_JJ must be finite"; return false; }
    for (int q = 0; q < 3; ++q)
      if (!std::isfinite(c->d_JPi[q])) { *why = "d_JPi must be finite"; return false; }
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(c->kappa_T2[i])) { *why = "kappa_T2 must be finite"; return false; }
  }
  return true;
}

Params to_params(const ccake_config& c) {
  Params p;
  p.dim = c.dim;
  p.hyperbolic = c.coords == CCAKE_HYPERBOLIC;
  p.viscous = c.viscous ? 1 : 0;
  p.ncharge = c.ncharge;
  p.density_mode = c.density_mode;
  p.mixed = c.precision == CCAKE_MIXED;
  p.h = c.h;
  p.eta_over_s = c.eta_over_s;
  p.zeta_peak = c.zeta_peak;
  p.zeta_Tpeak = c.zeta_Tpeak;
  p.zeta_width = c.zeta_width;
  p.taupi_coeff = c.taupi_coeff;
  p.tauPi_ratio = c.tauPi_ratio;
  p.c_PiPi = c.c_PiPi;
  p.c_Pipi = c.c_Pipi;
  p.c_pipi = c.c_pipi;
  p.c_piPi = c.c_piPi;
  p.diffusion = c.diffusion ? 1 : 0;
  p.pad_d = 0;
  for (int i = 0; i < 9; ++i) p.kappa_T2[i] = c.diffusion ? c.kappa_T2[i] : 0.0;
  p.tauJ_coeff = c.diffusion ? c.tauJ_coeff : 1.0;
  p.c_JJ = c.diffusion ? c.c_JJ : 0.0;
  p.c_pisig = c.viscous ? c.c_pisig : 0.0;
  for (int q = 0; q < 3; ++q) p.d_JPi[q] = (c.diffusion && c.viscous) ? c.d_JPi[q] : 0.0;
  p.cell_edge = 2.0 * c.h + c.skin;
  p.e_fo = 0.0;
  return p;
}

uint32_t live_rows(const Params& p) {
  uint32_t m = 0;
  for (int k = 0; k < p.dim; ++k) m |= 1u << (R_X1 + k);
  for (int k = 0; k < p.dim; ++k) m |= 1u << (R_U1 + k);
  m |= 1u << R_S;
  for (int q = 0; q < p.ncharge; ++q) m |= 1u << (R_NB + q);
  if (p.viscous) {
    m |= 1u << R_B;
    m |= (1u << R_P11) | (1u << R_P12) | (1u << R_P22) | (1u << R_P33);
    if (p.dim == 3) m |= (1u << R_P13) | (1u << R_P23);
  }
  if (p.diffusion)
    for (int q = 0; q < 3; ++q)
      for (int k = 0; k < p.dim; ++k) m |= 1u << (R_JB1 + 3 * q + k);
  return m;
}

int64_t cell_capacity(const ccake_config& c, int64_t n) {
  (void)c;
  return 4 * n + 8192;
}

static size_t take(size_t* o, size_t bytes) {
  size_t at = *o;
  *o += (bytes + 255) & ~size_t(255);
  return at;
}

Layout make_layout(int64_t cap, int64_t ccap, int nev, int dim) {
  Layout L;
  size_t o = 0;
  const size_t D8 = sizeof(double), I4 = sizeof(int32_t);
  L.Y0 = take(&o, D8 * NROW * cap);
  L.Ys = take(&o, D8 * NROW * cap);
  L.Y1 = take(&o, D8 * NROW * cap);
  L.th = take(&o, D8 * NTH * cap);
  L.rec = take(&o, D8 * NREC * cap);
  L.recf = take(&o, sizeof(float) * NREC * cap);
  L.drec = take(&o, D8 * NDREC * cap);
  L.warm = take(&o, D8 * NWARM * cap);
  L.warms = take(&o, D8 * NWARM * cap);
  L.dsum = take(&o, D8 * NDSUM * cap);
  L.gsum = take(&o, D8 * NGSUM * cap);
  L.aux = take(&o, D8 * NAUXROW * cap);
  L.id = take(&o, I4 * cap);
  L.ids = take(&o, I4 * cap);
  L.ev = take(&o, I4 * cap);
  L.key = take(&o, I4 * cap);
  L.keys = take(&o, I4 * cap);
  L.perm = take(&o, I4 * cap);
  L.xbin = take(&o, D8 * cap);
  L.rows = take(&o, I4 * ROW_CACHE * cap);
  L.fo_rec = take(&o, D8 * FO_NCOL * cap);
  L.fo_slot = take(&o, I4 * cap);
  L.fo_mark = take(&o, I4 * cap);
  L.fo_ctr = take(&o, I4 * 2);
  L.slist = take(&o, sizeof(uint16_t) * (size_t)list_cap(dim) * cap);
  L.scnt = take(&o, I4 * cap);
  L.cs = take(&o, I4 * (ccap + 1));
  L.cf = take(&o, I4 * (ccap + 1));
  L.evt = take(&o, sizeof(EventDev) * nev);
  L.scratch = take(&o, 64 + D8 * 8 * nev);
  L.src = take(&o, sizeof(SourceSet));
  L.total = o;
  return L;
}

BatchDev bind_batch(char* base, const Layout& L, int64_t cap, int64_t ccap, int nev, int dim) {
  BatchDev b;
  b.Y0 = (double*)(base + L.Y0);
  b.Ys = (double*)(base + L.Ys);
  b.Y1 = (double*)(base + L.Y1);
  b.th = (double*)(base + L.th);
  b.rec = (double*)(base + L.rec);
  b.recf = (float*)(base + L.recf);
  b.drec = (double*)(base + L.drec);
  b.warm = (double*)(base + L.warm);
  b.warms = (double*)(base + L.warms);
  b.dsum = (double*)(base + L.dsum);
  b.gsum = (double*)(base + L.gsum);
  b.id = (int32_t*)(base + L.id);
  b.ids = (int32_t*)(base + L.ids);
  b.ev = (int32_t*)(base + L.ev);
  b.key = (int32_t*)(base + L.key);
  b.keys = (int32_t*)(base + L.keys);
  b.perm = (int32_t*)(base + L.perm);
  b.xbin = (double*)(base + L.xbin);
  b.rows = (int32_t*)(base + L.rows);
  b.fo_rec = (double*)(base + L.fo_rec);
  b.fo_slot = (int32_t*)(base + L.fo_slot);
  b.fo_mark = (int32_t*)(base + L.fo_mark);
  b.fo_ctr = (uint32_t*)(base + L.fo_ctr);
  b.slist = (uint16_t*)(base + L.slist);
  b.scnt = (int32_t*)(base + L.scnt);
  b.cell_start = (int32_t*)(base + L.cs);
  b.cell_fill = (int32_t*)(base + L.cf);
  b.evt = (EventDev*)(base + L.evt);
  b.cap = cap;
  b.ccap = ccap;
  b.max_events = nev;
  return b;
}

}  // namespace ccake

#define HIPCHK(h, expr)                                                                \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail((h), CCAKE_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------- EoS ----

static ccake_status eos_alloc(ccake_eos** out) {
  if (!out) return CCAKE_E_ARG;
  ccake_eos* e = new ccake_eos();
  e->magic = HANDLE_EOS;
  memset(&e->dev, 0, sizeof e->dev);
  e->dev.max_iter = 60;
  e->dev.tol = 1e-13;
  hipError_t he = hipMalloc((void**)&e->d_bad, 64);
  if (he != hipSuccess) {
    delete e;
    return CCAKE_E_NOMEM;
  }
  *out = e;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_eos_create_conformal(ccake_eos** out, double fstar) {
  if (!(fstar > 0.0)) return CCAKE_E_ARG;
  ccake_status st = eos_alloc(out);
  if (st) return st;
  (*out)->dev.kind = EOS_CONFORMAL;
  (*out)->dev.fstar = fstar;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_eos_create_gas(ccake_eos** out, int32_t max_iter, double tol) {
  ccake_status st = eos_alloc(out);
  if (st) return st;
  (*out)->dev.kind = EOS_GAS;
  if (max_iter > 0) (*out)->dev.max_iter = max_iter;
  if (tol > 0.0) (*out)->dev.tol = tol;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_eos_create_table(ccake_eos** out, const int32_t n[4], const double lo[4],
                                               const double hi[4], const double* cols, int32_t max_iter,
                                               double tol) {
  if (!out || !n || !lo || !hi || !cols) return CCAKE_E_ARG;
  for (int k = 0; k < 4; ++k)
    if (n[k] < 2 || !(hi[k] > lo[k]) || !std::isfinite(lo[k]) || !std::isfinite(hi[k])) return CCAKE_E_ARG;
  if (!(lo[0] > 0.0)) return CCAKE_E_ARG;
  // node indices are 32-bit on the device
  if ((int64_t)n[0] * n[1] * n[2] * n[3] > (int64_t)INT32_MAX) return CCAKE_E_ARG;
  ccake_status st = eos_alloc(out);
  if (st) return st;
  ccake_eos* e = *out;
  e->dev.kind = EOS_TABLE;
  if (max_iter > 0) e->dev.max_iter = max_iter;
  if (tol > 0.0) e->dev.tol = tol;
  const int64_t nodes = (int64_t)n[0] * n[1] * n[2] * n[3];
  std::vector<double> tab((size_t)nodes * TC_STRIDE, 0.0);
  // input column c (p, s, nB, nS, nQ, cs2, kappa) -> node slot
  const int slot[7] = {TC_P, TC_S, TC_NB, TC_NS, TC_NQ, TC_CS2, TC_KAP};
  for (int c = 0; c < 7; ++c)
    for (int64_t i = 0; i < nodes; ++i) {
      double v = cols[(size_t)c * nodes + i];
      if (!std::isfinite(v)) {
        ccake_eos_destroy(e);
        *out = nullptr;
        return CCAKE_E_ARG;
      }
      tab[(size_t)i * TC_STRIDE + slot[c]] = v;
    }
  hipError_t he = hipMalloc((void**)&e->d_tab, tab.size() * sizeof(double));
  if (he != hipSuccess) {
    ccake_eos_destroy(e);
    *out = nullptr;
    return CCAKE_E_NOMEM;
  }
  he = hipMemcpy(e->d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    ccake_eos_destroy(e);
    *out = nullptr;
    return CCAKE_E_HIP;
  }
  for (int k = 0; k < 4; ++k) {
    e->dev.n[k] = n[k];
    e->dev.lo[k] = lo[k];
    e->dev.hi[k] = hi[k];
    e->dev.d[k] = (hi[k] - lo[k]) / (double)(n[k] - 1);
    e->dev.inv_d[k] = 1.0 / e->dev.d[k];
  }
  e->dev.tab = e->d_tab;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_eos_build_inverted(ccake_eos* eos, const ccake_inv_grid* g, void* stream) {
  if (!eos || !g) return CCAKE_E_ARG;
  if ((g->ncharge != 0 && g->ncharge != 3) || g->decade_lo >= g->decade_hi || g->decade_lo < -30 ||
      g->decade_hi > 30 || g->per_decade < 1 || g->per_decade > 100000)
    return fail(eos, CCAKE_E_ARG, "ccake_eos_build_inverted: bad s grid");
  InvDev v;
  memset(&v, 0, sizeof v);
  v.ncharge = g->ncharge;
  v.d0 = g->decade_lo;
  v.d1 = g->decade_hi;
  v.P = g->per_decade;
  v.ns = (int64_t)(v.d1 - v.d0) * v.P + 1;
  int64_t nodes = v.ns;
  for (int q = 0; q < 3; ++q) {
    if (g->ncharge) {
      if (g->nx[q] < 2 || g->nx[q] > 100000 || !std::isfinite(g->x_lo[q]) || !std::isfinite(g->x_hi[q]) ||
          !(g->x_hi[q] > g->x_lo[q]))
        return fail(eos, CCAKE_E_ARG, "ccake_eos_build_inverted: bad n/s grid of charge %d", q);
      v.nx[q] = g->nx[q];
      v.xlo[q] = g->x_lo[q];
      v.xhi[q] = g->x_hi[q];
      nodes *= g->nx[q];
    } else {
      v.nx[q] = 1;
    }
  }
  if (nodes > ((int64_t)1 << 28)) return fail(eos, CCAKE_E_CAPACITY, "ccake_eos_build_inverted: %lld nodes", (long long)nodes);
  hipStream_t s = (hipStream_t)stream;
  double* val = nullptr;
  if (hipMalloc((void**)&val, (size_t)nodes * IV_STRIDE * sizeof(double)) != hipSuccess)
    return fail(eos, CCAKE_E_NOMEM, "ccake_eos_build_inverted: %lld nodes", (long long)nodes);
  EosDev fwd = eos->dev;
  fwd.inv.val = nullptr;
  hipError_t he = hipMemsetAsync(eos->d_bad, 0, sizeof(uint32_t), s);
  if (he == hipSuccess) he = launch_inv_build(fwd, v, val, nodes, eos->d_bad, s);
  uint32_t bad = 0;
  if (he == hipSuccess) he = hipMemcpyAsync(&bad, eos->d_bad, sizeof bad, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess || bad) {
    (void)hipFree(val);
    if (he != hipSuccess) return fail(eos, CCAKE_E_HIP, "ccake_eos_build_inverted: %s", hipGetErrorString(he));
    return fail(eos, CCAKE_E_EOS_NOCONV, "ccake_eos_build_inverted: %u node inversions did not converge", bad);
  }
  if (eos->d_inv) (void)hipFree(eos->d_inv);
  eos->d_inv = val;
  v.val = val;
  eos->dev.inv = v;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_eos_offline_eval(ccake_eos* eos, int32_t fallback, int64_t n, const double* in,
                                               double* out, int32_t* inside, void* stream) {
  if (!eos || n < 0 || (n > 0 && (!in || !out || !inside))) return CCAKE_E_ARG;
  if (!eos->dev.inv.val) return fail(eos, CCAKE_E_STATE, "ccake_eos_offline_eval: no inverted table");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(eos, launch_inv_eval(eos->dev, fallback ? 1 : 0, n, in, out, inside, s));
  HIPCHK(eos, hipStreamSynchronize(s));
  return CCAKE_OK;
}

extern "C" ccake_status ccake_eos_destroy(ccake_eos* eos) {
  if (!eos) return CCAKE_OK;
  if (eos->d_tab) (void)hipFree(eos->d_tab);
  if (eos->d_inv) (void)hipFree(eos->d_inv);
  if (eos->d_bad) (void)hipFree(eos->d_bad);
  delete eos;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_eos_invert(ccake_eos* eos, int32_t mode, int32_t ncharge, int64_t n, const double* in,
                                         double* out, int32_t* in_table, void* stream) {
  if (!eos) return CCAKE_E_ARG;
  if ((mode != 0 && mode != 1) || (ncharge != 0 && ncharge != 3) || n < 0 || (n > 0 && (!in || !out)))
    return fail(eos, CCAKE_E_ARG, "ccake_eos_invert: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(eos, hipMemsetAsync(eos->d_bad, 0, sizeof(uint32_t), s));
  HIPCHK(eos, launch_eos_invert(eos->dev, mode, ncharge, n, in, out, in_table, eos->d_bad, s));
  uint32_t bad = 0;
  HIPCHK(eos, hipMemcpyAsync(&bad, eos->d_bad, sizeof bad, hipMemcpyDeviceToHost, s));
  HIPCHK(eos, hipStreamSynchronize(s));
  if (bad) return fail(eos, CCAKE_E_EOS_NOCONV, "%u inversions did not converge", bad);
  return CCAKE_OK;
}

// ------------------------------------------------------------ simulation ----

extern "C" ccake_status ccake_workspace_bytes(const ccake_config* cfg, int64_t n, size_t* bytes) {
  std::string why;
  if (!bytes || n <= 0 || !validate_config(cfg, &why)) return CCAKE_E_ARG;
  if (n > INT32_MAX / 2) return CCAKE_E_CAPACITY;
  *bytes = make_layout(n, cell_capacity(*cfg, n), 1, cfg->dim).total;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_create(ccake_sim** out, const ccake_config* cfg, const ccake_eos* eos, int64_t n,
                                     void* workspace, size_t bytes, void* stream) {
  std::string why;
  if (!out || !eos || !workspace || n <= 0) return CCAKE_E_ARG;
  if (!validate_config(cfg, &why)) return CCAKE_E_ARG;
  if (((uintptr_t)workspace & 255) != 0) return CCAKE_E_ARG;
  if (eos->dev.kind == EOS_CONFORMAL && cfg->ncharge != 0) return CCAKE_E_ARG;
  if (eos->dev.inv.val && eos->dev.inv.ncharge != cfg->ncharge) return CCAKE_E_ARG;
  const int64_t ccap = cell_capacity(*cfg, n);
  Layout L = make_layout(n, ccap, 1, cfg->dim);
  if (bytes < L.total) return CCAKE_E_CAPACITY;
  ccake_sim* s = new ccake_sim();
  s->magic = HANDLE_SIM;
  s->cfg = *cfg;
  s->prm = to_params(*cfg);
  s->eos = eos->dev;
  s->n = n;
  s->ccap = ccap;
  s->L = L;
  s->base = (char*)workspace;
  s->b = bind_batch(s->base, L, n, ccap, 1, cfg->dim);
  s->stream = (hipStream_t)stream;
  s->use_graph = getenv("CCAKE_NO_GRAPH") == nullptr && stream != nullptr;
  s->prm.src = (const SourceSet*)(s->base + L.src);
  if (hipHostMalloc((void**)&s->h_evt, sizeof(EventDev), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&s->h_src, sizeof(SourceSet), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&s->evt_done, hipEventDisableTiming) != hipSuccess) {
    ccake_destroy(s);
    return CCAKE_E_NOMEM;
  }
  memset(s->h_src, 0, sizeof(SourceSet));
  // slot -> event map: every slot belongs to event 0; cell counts start at zero
  // (the binning leaves them zero after every use)
  std::vector<int32_t> ev((size_t)n, 0);
  hipError_t he = hipMemcpy(s->b.ev, ev.data(), n * sizeof(int32_t), hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemset(s->b.cell_fill, 0, sizeof(int32_t) * (ccap + 1));
  if (he == hipSuccess) he = hipMemset(s->base + L.src, 0, sizeof(SourceSet));
  // no freeze-out record yet; no slot marked
  if (he == hipSuccess) he = hipMemset(s->b.fo_mark, 0xFF, sizeof(int32_t) * n);
  if (he == hipSuccess) he = hipMemset(s->b.fo_ctr, 0, 2 * sizeof(uint32_t));
  if (he == hipSuccess) he = hipDeviceSynchronize();
  if (he != hipSuccess) {
    ccake_destroy(s);
    return CCAKE_E_HIP;
  }
  *out = s;
  return CCAKE_OK;
}

static ccake_status write_event(ccake_sim* s, double t, double dt) {
  EventDev E;
  memset(&E, 0, sizeof E);
  E.p_base = 0;
  E.c_base = 0;
  E.n = (int32_t)s->n;
  E.c_cap = (int32_t)s->ccap;
  E.active = 1;
  E.t = t;
  E.dt = dt;
  E.first_bad = INT32_MAX;
  E.edge = s->prm.cell_edge;
  E.rebin = 1;  // a single simulation schedules its binning on the host
  for (int k = 0; k < 3; ++k) {
    E.bb_min[k] = BB_EMPTY_MIN;
    E.bb_max[k] = BB_EMPTY_MAX;
  }
  *s->h_evt = E;
  HIPCHK(s, hipMemcpyAsync(s->b.evt, s->h_evt, sizeof(EventDev), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return CCAKE_OK;
}

static ccake_status fetch_event(ccake_sim* s) {
  HIPCHK(s, hipMemcpyAsync(s->h_evt, s->b.evt, sizeof(EventDev), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return CCAKE_OK;
}

static ccake_status sticky(ccake_sim* s, const EventDev& E) {
  if (E.nonfinite)
    return fail(s, CCAKE_E_NONFINITE, "%u non-finite particle updates (first particle %d)", E.nonfinite,
                E.first_bad);
  if (E.noconv) return fail(s, CCAKE_E_EOS_NOCONV, "%u EoS inversions did not converge", E.noconv);
  if (E.capacity_err) return fail(s, CCAKE_E_CAPACITY, "cell grid capacity exceeded or non-finite positions");
  return CCAKE_OK;
}

// copy [rows][n] from the caller (host or device) into device dst
static ccake_status stage_in(ccake_sim* s, double* dst, const double* src, size_t count, int mem) {
  HIPCHK(s, hipMemcpyAsync(dst, src, count * sizeof(double),
                           mem == CCAKE_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
  return CCAKE_OK;
}

static ccake_status stage_out(ccake_sim* s, double* dst, const double* src, size_t count, int mem) {
  HIPCHK(s, hipMemcpyAsync(dst, src, count * sizeof(double),
                           mem == CCAKE_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return CCAKE_OK;
}

static ccake_status reset_surface(ccake_sim* s);

extern "C" ccake_status ccake_init_particles(ccake_sim* s, double t0, const double* xi, const double* u,
                                             int32_t dens_kind, const double* dens, int32_t mem) {
  if (!s) return CCAKE_E_ARG;
  if (!xi || !u || !dens || (dens_kind != 0 && dens_kind != 1) || (mem != CCAKE_HOST && mem != CCAKE_DEVICE))
    return fail(s, CCAKE_E_ARG, "ccake_init_particles: bad arguments");
  if (!std::isfinite(t0) || (s->prm.hyperbolic && !(t0 > 0.0))) return fail(s, CCAKE_E_ARG, "t0 must be > 0");
  const int64_t n = s->n;
  const int D = s->prm.dim;
  // validate on the host
  std::vector<double> hx((size_t)D * n), hu((size_t)D * n), hd((size_t)4 * n);
  hipMemcpyKind k = mem == CCAKE_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  HIPCHK(s, hipMemcpy(hx.data(), xi, hx.size() * sizeof(double), k));
  HIPCHK(s, hipMemcpy(hu.data(), u, hu.size() * sizeof(double), k));
  HIPCHK(s, hipMemcpy(hd.data(), dens, hd.size() * sizeof(double), k));
  for (double v : hx)
    if (!std::isfinite(v)) return fail(s, CCAKE_E_ARG, "non-finite particle position");
  for (double v : hu)
    if (!std::isfinite(v)) return fail(s, CCAKE_E_ARG, "non-finite flow velocity");
  for (int64_t i = 0; i < 4 * n; ++i)
    if (!std::isfinite(hd[i])) return fail(s, CCAKE_E_ARG, "non-finite density");
  for (int64_t i = 0; i < n; ++i)
    if (!(hd[i] > 0.0)) return fail(s, CCAKE_E_ARG, "entropy / energy density must be positive (particle %lld)", (long long)i);
  std::vector<double> up((size_t)NROW * n, 0.0);
  for (int d = 0; d < D; ++d) {
    memcpy(&up[(size_t)(R_X1 + d) * n], &hx[(size_t)d * n], n * sizeof(double));
    memcpy(&up[(size_t)(R_U1 + d) * n], &hu[(size_t)d * n], n * sizeof(double));
  }
  ccake_status st = write_event(s, t0, 0.0);
  if (st) return st;
  HIPCHK(s, hipMemcpy(s->b.Y1, up.data(), up.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(s, hipMemcpy(s->b.rec, hd.data(), hd.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(s, launch_upload(s->b, 0, n, s->b.Y1, NROW, s->stream));
  HIPCHK(s, launch_bin(s->b, s->prm, 1, n, n, 0x1FFFFu, s->stream));
  HIPCHK(s, launch_init(s->b, s->prm, s->eos, dens_kind, s->b.rec, n, s->stream));
  HIPCHK(s, launch_commit(s->b, n, 0x1FFFFu, s->stream));
  st = reset_surface(s);
  if (st) return st;
  st = fetch_event(s);
  if (st) return st;
  s->t = t0;
  s->initialised = true;
  s->need_bin = true;
  return sticky(s, *s->h_evt);
}

extern "C" ccake_status ccake_set_state(ccake_sim* s, double t, const double* y, int32_t mem) {
  if (!s) return CCAKE_E_ARG;
  if (!y || !std::isfinite(t)) return fail(s, CCAKE_E_ARG, "ccake_set_state: bad arguments");
  ccake_status st = write_event(s, t, 0.0);
  if (st) return st;
  st = stage_in(s, s->b.Y1, y, (size_t)NROW * s->n, mem);
  if (st) return st;
  HIPCHK(s, launch_upload(s->b, 0, s->n, s->b.Y1, NROW, s->stream));
  st = reset_surface(s);
  if (st) return st;
  s->t = t;
  s->initialised = true;
  s->need_bin = true;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_get_state(ccake_sim* s, double* y, int32_t mem) {
  if (!s) return CCAKE_E_ARG;
  if (!y || !s->initialised) return fail(s, CCAKE_E_STATE, "ccake_get_state: not initialised");
  HIPCHK(s, launch_unsort(s->b, 0, s->n, live_rows(s->prm), s->b.Y1, s->stream));
  return stage_out(s, y, s->b.Y1, (size_t)NROW * s->n, mem);
}

extern "C" ccake_status ccake_time(const ccake_sim* s, double* t) {
  if (!s || !t) return CCAKE_E_ARG;
  *t = s->t;
  return CCAKE_OK;
}

// 2 around the binning, then per stage the start and stop events of its four
// kernels (recorded by their dispatches)
static const int PROF_MARKS = 18;

// One Heun step.  With rebin, the particles are binned and gathered into cell
// order first.  Without, the step runs on the home arrays, which the previous
// step left in the cell order of the last binning (its update writes the home
// state at the sorted slots): the stage kernels get a view of the batch whose
// step-start state, warm starts and ids are the home ones, updated in place.
static ccake_status enqueue_step(ccake_sim* s, const hipEvent_t* marks, bool rebin) {
  BatchDev b = s->b;
  if (rebin) {
    HIPCHK(s, launch_bin(s->b, s->prm, 1, s->n, s->n, live_rows(s->prm), s->stream, marks));
  } else {
    if (marks) {
      HIPCHK(s, hipEventRecord(marks[0], s->stream));
      HIPCHK(s, hipEventRecord(marks[1], s->stream));
    }
    b.Ys = b.Y0;
    b.warms = b.warm;
    b.ids = b.id;
  }
  HIPCHK(s, launch_passes(b, s->prm, s->eos, s->n, 0, nullptr, nullptr, s->stream, marks ? marks + 2 : nullptr));
  HIPCHK(s, launch_advance(s->b, s->stream));
  return CCAKE_OK;
}

// Whether the next step of size dt starting at x0 = t must rebin, and the
// bookkeeping of the displacement bound.
static bool next_rebin(ccake_sim* s, double t, double dt) {
  const double vmax = s->prm.hyperbolic && s->prm.dim == 3 ? std::fmax(1.0, 1.0 / t) : 1.0;
  const double d = dt * vmax;
  const bool rebin = s->need_bin || 2.0 * (s->disp_bound + d) > s->cfg.skin;
  if (rebin) s->disp_bound = 0.0;
  s->disp_bound += d;
  s->need_bin = false;
  return rebin;
}

// accumulate the kernel durations of nsteps profiled steps (synchronises)
static ccake_status collect_profile(ccake_sim* s, int nsteps) {
  HIPCHK(s, hipStreamSynchronize(s->stream));
  for (int k = 0; k < nsteps; ++k) {
    const hipEvent_t* m = &s->prof_ev[(size_t)k * PROF_MARKS];
    float a = 0.f;
    HIPCHK(s, hipEventElapsedTime(&a, m[0], m[1]));
    s->prof_ms[0] += a;
    s->prof_n[0] += 1;
    for (int st = 0; st < 2; ++st) {
      const hipEvent_t* q = m + 2 + 8 * st;
      for (int g = 0; g < 4; ++g) {
        float x = 0.f;
        HIPCHK(s, hipEventElapsedTime(&x, q[2 * g], q[2 * g + 1]));
        s->prof_ms[1 + g] += x;
        s->prof_n[1 + g] += 1;
      }
    }
  }
  return CCAKE_OK;
}

extern "C" ccake_status ccake_set_profiling(ccake_sim* s, int32_t enable) {
  if (!s) return CCAKE_E_ARG;
  s->prof = enable != 0;
  for (int k = 0; k < CCAKE_NPROF; ++k) {
    s->prof_ms[k] = 0.0;
    s->prof_n[k] = 0;
  }
  return CCAKE_OK;
}

extern "C" ccake_status ccake_kernel_times(ccake_sim* s, double* ms, int64_t* launches) {
  if (!s || !ms || !launches) return CCAKE_E_ARG;
  for (int k = 0; k < CCAKE_NPROF; ++k) {
    ms[k] = s->prof_ms[k];
    launches[k] = s->prof_n[k];
  }
  return CCAKE_OK;
}

extern "C" ccake_status ccake_step(ccake_sim* s, double dt, int32_t nsteps) {
  if (!s) return CCAKE_E_ARG;
  if (!s->initialised) return fail(s, CCAKE_E_STATE, "ccake_step before initialisation");
  if (!(dt > 0.0) || nsteps < 0) return fail(s, CCAKE_E_ARG, "dt must be > 0 and nsteps >= 0");
  const double vmax = s->prm.hyperbolic && s->prm.dim == 3 ? std::fmax(1.0, 1.0 / s->t) : 1.0;
  if (2.0 * dt * vmax > s->cfg.skin)
    return fail(s, CCAKE_E_ARG, "skin %.4g fm is below 2 dt max(1, 1/x0) = %.4g fm", s->cfg.skin, 2.0 * dt * vmax);
  // sticky errors already visible from an earlier call
  if (s->pending && hipEventQuery(s->evt_done) == hipSuccess) {
    s->pending = false;
    ccake_status st = sticky(s, *s->h_evt);
    if (st) return st;
  }
  if (nsteps == 0) return CCAKE_OK;
  if (s->pending) {
    HIPCHK(s, hipEventSynchronize(s->evt_done));
    s->pending = false;
    ccake_status st = sticky(s, *s->h_evt);
    if (st) return st;
  }
  s->dt_host = dt;
  HIPCHK(s, hipMemcpyAsync(&s->b.evt[0].dt, &s->dt_host, sizeof(double), hipMemcpyHostToDevice, s->stream));
  if (s->prof) {
    // direct launches bracketed by timing events
    const size_t need = (size_t)nsteps * PROF_MARKS;
    while (s->prof_ev.size() < need) {
      hipEvent_t e;
      HIPCHK(s, hipEventCreate(&e));
      s->prof_ev.push_back(e);
    }
    for (int k = 0; k < nsteps; ++k) {
      const bool rebin = next_rebin(s, s->t + k * dt, dt);
      ccake_status st = enqueue_step(s, &s->prof_ev[(size_t)k * PROF_MARKS], rebin);
      if (st) return st;
    }
    ccake_status st = collect_profile(s, nsteps);
    if (st) return st;
    s->t += dt * nsteps;
    HIPCHK(s, hipMemcpyAsync(s->h_evt, s->b.evt, sizeof(EventDev), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipEventRecord(s->evt_done, s->stream));
    s->pending = true;
    return CCAKE_OK;
  }
  for (int k = 0; k < nsteps; ++k) {
    const int rebin = next_rebin(s, s->t + k * dt, dt) ? 1 : 0;
    if (s->use_graph && !s->graph_ready[rebin]) {
      // capture this kind of step once; later steps replay it
      hipError_t e1 = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
      if (e1 == hipSuccess) {
        ccake_status st = enqueue_step(s, nullptr, rebin != 0);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(s->stream, &g);
        if (st == CCAKE_OK && e2 == hipSuccess && g &&
            hipGraphInstantiate(&s->graph[rebin], g, nullptr, nullptr, 0) == hipSuccess) {
          s->graph_ready[rebin] = true;
        } else {
          s->use_graph = false;
        }
        if (g) (void)hipGraphDestroy(g);
      } else {
        s->use_graph = false;
      }
      (void)hipGetLastError();
    }
    if (s->use_graph && s->graph_ready[rebin]) {
      HIPCHK(s, hipGraphLaunch(s->graph[rebin], s->stream));
    } else {
      ccake_status st = enqueue_step(s, nullptr, rebin != 0);
      if (st) return st;
    }
  }
  s->t += dt * nsteps;
  HIPCHK(s, hipMemcpyAsync(s->h_evt, s->b.evt, sizeof(EventDev), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipEventRecord(s->evt_done, s->stream));
  s->pending = true;
  return CCAKE_OK;
}

static_assert(CCAKE_MAX_SOURCES == MAX_SOURCES, "source table size");
static_assert(CCAKE_NAUX == NAUXROW, "diagnostic rows");

extern "C" ccake_status ccake_set_sources(ccake_sim* s, int32_t nsrc, const ccake_source* src) {
  if (!s) return CCAKE_E_ARG;
  if (nsrc < 0 || nsrc > CCAKE_MAX_SOURCES || (nsrc > 0 && !src))
    return fail(s, CCAKE_E_ARG, "ccake_set_sources: nsrc must be in [0, %d]", CCAKE_MAX_SOURCES);
  const int D = s->prm.dim;
  for (int k = 0; k < nsrc; ++k) {
    for (int d = 0; d < D; ++d)
      if (!(src[k].width[d] > 0.0) || !std::isfinite(src[k].width[d]))
        return fail(s, CCAKE_E_ARG, "ccake_set_sources: source %d has a non-positive width", k);
  }
  HIPCHK(s, hipStreamSynchronize(s->stream));  // the staging buffer may still feed an earlier copy
  SourceSet& S = *s->h_src;
  memset(&S, 0, sizeof S);
  S.n = nsrc;
  for (int k = 0; k < nsrc; ++k) {
    SourceDev& d = S.s[k];
    d.norm = 1.0;
    for (int a = 0; a < 3; ++a) {
      d.c0[a] = src[k].x0[a];
      d.vel[a] = src[k].vel[a];
      d.iw2[a] = a < D ? 1.0 / (2.0 * src[k].width[a] * src[k].width[a]) : 0.0;
      if (a < D) d.norm /= std::sqrt(2.0 * 3.14159265358979323846) * src[k].width[a];
    }
    d.t_on = src[k].t_on;
    d.t_off = src[k].t_off;
    for (int m = 0; m < 4; ++m) d.dpdt[m] = src[k].dpdt[m];
    for (int q = 0; q < 3; ++q) d.dndt[q] = q < s->prm.ncharge ? src[k].dndt[q] : 0.0;
  }
  HIPCHK(s, hipMemcpyAsync(s->base + s->L.src, &S, sizeof S, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return CCAKE_OK;
}

extern "C" ccake_status ccake_check(ccake_sim* s) {
  if (!s) return CCAKE_E_ARG;
  ccake_status st = fetch_event(s);
  if (st) return st;
  s->pending = false;
  return sticky(s, *s->h_evt);
}

// evaluation at the current state: bin, pass 1 and (optionally) pass 2 in rate mode
static ccake_status evaluate(ccake_sim* s, bool rates) {
  if (!s->initialised) return fail(s, CCAKE_E_STATE, "not initialised");
  double* aux = (double*)(s->base + s->L.aux);
  HIPCHK(s, hipMemsetAsync(aux, 0, sizeof(double) * NAUXROW * s->n, s->stream));
  HIPCHK(s, launch_bin(s->b, s->prm, 1, s->n, s->n, live_rows(s->prm), s->stream));
  HIPCHK(s, launch_passes(s->b, s->prm, s->eos, s->n, 1, rates ? s->b.Y1 : nullptr, aux, s->stream));
  // the home arrays keep their order while the cells now index the sorted copy
  s->need_bin = true;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_rhs(ccake_sim* s, double* f, double* aux, int32_t mem) {
  if (!s) return CCAKE_E_ARG;
  ccake_status st = evaluate(s, true);
  if (st) return st;
  if (f) {
    st = stage_out(s, f, s->b.Y1, (size_t)NROW * s->n, mem);
    if (st) return st;
  }
  if (aux) {
    st = stage_out(s, aux, (double*)(s->base + s->L.aux), (size_t)NAUXROW * s->n, mem);
    if (st) return st;
  }
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return CCAKE_OK;
}

extern "C" ccake_status ccake_read(ccake_sim* s, int32_t field, double* out, int32_t mem) {
  if (!s) return CCAKE_E_ARG;
  if (field < 0 || field >= CCAKE_NAUX || !out) return fail(s, CCAKE_E_ARG, "ccake_read: bad field");
  ccake_status st = evaluate(s, true);
  if (st) return st;
  return stage_out(s, out, (double*)(s->base + s->L.aux) + (size_t)field * s->n, (size_t)s->n, mem);
}

extern "C" ccake_status ccake_read_fields(ccake_sim* s, uint64_t mask, double* const* out, int32_t mem) {
  if (!s) return CCAKE_E_ARG;
  if (!out || (mask >> CCAKE_NAUX) != 0 || (mem != CCAKE_HOST && mem != CCAKE_DEVICE))
    return fail(s, CCAKE_E_ARG, "ccake_read_fields: bad arguments");
  for (int k = 0; k < CCAKE_NAUX; ++k)
    if (((mask >> k) & 1u) && !out[k]) return fail(s, CCAKE_E_ARG, "ccake_read_fields: field %d has no output", k);
  ccake_status st = evaluate(s, true);
  if (st) return st;
  const double* aux = (const double*)(s->base + s->L.aux);
  for (int k = 0; k < CCAKE_NAUX; ++k)
    if ((mask >> k) & 1u) {
      st = stage_out(s, out[k], aux + (size_t)k * s->n, (size_t)s->n, mem);
      if (st) return st;
    }
  return CCAKE_OK;
}

extern "C" ccake_status ccake_totals(ccake_sim* s, double* out, ccake_counters* cnt) {
  if (!s) return CCAKE_E_ARG;
  if (!out) return fail(s, CCAKE_E_ARG, "ccake_totals: out is NULL");
  ccake_status st = evaluate(s, false);
  if (st) return st;
  double* d = (double*)(s->base + s->L.scratch + 64);
  HIPCHK(s, launch_totals(s->b, s->prm, 1, d, s->stream));
  HIPCHK(s, hipMemcpyAsync(out, d, 8 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  st = fetch_event(s);
  if (st) return st;
  if (cnt) {
    const EventDev& E = *s->h_evt;
    cnt->nonfinite = E.nonfinite;
    cnt->noconv = E.noconv;
    cnt->backup = E.backup;
    cnt->newton_iters = E.newton_iters;
    cnt->first_bad = E.first_bad == INT32_MAX ? -1 : E.first_bad;
    cnt->capacity_err = E.capacity_err;
    // per-particle iterations and table flags of this evaluation
    std::vector<double> it((size_t)s->n), tab((size_t)s->n);
    const double* aux = (const double*)(s->base + s->L.aux);
    st = stage_out(s, it.data(), aux + (size_t)CCAKE_AUX_NEWTON * s->n, (size_t)s->n, CCAKE_HOST);
    if (st) return st;
    st = stage_out(s, tab.data(), aux + (size_t)CCAKE_AUX_INTABLE * s->n, (size_t)s->n, CCAKE_HOST);
    if (st) return st;
    cnt->in_table = 0;
    for (int k = 0; k < CCAKE_NEWTON_BINS; ++k) cnt->newton_hist[k] = 0;
    for (int64_t i = 0; i < s->n; ++i) {
      const double v = it[(size_t)i];
      const int bin = v >= CCAKE_NEWTON_BINS - 1 ? CCAKE_NEWTON_BINS - 1 : (v > 0.0 ? (int)v : 0);
      cnt->newton_hist[bin] += 1;
      cnt->in_table += tab[(size_t)i] != 0.0 ? 1 : 0;
    }
  }
  return CCAKE_OK;
}

extern "C" ccake_status ccake_debug_pairs(ccake_sim* s, int64_t cap, int32_t* a, int32_t* b, int64_t* npairs) {
  if (!s) return CCAKE_E_ARG;
  if (!npairs || cap < 0 || (cap > 0 && (!a || !b))) return fail(s, CCAKE_E_ARG, "ccake_debug_pairs: bad arguments");
  if (!s->initialised) return fail(s, CCAKE_E_STATE, "not initialised");
  int64_t* counter = (int64_t*)(s->base + s->L.scratch);
  HIPCHK(s, launch_bin(s->b, s->prm, 1, s->n, s->n, live_rows(s->prm), s->stream));
  s->need_bin = true;
  HIPCHK(s, hipMemsetAsync(counter, 0, sizeof(int64_t), s->stream));
  HIPCHK(s, launch_pairs(s->b, s->prm, 0, s->n, counter, cap, a, b, s->stream));
  HIPCHK(s, hipMemcpyAsync(npairs, counter, sizeof(int64_t), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return CCAKE_OK;
}

extern "C" ccake_status ccake_debug_pairs_cached(ccake_sim* s, int64_t cap, int32_t* a, int32_t* b,
                                                int64_t* npairs) {
  if (!s) return CCAKE_E_ARG;
  if (!npairs || cap < 0 || (cap > 0 && (!a || !b)))
    return fail(s, CCAKE_E_ARG, "ccake_debug_pairs_cached: bad arguments");
  if (!s->initialised) return fail(s, CCAKE_E_STATE, "not initialised");
  if (s->need_bin) return fail(s, CCAKE_E_STATE, "no binning to reuse: the next step bins first");
  int64_t* counter = (int64_t*)(s->base + s->L.scratch);
  // the view of a step that keeps its binning: the home arrays are in the
  // cell order of the last binning
  BatchDev v = s->b;
  v.Ys = v.Y0;
  v.warms = v.warm;
  v.ids = v.id;
  HIPCHK(s, hipMemsetAsync(counter, 0, sizeof(int64_t), s->stream));
  HIPCHK(s, launch_pairs_cached(v, s->prm, s->n, counter, cap, a, b, s->stream));
  HIPCHK(s, hipMemcpyAsync(npairs, counter, sizeof(int64_t), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return CCAKE_OK;
}

static_assert(CCAKE_FO_NCOL == FO_NCOL && CCAKE_FO_TEMP == FO_TEMP && CCAKE_FO_DS0 == FO_DS0, "record columns");

// forget the surface records and every particle's crossing history (no
// previous energy density, nothing frozen); rows W_EPREV and W_FROZEN are the
// last two warm-start rows, contiguous in both copies
static ccake_status reset_surface(ccake_sim* s) {
  static_assert(W_FROZEN == W_EPREV + 1 && NWARM == W_FROZEN + 1, "surface rows last");
  const size_t cap = (size_t)s->b.cap;
  HIPCHK(s, hipMemsetAsync(s->b.warm + (size_t)W_EPREV * cap, 0, 2 * cap * sizeof(double), s->stream));
  HIPCHK(s, hipMemsetAsync(s->b.warms + (size_t)W_EPREV * cap, 0, 2 * cap * sizeof(double), s->stream));
  HIPCHK(s, hipMemsetAsync(s->b.fo_mark, 0xFF, cap * sizeof(int32_t), s->stream));
  HIPCHK(s, hipMemsetAsync(s->b.fo_ctr, 0, 2 * sizeof(uint32_t), s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return CCAKE_OK;
}

extern "C" ccake_status ccake_set_freezeout(ccake_sim* s, double e_fo) {
  if (!s) return CCAKE_E_ARG;
  if (!(e_fo >= 0.0) || !std::isfinite(e_fo))
    return fail(s, CCAKE_E_ARG, "ccake_set_freezeout: e_fo must be finite and >= 0");
  HIPCHK(s, hipStreamSynchronize(s->stream));
  ccake_status st = reset_surface(s);
  if (st) return st;
  s->prm.e_fo = e_fo;
  // captured steps hold the old parameters
  for (int k = 0; k < 2; ++k) {
    if (s->graph_ready[k]) (void)hipGraphExecDestroy(s->graph[k]);
    s->graph_ready[k] = false;
  }
  return CCAKE_OK;
}

extern "C" ccake_status ccake_freezeout_records(ccake_sim* s, int64_t cap, double* out, int64_t* count,
                                               int32_t mem) {
  if (!s) return CCAKE_E_ARG;
  if (!count || cap < 0 || (cap > 0 && !out) || (mem != CCAKE_HOST && mem != CCAKE_DEVICE))
    return fail(s, CCAKE_E_ARG, "ccake_freezeout_records: bad arguments");
  uint32_t ctr = 0;
  HIPCHK(s, hipMemcpyAsync(&ctr, s->b.fo_ctr, sizeof ctr, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  const int64_t found = std::min<int64_t>((int64_t)ctr, s->b.cap);
  *count = found;
  const int64_t m = std::min(found, cap);
  if (m > 0) return stage_out(s, out, s->b.fo_rec, (size_t)m * FO_NCOL, mem);
  return CCAKE_OK;
}

extern "C" ccake_status ccake_destroy(ccake_sim* s) {
  if (!s) return CCAKE_OK;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (int k = 0; k < 2; ++k)
    if (s->graph_ready[k]) (void)hipGraphExecDestroy(s->graph[k]);
  if (s->evt_done) (void)hipEventDestroy(s->evt_done);
  for (hipEvent_t e : s->prof_ev) (void)hipEventDestroy(e);
  if (s->h_evt) (void)hipHostFree(s->h_evt);
  if (s->h_src) (void)hipHostFree(s->h_src);
  delete s;
  return CCAKE_OK;
}

extern "C" const char* ccake_last_error(const void* handle) {
  if (!handle) return "null handle";
  const Handle* h = (const Handle*)handle;
  if (h->magic != HANDLE_EOS && h->magic != HANDLE_SIM && h->magic != HANDLE_SERVER) return "not a ccake handle";
  return h->err.c_str();
}

// Internal host-side definitions shared by runtime.cpp and server.cpp.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "ccake.h"
#include "common.h"

namespace ccake {

enum : uint32_t { HANDLE_EOS = 0xCCA0E05u, HANDLE_SIM = 0xCCA051Au, HANDLE_SERVER = 0xCCA05E7u };

struct Handle {
  uint32_t magic = 0;
  std::string err;
};

// byte offsets of the arrays of one batch inside its workspace
struct Layout {
  size_t Y0, Ys, Y1, th, rec, recf, drec, warm, warms, dsum, gsum, aux, id, ids, ev, key, keys, perm, xbin, rows, fo_rec, fo_slot, fo_mark, fo_ctr, slist, scnt, cs, cf, evt,
      scratch, src, total;
};

ccake_status fail(Handle* h, ccake_status code, const char* fmt, ...);
bool validate_config(const ccake_config* c, std::string* why);
Params to_params(const ccake_config& c);
uint32_t live_rows(const Params& p);
int64_t cell_capacity(const ccake_config& c, int64_t n);
Layout make_layout(int64_t cap, int64_t ccap, int nev, int dim);
BatchDev bind_batch(char* base, const Layout& L, int64_t cap, int64_t ccap, int nev, int dim);

}  // namespace ccake

struct ccake_eos : ccake::Handle {
  ccake::EosDev dev;
  double* d_tab = nullptr;
  double* d_inv = nullptr;  // offline inverted table (dev.inv.val)
  uint32_t* d_bad = nullptr;
};

struct ccake_sim : ccake::Handle {
  ccake_config cfg;
  ccake::Params prm;
  ccake::EosDev eos;
  ccake::BatchDev b;
  ccake::Layout L;
  char* base = nullptr;
  int64_t n = 0, ccap = 0;
  hipStream_t stream = nullptr;
  double t = 0.0, dt_host = 0.0;
  ccake::SourceSet* h_src = nullptr;  // pinned staging of the source table
  bool initialised = false;
  bool use_graph = false, pending = false;
  // graph[1]: a step that rebins first; graph[0]: a step on the last binning
  bool graph_ready[2] = {false, false};
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  // rebinning schedule: the binning is reused while twice the accumulated
  // displacement bound sum(dt max(1, 1/x0)) since it stays within the skin
  bool need_bin = true;
  double disp_bound = 0.0;
  hipEvent_t evt_done = nullptr;
  ccake::EventDev* h_evt = nullptr;  // pinned copy of the event record
  // kernel timing with HIP events on the simulation's stream (profiling mode)
  bool prof = false;
  std::vector<hipEvent_t> prof_ev;
  double prof_ms[CCAKE_NPROF] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t prof_n[CCAKE_NPROF] = {0, 0, 0, 0, 0};
};

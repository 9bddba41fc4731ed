// Host-side launchers of the HIP kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace ccake {

// marks (optional): 2 events recorded before and after the binning kernels
// max_event_n bounds the particles of any event that is binned
hipError_t launch_bin(const BatchDev& b, const Params& prm, int nevents, int64_t nslots, int64_t max_event_n,
                      uint32_t rowmask, hipStream_t s, const hipEvent_t* marks = nullptr);
// which = 0: full Heun step (two stages); which = 1: pass 1 (+ pass 2 in rate mode when fout != null)
// marks (optional, which = 0): 5 events around pass 1 / pass 2 of both stages
hipError_t launch_passes(const BatchDev& b, const Params& prm, const EosDev& eos, int64_t nslots, int which,
                         double* fout, double* aux, hipStream_t s, const hipEvent_t* marks = nullptr);
hipError_t launch_advance(const BatchDev& b, hipStream_t s);
// only_event >= 0 restricts the initialisation to that event
hipError_t launch_init(const BatchDev& b, const Params& prm, const EosDev& eos, int dens_kind, const double* dens,
                       int64_t nslots, hipStream_t s, int only_event = -1);
hipError_t launch_schedule(const BatchDev& b, double skin, bool hyper3d, hipStream_t s);
hipError_t launch_bin_only(const BatchDev& b, int e, hipStream_t s);
hipError_t launch_commit(const BatchDev& b, int64_t nslots, uint32_t rowmask, hipStream_t s);
hipError_t launch_pairs(const BatchDev& b, const Params& prm, int e, int64_t n, int64_t* counter, int64_t cap,
                        int32_t* pa, int32_t* pb, hipStream_t s);
// the pairs the density pass accepts on the state b.Ys through the slots'
// neighbour rows of the last binning (no binning), original ids
hipError_t launch_pairs_cached(const BatchDev& b, const Params& prm, int64_t nslots, int64_t* counter,
                               int64_t cap, int32_t* pa, int32_t* pb, hipStream_t s);
hipError_t launch_unsort(const BatchDev& b, int e, int64_t n, uint32_t rowmask, double* out, hipStream_t s);
hipError_t launch_upload(const BatchDev& b, int e, int64_t n, const double* in, int nrows, hipStream_t s);
hipError_t launch_totals(const BatchDev& b, const Params& prm, int nevents, double* out, hipStream_t s);
hipError_t launch_inv_build(const EosDev& eos, const InvDev& v, double* val, int64_t nodes, uint32_t* bad,
                            hipStream_t s);
hipError_t launch_inv_eval(const EosDev& eos, int fallback, int64_t n, const double* in, double* out,
                           int32_t* inside, hipStream_t s);
hipError_t launch_eos_invert(const EosDev& eos, int mode, int nq, int64_t n, const double* in, double* out,
                             int32_t* in_table, uint32_t* bad, hipStream_t s);

}  // namespace ccake

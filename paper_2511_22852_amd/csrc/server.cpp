// Serving loop (continuous batching of events); filled in below.
#include "ccake.h"
#include "runtime.h"

using namespace ccake;

struct ccake_server : Handle {};

extern "C" ccake_status ccake_server_create(ccake_server** out, const ccake_config*, const ccake_eos*, size_t, int64_t,
                                            int32_t, double, void*) {
  if (out) *out = nullptr;
  return CCAKE_E_STATE;
}
extern "C" ccake_status ccake_server_submit(ccake_server*, const ccake_event_desc*, int64_t*) { return CCAKE_E_STATE; }
extern "C" ccake_status ccake_server_poll(ccake_server*, ccake_event_result*, int32_t, int32_t*) { return CCAKE_E_STATE; }
extern "C" ccake_status ccake_server_drain(ccake_server*) { return CCAKE_E_STATE; }
extern "C" ccake_status ccake_server_release(ccake_server*, ccake_event_result*) { return CCAKE_E_STATE; }
extern "C" ccake_status ccake_server_stats(ccake_server*, double*, int64_t*, int64_t*, int32_t*) { return CCAKE_E_STATE; }
extern "C" ccake_status ccake_server_destroy(ccake_server*) { return CCAKE_OK; }

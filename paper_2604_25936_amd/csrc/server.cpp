// Serving loop (continuous batching of query requests on one GPU).
#include "sand_host.h"

using namespace sand;

extern "C" sand_status sand_server_create(int device, size_t budget, int32_t precision,
                                          int32_t n_streams, sand_server* out) {
  (void)device; (void)budget; (void)precision; (void)n_streams;
  if (out) *out = nullptr;
  return fail(SAND_ERR_UNSUPPORTED, "sand_server_create: not built yet");
}
extern "C" sand_status sand_server_submit(sand_server, sand_model, sand_depthmap, const float*,
                                          int64_t, float*, uint64_t*) {
  return fail(SAND_ERR_UNSUPPORTED, "sand_server_submit: not built yet");
}
extern "C" sand_status sand_server_wait(sand_server, uint64_t, double, sand_req_stats*) {
  return fail(SAND_ERR_UNSUPPORTED, "sand_server_wait: not built yet");
}
extern "C" void sand_server_destroy(sand_server) {}

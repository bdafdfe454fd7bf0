// Continuous-batching server (placeholder until the batched driver lands).
#include "povar.h"
#include "povar_host.h"

using namespace povar;

extern "C" {
povar_status povar_server_create(povar_ctx ctx, uint64_t, int32_t, povar_server* out) {
  if (out) *out = nullptr;
  set_error(ctx, "server not available in this build");
  return POVAR_ESTATE;
}
povar_status povar_server_submit(povar_server, int32_t, int32_t, int64_t, const int32_t*, const int32_t*,
                                 const double*, const double*, const povar_options*, uint64_t*) {
  return POVAR_ESTATE;
}
povar_status povar_server_poll(povar_server, uint64_t, povar_report*, double*, double*, double*) {
  return POVAR_ESTATE;
}
povar_status povar_server_stats(povar_server, int32_t*, int32_t*, int64_t*, int64_t*) { return POVAR_ESTATE; }
povar_status povar_server_destroy(povar_server) { return POVAR_ESTATE; }
}

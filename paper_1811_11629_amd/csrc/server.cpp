// Continuous-batching server (placeholder until the request loop lands).
#include "host_internal.h"

extern "C" {
int rsaprng_server_create(rsaprng_pool_t, const rsaprng_server_opts*, rsaprng_server_t*) {
  return RSAPRNG_E_ARG;
}
int rsaprng_server_submit(rsaprng_server_t, uint32_t, uint64_t, uint64_t, uint64_t) {
  return RSAPRNG_E_ARG;
}
int rsaprng_server_poll(rsaprng_server_t, rsaprng_completion*, size_t) { return RSAPRNG_E_ARG; }
int rsaprng_server_release(rsaprng_server_t, uint64_t) { return RSAPRNG_E_ARG; }
double rsaprng_server_now(rsaprng_server_t) { return 0.0; }
int rsaprng_server_stats(rsaprng_server_t, uint64_t*, uint64_t*, uint64_t*, uint64_t*) {
  return RSAPRNG_E_ARG;
}
void rsaprng_server_destroy(rsaprng_server_t) {}
}

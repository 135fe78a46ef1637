// Serving request loop.
#include "hrrm.h"
#include "hrrm_ctx.h"

extern "C" {
int hrrm_server_create(hrrm_ctx, size_t, int32_t, int32_t, hrrm_server*) {
  return hrrm::fail(HRRM_EUNSUPPORTED, "server not built yet");
}
int hrrm_server_submit(hrrm_server, const hrrm_request*, uint64_t*) { return HRRM_EUNSUPPORTED; }
int hrrm_server_poll(hrrm_server, uint64_t, hrrm_result*) { return HRRM_EUNSUPPORTED; }
int hrrm_server_release(hrrm_server, uint64_t) { return HRRM_EUNSUPPORTED; }
int hrrm_server_cancel(hrrm_server, uint64_t) { return HRRM_EUNSUPPORTED; }
double hrrm_server_now(hrrm_server) { return 0.0; }
int hrrm_server_destroy(hrrm_server) { return HRRM_OK; }
}

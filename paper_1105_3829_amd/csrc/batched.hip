// Persistent batched kernel (many uneven images in one launch).
#include "hrrm.h"
#include "hrrm_ctx.h"

namespace hrrm {
void Context::release_batch() {}
}  // namespace hrrm

extern "C" {
int32_t hrrm_batch_capacity(void) { return 0; }
int hrrm_median2d_batched(hrrm_ctx, const hrrm_image*, int32_t, void*) {
  return hrrm::fail(HRRM_EUNSUPPORTED, "batched launch not built yet");
}
}

// Tile autotuner.
#include "hrrm.h"
#include "hrrm_ctx.h"

extern "C" {
int hrrm_autotune(hrrm_ctx, hrrm_dtype, int32_t, hrrm_variant, int64_t, int64_t, const char*,
                  int32_t*) {
  return hrrm::fail(HRRM_EUNSUPPORTED, "autotune not built yet");
}
int hrrm_load_tuning(hrrm_ctx, const char*) {
  return hrrm::fail(HRRM_EUNSUPPORTED, "autotune not built yet");
}
}

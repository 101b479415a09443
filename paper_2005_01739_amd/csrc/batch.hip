// Batched boxes (filled in below).
#include "common.h"
extern "C" hipster_status hipster_batch(hipster_ctx *ctx, int, hipster_box_job *, hipster_diag *) {
  if (!ctx) return HIPSTER_EINVAL;
  return HIPSTER_EUNSUPPORTED;
}

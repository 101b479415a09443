// Batched boxes (filled in below).
#include "common.h"
extern "C" hipster_status hipster_batch(hipster_ctx *, int, hipster_box_job *, hipster_diag *) {
  return HIPSTER_EUNSUPPORTED;
}

// Bispectrum kernels (filled in below).
#include "common.h"
extern "C" hipster_status hipster_bk_ell(hipster_ctx *, const hipster_points *, const hipster_points *,
                                         const hipster_params *, double *, hipster_diag *) {
  return HIPSTER_EUNSUPPORTED;
}

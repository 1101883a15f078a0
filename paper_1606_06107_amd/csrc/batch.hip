// Batched shock tubes (declared in include/lbm.h).
#include <hip/hip_runtime.h>

#include "lbm.h"

extern "C" {
size_t lbm_batch_workspace_bytes(const lbm_batch_desc *desc) { (void)desc; return 0; }
lbm_status lbm_batch_init(const lbm_batch_desc *, const double *, const double *, const double *,
                          void *) { return LBM_EUNSUPPORTED; }
lbm_status lbm_batch_step(const lbm_batch_desc *, void *) { return LBM_EUNSUPPORTED; }
lbm_status lbm_batch_moments(const lbm_batch_desc *, double *, double *, double *, void *) {
    return LBM_EUNSUPPORTED;
}
}

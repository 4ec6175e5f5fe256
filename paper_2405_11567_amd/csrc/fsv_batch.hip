// Batched evaluation of many independent instances (built in a later step).
#include <hip/hip_runtime.h>

#include "../../include/fsv.h"

extern "C" {

int fsv_batch_create(fsv_batch **out, const fsv_problem *, int32_t, void *) {
    if (out) *out = nullptr;
    return FSV_ESTATE;
}
int fsv_batch_destroy(fsv_batch *) { return FSV_OK; }
int fsv_batch_energy_grad(fsv_batch *, const double *, double *, double *) { return FSV_ESTATE; }
size_t fsv_batch_bytes(const fsv_batch *) { return 0; }

}  // extern "C"

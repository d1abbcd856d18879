// Batched solves: k right-hand sides against one hierarchy.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace giamg {

int solve_batch(Handle& H, const double* B, double* X, int32_t k, double tol, giamg_info* infos) {
    (void)H; (void)B; (void)X; (void)k; (void)tol; (void)infos;
    throw Error(GIAMG_ENOTSUP, "batched solve not available yet");
}

}  // namespace giamg

// Launcher of the bfloat16 cell operator without the filter's recurrence
// terms (H X and the adjoint's products); the kernel is in cell_bf16.h, the
// variant with the recurrence terms in hx_bf16_epi.hip.
#include "cell_bf16.h"

namespace chfsi {

hipError_t launch_cell_op_bf16(const chfsi_ctx *c, int mode, int flags, double alpha, const void *X, void *Y,
                               int64_t nvec, int64_t ld, hipStream_t s, const EpiArgs *epi) {
    if (mode != MODE_HAM) return hipErrorInvalidValue;
    if (flags & FLAG_EPI) return launch_cell_op_bf16_epi(c, flags, alpha, X, Y, nvec, ld, s, epi);
    return dispatch_cell_bf16<false>(c, flags, alpha, X, Y, nvec, ld, s, nullptr);
}

}  // namespace chfsi

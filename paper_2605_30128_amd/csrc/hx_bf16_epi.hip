// Launcher of the bfloat16 cell operator with the filter step's recurrence
// terms added at the first touch of each node (FLAG_EPI; eq. rChFSIrecurrence).
#include "cell_bf16.h"

namespace chfsi {

hipError_t launch_cell_op_bf16_epi(const chfsi_ctx *c, int flags, double alpha, const void *X, void *Y,
                                   int64_t nvec, int64_t ld, hipStream_t s, const EpiArgs *epi) {
    return dispatch_cell_bf16<true>(c, flags, alpha, X, Y, nvec, ld, s, epi);
}

}  // namespace chfsi

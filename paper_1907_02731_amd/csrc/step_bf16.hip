// Step-kernel instantiations for __bf16 storage: both block shapes, every
// (r_s, r_t), single-clip and batched.
#include "step_kernel.h"

namespace sfseg {

static const detail::StepFns& fns_bf16(int shape, int rs, int rt) {
    static const detail::StepTable<__bf16> table;
    return table.fns[shape][rs * (SFSEG_MAX_RT + 1) + rt];
}

hipError_t launch_step_bf16(int shape, int rs, int rt, const StepParams& p, int grid,
                           hipStream_t s) {
    return fns_bf16(shape, rs, rt).launch(p, grid, s);
}

hipError_t occ_step_bf16(int shape, int rs, int rt, int* blocks) {
    return fns_bf16(shape, rs, rt).occ(blocks);
}

hipError_t launch_batch_bf16(int shape, int rs, int rt, const BatchParams& p, int grid,
                            hipStream_t s) {
    return fns_bf16(shape, rs, rt).batch(p, grid, s);
}

hipError_t occ_batch_bf16(int shape, int rs, int rt, int* blocks) {
    return fns_bf16(shape, rs, rt).batch_occ(blocks);
}

}  // namespace sfseg

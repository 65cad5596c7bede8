// Step-kernel instantiations for float storage: both block shapes, every
// (r_s, r_t), single-clip and batched, and the two-feature-channel step.
#include "step_kernel.h"

namespace sfseg {

// Kernel shapes 0, 1: one feature channel; 2, 3: two (step kernel only).
static const detail::StepFns& fns_f32(int shape, int rs, int rt) {
    static const detail::StepTable<float> table;
    static const detail::StepTable2<float> table2;
    const int comb = rs * (SFSEG_MAX_RT + 1) + rt;
    return shape < 2 ? table.fns[shape][comb] : table2.fns[shape - 2][comb];
}

hipError_t launch_step_f32(int shape, int rs, int rt, const StepParams& p, int grid,
                           hipStream_t s) {
    return fns_f32(shape, rs, rt).launch(p, grid, s);
}

hipError_t occ_step_f32(int shape, int rs, int rt, int* blocks) {
    return fns_f32(shape, rs, rt).occ(blocks);
}

hipError_t launch_batch_f32(int shape, int rs, int rt, const BatchParams& p, int grid,
                            hipStream_t s) {
    const auto& f = fns_f32(shape, rs, rt);
    return f.batch ? f.batch(p, grid, s) : hipErrorInvalidValue;
}

hipError_t occ_batch_f32(int shape, int rs, int rt, int* blocks) {
    const auto& f = fns_f32(shape, rs, rt);
    return f.batch_occ ? f.batch_occ(blocks) : hipErrorInvalidValue;
}

}  // namespace sfseg

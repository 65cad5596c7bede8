// Step-kernel instantiations for float storage: both block shapes, every
// (r_s, r_t), single-clip and batched, the matrix-core step and the
// two-feature-channel step.
#include "step_fused.h"
#include "step_kernel.h"
#include "step_mfma.h"

namespace sfseg {

// Kernel variants 0, 1: one feature channel; 2: matrix-core spatial passes
// (one channel, r_t <= 2); 3: two fused steps (one channel, r_s <= 5,
// r_t <= 2); 4, 5: two channels (step kernel only).
static const detail::StepFns& fns_f32(int shape, int rs, int rt) {
    static const detail::StepTable<float> table;
    static const detail::MfmaTable mfma;
    static const detail::FusedTable fused;
    static const detail::StepTable2<float> table2;
    const int comb = rs * (SFSEG_MAX_RT + 1) + rt;
    if (shape < 2) return table.fns[shape][comb];
    if (shape == SHAPE_MFMA) return mfma.fns[comb];
    if (shape == SHAPE_FUSED2) return fused.fns[comb];
    return table2.fns[shape - STEP_SHAPES][comb];
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

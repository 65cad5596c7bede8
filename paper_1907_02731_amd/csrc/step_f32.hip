// Step-kernel instantiations for float storage, every (r_s, r_t) pair.
#include "step_kernel.h"

namespace sfseg {

hipError_t launch_step_f32(int rs, int rt, const StepParams& p, int grid, hipStream_t s) {
    static const detail::StepTable<float> table;
    return table.launch[rs * (SFSEG_MAX_RT + 1) + rt](p, grid, s);
}

hipError_t occ_step_f32(int rs, int rt, int* blocks) {
    static const detail::StepTable<float> table;
    return table.occ[rs * (SFSEG_MAX_RT + 1) + rt](blocks);
}

}  // namespace sfseg

// Step-kernel instantiations for __bf16 storage: both block shapes, every (r_s, r_t).
#include "step_kernel.h"

namespace sfseg {

static const detail::StepTable<__bf16>& table_bf16() {
    static const detail::StepTable<__bf16> table;
    return table;
}

hipError_t launch_step_bf16(int shape, int rs, int rt, const StepParams& p, int grid,
                           hipStream_t s) {
    return table_bf16().launch[shape][rs * (SFSEG_MAX_RT + 1) + rt](p, grid, s);
}

hipError_t occ_step_bf16(int shape, int rs, int rt, int* blocks) {
    return table_bf16().occ[shape][rs * (SFSEG_MAX_RT + 1) + rt](blocks);
}

}  // namespace sfseg

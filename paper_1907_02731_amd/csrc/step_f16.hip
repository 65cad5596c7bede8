// Step-kernel instantiations for _Float16 storage: both block shapes, every (r_s, r_t).
#include "step_kernel.h"

namespace sfseg {

static const detail::StepTable<_Float16>& table_f16() {
    static const detail::StepTable<_Float16> table;
    return table;
}

hipError_t launch_step_f16(int shape, int rs, int rt, const StepParams& p, int grid,
                           hipStream_t s) {
    return table_f16().launch[shape][rs * (SFSEG_MAX_RT + 1) + rt](p, grid, s);
}

hipError_t occ_step_f16(int shape, int rs, int rt, int* blocks) {
    return table_f16().occ[shape][rs * (SFSEG_MAX_RT + 1) + rt](blocks);
}

}  // namespace sfseg

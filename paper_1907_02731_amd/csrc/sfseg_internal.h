// Internal declarations shared by the kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfseg.h"

namespace sfseg {

// Iteration state kept in device memory.  The fused step kernel reads it at
// launch and its last block writes the next values, so a chain of step
// launches (or a captured graph of them) runs without host round trips.
//
// The iterate is held unnormalised: buffer Y_k with x_k = s * Y_k, where
// s = 1 / ||Y_k|| is computed in float64 from the stored values.  A step
// writes Y_{k+1} = c * M Y_k with the float32 multiplier c = fl32(s * gain).
struct DevState {
    double s;       // 1 / ||Y_k||
    double lambda;  // x_{k-1}^T M x_{k-1} of the last step
    double delta;   // ||x_k - x_{k-1}||_2 of the last step
    double tol;     // stop once delta < tol
    double gain;    // keeps stored values O(1) for 16-bit storage
    float c;        // multiplier applied by the next step
    int32_t k;      // steps done
    int32_t max_iters;
    int32_t done;       // 1: later step launches return at once
    int32_t status;     // SFSEG_OK or the error that stopped the iteration
    int32_t converged;  // delta < tol reached
    uint32_t ticket;    // arrival counter of the current launch (reset by the last block)
    int32_t pad;
};

// Arguments of the fused step kernel (passed by value).
struct StepParams {
    const void* x;  // Y_k, storage dtype, T*H*W
    const void* w;  // S^p, storage dtype
    const void* f;  // F, storage dtype
    void* y;        // Y_{k+1}, storage dtype
    DevState* st;
    double* partials;  // 2 doubles per block
    int32_t T, H, W;
    int32_t tiles_x, tiles_y;
    int64_t n_units;  // tiles_x * tiles_y * T  (tile-major, frame-minor work units)
    float gs[SFSEG_MAX_RS + 1];  // spatial taps g_s[d], d = 0..r_s
    float gt[SFSEG_MAX_RT + 1];  // temporal taps g_t[d], d = 0..r_t
    float alpha;
};

// Output tile of one block and frame: TILE_X columns x TILE_Y rows.
constexpr int STEP_THREADS = 256;
constexpr int TILE_X = 64;
constexpr int TILE_Y = 16;

hipError_t launch_step(int dtype, int rs, int rt, const StepParams& p, int grid,
                       hipStream_t stream);
hipError_t step_max_blocks_per_cu(int dtype, int rs, int rt, int* blocks);

hipError_t launch_prep(int dtype, const float* S, const float* F, double p, void* w, void* f,
                       void* s0, int64_t n, int32_t* bad_flag, int grid, hipStream_t stream);
// Copy the start vector into Y_0 (storage dtype) and set up the state.
// src_is_storage: src points to a storage-dtype volume (the kept copy of S)
// rather than float32.
hipError_t launch_init(int dtype, const void* src, int src_is_storage, void* y0, int64_t n,
                       DevState* st, double* partials, int grid, hipStream_t stream);
hipError_t launch_eigvec(int dtype, const void* y, const DevState* st, float* out, int64_t n,
                         int grid, hipStream_t stream);
hipError_t launch_to_storage(int dtype, const float* src, void* dst, int64_t n, int grid,
                             hipStream_t stream);
hipError_t launch_from_storage(int dtype, const void* src, float* dst, int64_t n, int grid,
                               hipStream_t stream);

}  // namespace sfseg

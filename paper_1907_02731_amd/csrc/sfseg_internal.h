// Internal declarations shared by the kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfseg.h"

namespace sfseg {

// Iteration state kept in device memory, so a chain of step launches (or a
// captured graph of them) runs without host round trips.
//
// The iterate is held unnormalised: buffer Y_k with x_k = s * Y_k, where
// s = 1 / ||Y_k|| is computed in float64 from the stored values.  A step
// writes Y_{k+1} = c * M Y_k with the float32 multiplier c = fl32(s * gain).
//
// Single clips keep two slots, one per iterate buffer.  A step launch reads
// the slot of its input buffer and writes the slot of its output buffer; its
// blocks leave only their float64 partial sums.  The next launch (or a
// one-block finish launch) folds those sums into the state: every one of its
// blocks adds them in the same fixed order, so all take the same scale and
// the same stop decision, and block 0 records the result.  No block waits on
// another inside a launch, so no launch needs a device-wide memory fence.
// Batched clips keep one slot each; a one-block-per-clip launch after each
// batched step folds them.
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
    int32_t pending;    // 1 (2): the partial sums of the step (the two fused steps) that
                        // wrote this slot's buffer are not folded in yet (single clips)
};

// Zero-padded storage layout of every internal volume: frames of Hp x Wp
// elements with the H x W picture at row PT and column PL.  Tiles of
// TILE_X x TILE_Y cover the picture; the padding holds a full halo around
// every tile and is never written with anything but zeros.
struct Layout {
    int32_t T, H, W;
    int32_t Hp, Wp;
    int32_t PT, PL;
    int32_t tiles_x, tiles_y;
    int64_t frame;  // Hp * Wp
    int64_t total;  // T * frame
};

// Arguments of the fused step kernel (passed by value).
struct StepParams {
    const void* x;  // Y_k, storage dtype, padded layout
    const void* w;  // S^p
    const void* f;  // F
    void* y;        // Y_{k+1}
    const DevState* st_in;  // state of x
    DevState* st_out;       // state of y (written by block 0)
    const double* part_in;  // partial sums of the step that wrote x (2 per block)
    double* part_out;       // this launch's partial sums (2 per block)
    const int4* items;   // per logical block: tile origin x, y (picture coords), frames [z, w)
    int32_t T, Wp, PT, PL;
    int64_t frame;
    int64_t fstride;  // elements between consecutive feature channels of f
    float gs[SFSEG_MAX_RS + 1];  // spatial taps g_s[d], d = 0..r_s
    float gt[SFSEG_MAX_RT + 1];  // temporal taps g_t[d], d = 0..r_t
    float alpha;
    int32_t half;  // fused two-step kernel: stop after the first step
};

// One clip of a batch, as the batched step kernel sees it.
struct BatchClip {
    const void* buf[2];  // Y_k ping-pong buffers (storage dtype, padded layout)
    const void* w;
    const void* f;
    DevState* st;
    int64_t frame;
    int32_t T, Wp, PT, PL;
    int32_t first_item, n_items;  // the clip's items are items[first_item .. +n_items)
};

// Arguments of the batched persistent step kernel (passed by value).
struct BatchParams {
    const BatchClip* clips;
    const int4* items;    // {clip, x0 | y0 << 16, t0, t1}
    double* partials;     // 2 doubles per item
    uint32_t* queue;      // [0..7] next offset in each XCD's run, [8] unused
    int32_t qfirst[8];    // first item of each XCD's run
    int32_t qcount[8];    // items in each XCD's run
    int32_t parity;       // clips still iterating read buf[parity], write buf[1 - parity]
    float gs[SFSEG_MAX_RS + 1];
    float gt[SFSEG_MAX_RT + 1];
    float alpha;
};

// Output tile of one block and frame: TILE_X columns x TILE_Y rows.
constexpr int TILE_X = 64;
constexpr int TILE_Y = 16;
// Block shapes of the step kernel: 0 = 256 threads, 4 outputs each along x;
// 1 = 512 threads, 2 outputs each; 2 = 256 threads with the spatial passes on
// the matrix cores (float32 storage, one feature channel, r_t <= 2); 3 = two
// steps fused per launch on 32 x 8 tiles (float32 storage, one feature
// channel, r_s <= 5, r_t <= 2).
constexpr int STEP_SHAPES = 4;
constexpr int SHAPE_MFMA = 2;
constexpr int SHAPE_FUSED2 = 3;
constexpr int MFMA_MAX_RT = 2;
constexpr int FUSED_MAX_RS = 5;
constexpr int FUSED_MAX_RT = 2;
constexpr int FUSED_TILE_X = 32;
constexpr int FUSED_TILE_Y = 8;
// Kernel variant of a plan: 0..3 the block shapes with one feature channel,
// 4..5 shapes 0..1 with two (float32 storage only).
constexpr int KERNEL_VARIANTS = 6;
constexpr int kernel_shape(int shape, int nf) { return nf == 1 ? shape : STEP_SHAPES + shape; }
constexpr int step_threads(int shape) { return shape == 1 ? 512 : 256; }
// Steps one launch of a plan's kernel takes.
constexpr int steps_per_launch(int shape) { return shape == SHAPE_FUSED2 ? 2 : 1; }
// Whether a plan's block shape exists for a storage type, feature-channel
// count and radii (batched contexts: shapes 0..1 only).
constexpr bool shape_supported(int shape, int dtype, int nf, int rs, int rt, bool batch) {
    return shape >= 0 && shape < STEP_SHAPES &&
           (shape != SHAPE_MFMA ||
            (!batch && dtype == SFSEG_F32 && nf == 1 && rt <= MFMA_MAX_RT)) &&
           (shape != SHAPE_FUSED2 || (!batch && dtype == SFSEG_F32 && nf == 1 &&
                                      rs <= FUSED_MAX_RS && rt <= FUSED_MAX_RT));
}

hipError_t launch_step(int dtype, int shape, int rs, int rt, const StepParams& p, int grid,
                       hipStream_t stream);
// One block: fold the partial sums `part` (2 per block of a step launch of
// `nblocks` blocks) into slot st2[slot] if they are pending, then copy the
// state into both slots st2[0] and st2[1].
hipError_t launch_step_finish(DevState* st2, int slot, const double* part, int nblocks,
                              hipStream_t stream);
hipError_t step_max_blocks_per_cu(int dtype, int shape, int rs, int rt, int* blocks);
hipError_t launch_batch_step(int dtype, int shape, int rs, int rt, const BatchParams& p, int grid,
                             hipStream_t stream);
hipError_t batch_max_blocks_per_cu(int dtype, int shape, int rs, int rt, int* blocks);
// After each batched step: one block per clip folds the partial sums of each
// clip that was iterating into its state; block 0 resets the 9 queue counters.
hipError_t launch_batch_finish(const BatchClip* clips, int n_clips, const double* partials,
                               uint32_t* queue, hipStream_t stream);

// Element-wise kernels between unpadded float32 volumes (the ABI) and padded
// storage volumes (the library's internal layout).
hipError_t launch_prep(int dtype, const float* S, const float* F, double p, void* w, void* f,
                       void* s0, const Layout& L, int32_t* bad_flag, int grid,
                       hipStream_t stream);
// Copy the start vector into Y_0 (storage dtype) and set up the state.
// src_is_storage: src is a padded storage volume (the kept copy of S) rather
// than an unpadded float32 volume.
hipError_t launch_init(int dtype, const void* src, int src_is_storage, void* y0, const Layout& L,
                       DevState* st, double* partials, int grid, hipStream_t stream);
hipError_t launch_eigvec(int dtype, const void* y, const DevState* st, float* out,
                         const Layout& L, int grid, hipStream_t stream);
hipError_t launch_to_storage(int dtype, const float* src, void* dst, const Layout& L, int grid,
                             hipStream_t stream);
hipError_t launch_from_storage(int dtype, const void* src, float* dst, const Layout& L, int grid,
                               hipStream_t stream);

}  // namespace sfseg

// Host-side internals shared by the C-ABI translation units: the context
// object, error reporting and layout helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "sfseg.h"
#include "sfseg_internal.h"

namespace sfseg_host {

// Record a message for sfseg_last_error() (per thread) and return `code`.
int fail(int code, const char* fmt, ...);
size_t dtype_size(int dtype);

constexpr int kChunk = 16;  // steps per captured graph / per host check

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::sfseg_host::fail(e_ == hipErrorOutOfMemory ? SFSEG_ERR_OOM          \
                                                                : SFSEG_ERR_HIP,         \
                                      "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                                      __FILE__, __LINE__);                               \
    } while (0)

sfseg::Layout make_layout(const sfseg_config& c);
void axis_taps(int r, double sigma, float* out);
double storage_gain(const sfseg_config& c, int64_t n);
int max_chunks(const sfseg_config& c);
int run_init(hipStream_t stream, const sfseg_config& c, const sfseg::Layout& L, int64_t n,
             const void* src, int src_is_storage, void* y0, sfseg::DevState* st,
             sfseg::DevState* h_st, double* partials, int grid, int32_t max_iters, double tol);

struct BatchState;
void destroy_batch(BatchState* b);

}  // namespace sfseg_host

struct sfseg_ctx;

namespace sfseg_host {
int batch_get_plan(const sfseg_ctx* ctx, sfseg_plan* out);
// Enqueue `count` steps, the first from buf[first_buf & 1]; *last_buf (may
// be NULL) receives the buffer that holds the result.
int launch_steps(sfseg_ctx* ctx, int first_buf, int count, int* last_buf);
// Buffer that holds the iterate after k steps of a run from buf[0].
int buffer_after(const sfseg_ctx* ctx, int k);
// Enqueue the one-block fold that completes the state of buf[slot] (the last
// step's output) and makes slot 0 current.
int launch_finish(sfseg_ctx* ctx, int slot);
int batch_set_plan(sfseg_ctx* ctx, int32_t shape, int32_t chunks);
// y = M x on the context's stream (sfseg_apply without the final wait).
int apply_async(sfseg_ctx* ctx, const float* x, float* y);
}  // namespace sfseg_host

struct sfseg_ctx {
    sfseg_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n = 0;
    void* w = nullptr;   // S^p
    void* f = nullptr;   // F
    void* s0 = nullptr;  // S (default start vector)
    void* buf[2] = {nullptr, nullptr};
    void* apply_in = nullptr;
    void* apply_out = nullptr;
    sfseg::DevState* st = nullptr;        // iteration state, one slot per iterate buffer
                                          // (slot 0 is current after every finish)
    sfseg::DevState* st_apply = nullptr;  // the two slots used by sfseg_apply
    sfseg::DevState* h_st = nullptr;      // pinned host copies: [0] final, [1..2] per-chunk
    int32_t* d_bad = nullptr;
    int32_t* h_bad = nullptr;
    double* partials = nullptr;   // element-wise kernels' block sums
    double* step_part = nullptr;  // step partial sums: set i belongs to the step that wrote buf[i]
    int step_part_slots = 0;      // blocks each set holds
    int4* items = nullptr;  // step-kernel work items, one per block
    size_t items_cap = 0;   // capacity of `items` in entries
    sfseg::Layout L{};
    int cus = 0;
    int nf = 1;             // pairwise feature channels (1 or 2)
    int shape = 0;          // step-kernel block shape (sfseg::step_threads)
    int chunks = 1;         // runs of frames per tile
    int step_grid = 0;
    int ew_grid = 0;  // grid of the element-wise kernels
    int partial_slots = 0;
    sfseg::StepParams params[2]{};  // step from buf[0] -> buf[1] and from buf[1] -> buf[0]
    hipGraphExec_t graph = nullptr;  // kChunk steps starting from buf[0]
    hipEvent_t ev[5]{};
    bool have_iterate = false;
    int cur = 0;  // buffer holding the current iterate
    sfseg_timing timing{};
    sfseg_host::BatchState* batch = nullptr;  // set for contexts made by sfseg_batch_create
    float* spec_buf = nullptr;      // sfseg_spectral_grad: work volume (T*H*W float32)
    double* spec_norms = nullptr;   // sfseg_spectral_grad: ||M y_i|| of the forward products
    int spec_norms_cap = 0;
    double* spec_part = nullptr;    // sfseg_spectral_grad: block sums
    double* h_spec = nullptr;       // pinned copy of the loss sums
    double* ritz_part = nullptr;    // sfseg_refine_frames: frame sums (block shares)
    double* h_ritz = nullptr;       // sfseg_refine_frames: pinned copy of them / the factors
    size_t ritz_cap = 0;            // doubles in ritz_part and h_ritz
    double* ritz_fac = nullptr;     // sfseg_refine_frames: frame factors on the device
    size_t ritz_fac_cap = 0;
};

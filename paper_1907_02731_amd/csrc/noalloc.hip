// sfseg_apply_noalloc: one application y = M x that allocates nothing.
//
// sfseg_apply stages x and y in padded storage-precision volumes that it
// allocates on its first call, sets its state slot with a host copy and
// blocks until the result is back.  Callers that may not allocate device
// memory or block (code under stream capture, serving loops) use this entry
// point instead: the staging volumes, the two state slots and the step
// kernel's float64 partial sums live in one file-scope device array,
// `scratch`, of SFSEG_NOALLOC_SCRATCH_BYTES; every launch is stream-ordered
// and the call returns without waiting.  The kernels are the library's own
// (conversion to storage, the fused step kernel, conversion back), so the
// result equals sfseg_apply's bit for bit.
//
// Each GPU holds its own copy of the array until the process ends.  Its
// device address is taken once per device with hipGetSymbolAddress (in host
// code the symbol's name is a host-side stand-in, never a device address)
// and every kernel argument uses that address.  All calls on one GPU share
// the array: calls that overlap in time on one GPU (two streams, two host
// threads) race and must be ordered by the caller.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "host_internal.h"

using sfseg::DevState;
using sfseg_host::fail;

static __device__ __align__(256) unsigned char scratch[SFSEG_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kAlign = 256;
constexpr size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_scratch[kMaxDevices];  // device address of `scratch`, per device

// Device address of this device's copy of `scratch` (taken on the first call
// on the device, with that device current).
int scratch_address(int device, unsigned char** out) {
    if (device < 0 || device >= kMaxDevices)
        return fail(SFSEG_ERR_INVALID_ARG, "device %d beyond the %d the no-alloc path tracks",
                    device, kMaxDevices);
    std::lock_guard<std::mutex> guard(g_lock);
    if (!g_scratch[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SFSEG_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                        hipGetErrorString(e));
        g_scratch[device] = p;
    }
    *out = (unsigned char*)g_scratch[device];
    return SFSEG_OK;
}

// Zero n16 16-byte words (the staging input's padding must read as zeros; the
// array keeps whatever the previous call on this GPU left in it).
__global__ __launch_bounds__(256) void zero_words(uint4* __restrict__ p, int64_t n16) {
    const uint4 z = {0u, 0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * 256)
        p[i] = z;
}

// State slot of a single application: unit scale, nothing pending, one step.
__global__ void apply_state(DevState* st) {
    if (threadIdx.x == 0) {
        DevState h{};
        h.s = 1.0;
        h.c = 1.0f;
        h.gain = 1.0;
        h.tol = -1.0;
        h.max_iters = 1;
        st[0] = h;
        st[1] = h;
    }
}

}  // namespace

extern "C" {

size_t sfseg_apply_noalloc_bytes(const sfseg_ctx* ctx) {
    if (!ctx || ctx->batch) return 0;
    const size_t vol = round_up((size_t)ctx->L.total * sfseg_host::dtype_size(ctx->cfg.storage));
    const size_t part = round_up(sizeof(double) * 2 * (size_t)ctx->step_grid);
    return round_up(2 * sizeof(DevState)) + part + 2 * vol;
}

int sfseg_apply_noalloc(sfseg_ctx* ctx, const float* x, float* y) {
    if (!ctx || !x || !y) return fail(SFSEG_ERR_INVALID_ARG, "ctx, x or y is NULL");
    if (ctx->batch) return fail(SFSEG_ERR_STATE, "batch context: sfseg_apply_noalloc works on one clip");
    if (x == (const float*)y) return fail(SFSEG_ERR_INVALID_ARG, "x and y may not alias");
    const size_t need = sfseg_apply_noalloc_bytes(ctx);
    if (need > (size_t)SFSEG_NOALLOC_SCRATCH_BYTES)
        return fail(SFSEG_ERR_INVALID_ARG,
                    "volume too large for the no-alloc scratch: needs %zu bytes, the array holds "
                    "%zu (use sfseg_apply)",
                    need, (size_t)SFSEG_NOALLOC_SCRATCH_BYTES);
    HIP_TRY(hipSetDevice(ctx->device));
    unsigned char* base = nullptr;
    if (int rc = scratch_address(ctx->device, &base)) return rc;

    const size_t vol = round_up((size_t)ctx->L.total * sfseg_host::dtype_size(ctx->cfg.storage));
    const size_t part = round_up(sizeof(double) * 2 * (size_t)ctx->step_grid);
    DevState* st = (DevState*)base;
    double* partials = (double*)(base + round_up(2 * sizeof(DevState)));
    void* in = base + round_up(2 * sizeof(DevState)) + part;
    void* out = (unsigned char*)in + vol;

    hipLaunchKernelGGL(zero_words, dim3(1024), dim3(256), 0, ctx->stream, (uint4*)in,
                       (int64_t)(vol / 16));
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(apply_state, dim3(1), dim3(64), 0, ctx->stream, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(sfseg::launch_to_storage(ctx->cfg.storage, x, in, ctx->L, ctx->ew_grid, ctx->stream));
    sfseg::StepParams p = ctx->params[0];
    p.x = in;
    p.y = out;
    p.st_in = st;
    p.st_out = st + 1;
    p.part_in = partials;
    p.part_out = partials;
    p.half = 1;  // one application (the fused kernel's one-step mode)
    HIP_TRY(sfseg::launch_step(ctx->cfg.storage, sfseg::kernel_shape(ctx->shape, ctx->nf),
                               ctx->cfg.r_s, ctx->cfg.r_t, p, ctx->step_grid, ctx->stream));
    HIP_TRY(sfseg::launch_from_storage(ctx->cfg.storage, out, y, ctx->L, ctx->ew_grid,
                                       ctx->stream));
    return SFSEG_OK;
}

}  // extern "C"

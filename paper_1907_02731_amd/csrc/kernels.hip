// Element-wise gfx950 kernels of the SFSeg power iteration (prep, start
// vector, eigenvector output, precision conversions) and the dispatch of the
// fused step kernel (step_kernel.h) over storage precision and radii.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "step_kernel.h"

namespace sfseg {

hipError_t launch_step_f32(int shape, int rs, int rt, const StepParams& p, int grid, hipStream_t s);
hipError_t launch_step_bf16(int shape, int rs, int rt, const StepParams& p, int grid, hipStream_t s);
hipError_t launch_step_f16(int shape, int rs, int rt, const StepParams& p, int grid, hipStream_t s);
hipError_t occ_step_f32(int shape, int rs, int rt, int* blocks);
hipError_t occ_step_bf16(int shape, int rs, int rt, int* blocks);
hipError_t occ_step_f16(int shape, int rs, int rt, int* blocks);
hipError_t launch_batch_f32(int shape, int rs, int rt, const BatchParams& p, int grid, hipStream_t s);
hipError_t launch_batch_bf16(int shape, int rs, int rt, const BatchParams& p, int grid, hipStream_t s);
hipError_t launch_batch_f16(int shape, int rs, int rt, const BatchParams& p, int grid, hipStream_t s);
hipError_t occ_batch_f32(int shape, int rs, int rt, int* blocks);
hipError_t occ_batch_bf16(int shape, int rs, int rt, int* blocks);
hipError_t occ_batch_f16(int shape, int rs, int rt, int* blocks);

namespace {
using detail::Stor;
using detail::block_partials_and_ticket;
using detail::fixed_order_sum;

// Row-parallel element-wise kernels.  Row r of the picture volume (r < T*H)
// is frame t = r / H, line y = r % H: unpadded at r * W, padded at
// t * frame + (y + PT) * Wp + PL.  Blocks stride over rows, threads over x.
__device__ __forceinline__ int64_t padded_row(const Layout& L, int64_t r) {
    const int64_t t = r / L.H, y = r - t * L.H;
    return t * L.frame + (y + L.PT) * (int64_t)L.Wp + L.PL;
}

// ---------------------------------------------------------------------------
// Prep: w = S^p (0^p = 0 for p > 0, w = 1 for p = 0), F and a copy of S in
// storage precision; flags NaN/Inf in S or F and S < 0 with p > 0.
// ---------------------------------------------------------------------------
template <typename TS>
__global__ __launch_bounds__(256) void prep_kernel(const float* __restrict__ S,
                                                   const float* __restrict__ F, float p,
                                                   TS* __restrict__ w, TS* __restrict__ f,
                                                   TS* __restrict__ s0, Layout L,
                                                   int32_t* bad) {
    int badv = 0;
    const int64_t rows = (int64_t)L.T * L.H;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t src = r * L.W, dst = padded_row(L, r);
        for (int x = threadIdx.x; x < L.W; x += blockDim.x) {
            const float sv = S[src + x];
            const float fv = F ? F[src + x] : sv;
            if (!isfinite(sv) || !isfinite(fv) || (p > 0.f && sv < 0.f)) badv = 1;
            const float wv = (p == 0.f) ? 1.f : (sv > 0.f ? powf(sv, p) : 0.f);
            Stor<TS>::st(w, dst + x, wv);
            Stor<TS>::st(f, dst + x, fv);
            Stor<TS>::st(s0, dst + x, sv);
        }
    }
    if (__any(badv) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

// Init: Y_0 = storage(x0); s = 1/||Y_0|| over the stored values; state reset.
template <typename TS>
__global__ __launch_bounds__(256) void init_kernel(const void* __restrict__ src, int src_is_storage,
                                                   TS* __restrict__ y0, Layout L, DevState* st,
                                                   double* partials) {
    __shared__ double fin[256];
    double ss = 0.0, bad = 0.0;
    const int64_t rows = (int64_t)L.T * L.H;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t dst = padded_row(L, r);
        for (int x = threadIdx.x; x < L.W; x += blockDim.x) {
            const float v = src_is_storage ? Stor<TS>::ld((const TS*)src, dst + x)
                                           : ((const float*)src)[r * L.W + x];
            const float q = Stor<TS>::rnd(v);
            if (!isfinite(q)) bad = 1.0;
            Stor<TS>::st(y0, dst + x, q);
            ss = fma((double)q, (double)q, ss);
        }
    }
    if (block_partials_and_ticket<256>(ss, bad, partials, blockIdx.x, &st->ticket, gridDim.x)) {
        const double tss = fixed_order_sum<256>(partials, gridDim.x, 0, fin);
        const double tbad = fixed_order_sum<256>(partials, gridDim.x, 1, fin);
        if (threadIdx.x == 0) {
            const double nrm = sqrt(tss);
            st->k = 0;
            st->converged = 0;
            st->lambda = 0.0;
            st->delta = INFINITY;
            st->status = SFSEG_OK;
            st->done = (st->max_iters <= 0) ? 1 : 0;
            if (tbad > 0.0 || !isfinite(nrm)) {
                st->status = SFSEG_ERR_NONFINITE;
                st->done = 1;
            } else if (!(nrm > 0.0)) {
                st->status = SFSEG_ERR_ZERO_NORM;
                st->done = 1;
            } else {
                st->s = 1.0 / nrm;
                st->c = (float)(st->s * st->gain);
            }
            __hip_atomic_store(&st->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// out = s * Y_k (the unit iterate), float32, unpadded.
template <typename TS>
__global__ __launch_bounds__(256) void eigvec_kernel(const TS* __restrict__ y, const DevState* st,
                                                     float* __restrict__ out, Layout L) {
    const double s = st->s;
    const int64_t rows = (int64_t)L.T * L.H;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t src = padded_row(L, r);
        for (int x = threadIdx.x; x < L.W; x += blockDim.x)
            out[r * L.W + x] = (float)((double)Stor<TS>::ld(y, src + x) * s);
    }
}

template <typename TS>
__global__ __launch_bounds__(256) void to_storage_kernel(const float* __restrict__ src,
                                                         TS* __restrict__ dst, Layout L) {
    const int64_t rows = (int64_t)L.T * L.H;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t d = padded_row(L, r);
        for (int x = threadIdx.x; x < L.W; x += blockDim.x) Stor<TS>::st(dst, d + x, src[r * L.W + x]);
    }
}

template <typename TS>
__global__ __launch_bounds__(256) void from_storage_kernel(const TS* __restrict__ src,
                                                           float* __restrict__ dst, Layout L) {
    const int64_t rows = (int64_t)L.T * L.H;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t sidx = padded_row(L, r);
        for (int x = threadIdx.x; x < L.W; x += blockDim.x) dst[r * L.W + x] = Stor<TS>::ld(src, sidx + x);
    }
}

}  // namespace

// `shape` is a kernel shape (kernel_shape): 0..1 for every storage type,
// 2..3 (two feature channels) for float32 only.
hipError_t launch_step(int dtype, int shape, int rs, int rt, const StepParams& p, int grid,
                       hipStream_t s) {
    if (shape < 0 || shape >= 2 * STEP_SHAPES || (shape >= STEP_SHAPES && dtype != SFSEG_F32) ||
        rs < 0 || rs > SFSEG_MAX_RS || rt < 0 || rt > SFSEG_MAX_RT)
        return hipErrorInvalidValue;
    switch (dtype) {
        case SFSEG_F32: return launch_step_f32(shape, rs, rt, p, grid, s);
        case SFSEG_BF16: return launch_step_bf16(shape, rs, rt, p, grid, s);
        case SFSEG_F16: return launch_step_f16(shape, rs, rt, p, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_step(int dtype, int shape, int rs, int rt, const BatchParams& p, int grid,
                             hipStream_t s) {
    if (shape < 0 || shape >= STEP_SHAPES || rs < 0 || rs > SFSEG_MAX_RS || rt < 0 ||
        rt > SFSEG_MAX_RT)
        return hipErrorInvalidValue;
    switch (dtype) {
        case SFSEG_F32: return launch_batch_f32(shape, rs, rt, p, grid, s);
        case SFSEG_BF16: return launch_batch_bf16(shape, rs, rt, p, grid, s);
        case SFSEG_F16: return launch_batch_f16(shape, rs, rt, p, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t batch_max_blocks_per_cu(int dtype, int shape, int rs, int rt, int* blocks) {
    if (shape < 0 || shape >= STEP_SHAPES || rs < 0 || rs > SFSEG_MAX_RS || rt < 0 ||
        rt > SFSEG_MAX_RT)
        return hipErrorInvalidValue;
    switch (dtype) {
        case SFSEG_F32: return occ_batch_f32(shape, rs, rt, blocks);
        case SFSEG_BF16: return occ_batch_bf16(shape, rs, rt, blocks);
        case SFSEG_F16: return occ_batch_f16(shape, rs, rt, blocks);
        default: return hipErrorInvalidValue;
    }
}

hipError_t step_max_blocks_per_cu(int dtype, int shape, int rs, int rt, int* blocks) {
    if (shape < 0 || shape >= 2 * STEP_SHAPES || (shape >= STEP_SHAPES && dtype != SFSEG_F32) ||
        rs < 0 || rs > SFSEG_MAX_RS || rt < 0 || rt > SFSEG_MAX_RT)
        return hipErrorInvalidValue;
    switch (dtype) {
        case SFSEG_F32: return occ_step_f32(shape, rs, rt, blocks);
        case SFSEG_BF16: return occ_step_bf16(shape, rs, rt, blocks);
        case SFSEG_F16: return occ_step_f16(shape, rs, rt, blocks);
        default: return hipErrorInvalidValue;
    }
}

#define SFSEG_DISPATCH_DTYPE(dtype, TS, ...)          \
    switch (dtype) {                                  \
        case SFSEG_F32: {                             \
            using TS = float;                         \
            __VA_ARGS__;                              \
            break;                                    \
        }                                             \
        case SFSEG_BF16: {                            \
            using TS = __bf16;                        \
            __VA_ARGS__;                              \
            break;                                    \
        }                                             \
        case SFSEG_F16: {                             \
            using TS = _Float16;                      \
            __VA_ARGS__;                              \
            break;                                    \
        }                                             \
        default:                                      \
            return hipErrorInvalidValue;              \
    }

hipError_t launch_prep(int dtype, const float* S, const float* F, double p, void* w, void* f,
                       void* s0, const Layout& L, int32_t* bad, int grid, hipStream_t stream) {
    SFSEG_DISPATCH_DTYPE(dtype, TS,
                         hipLaunchKernelGGL((prep_kernel<TS>), dim3(grid), dim3(256), 0, stream, S,
                                            F, (float)p, (TS*)w, (TS*)f, (TS*)s0, L, bad));
    return hipGetLastError();
}

hipError_t launch_init(int dtype, const void* src, int src_is_storage, void* y0, const Layout& L,
                       DevState* st, double* partials, int grid, hipStream_t stream) {
    SFSEG_DISPATCH_DTYPE(dtype, TS,
                         hipLaunchKernelGGL((init_kernel<TS>), dim3(grid), dim3(256), 0, stream,
                                            src, src_is_storage, (TS*)y0, L, st, partials));
    return hipGetLastError();
}

hipError_t launch_eigvec(int dtype, const void* y, const DevState* st, float* out,
                         const Layout& L, int grid, hipStream_t stream) {
    SFSEG_DISPATCH_DTYPE(dtype, TS,
                         hipLaunchKernelGGL((eigvec_kernel<TS>), dim3(grid), dim3(256), 0, stream,
                                            (const TS*)y, st, out, L));
    return hipGetLastError();
}

hipError_t launch_to_storage(int dtype, const float* src, void* dst, const Layout& L, int grid,
                             hipStream_t stream) {
    SFSEG_DISPATCH_DTYPE(dtype, TS,
                         hipLaunchKernelGGL((to_storage_kernel<TS>), dim3(grid), dim3(256), 0,
                                            stream, src, (TS*)dst, L));
    return hipGetLastError();
}

hipError_t launch_from_storage(int dtype, const void* src, float* dst, const Layout& L, int grid,
                               hipStream_t stream) {
    SFSEG_DISPATCH_DTYPE(dtype, TS,
                         hipLaunchKernelGGL((from_storage_kernel<TS>), dim3(grid), dim3(256), 0,
                                            stream, (const TS*)src, dst, L));
    return hipGetLastError();
}

}  // namespace sfseg

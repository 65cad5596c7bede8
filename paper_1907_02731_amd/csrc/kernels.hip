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
using detail::fixed_order_sum;

// Element-wise kernels walk the picture over a 2D grid: blockIdx.y strides
// over frames, blockIdx.x over groups of kEwRows rows of a frame, threads
// over x (stride 256), with the loads of a group issued before its stores.
// No integer division: a 64-bit division per row on the scalar unit, which
// the CU's waves share, limits a row-linear loop.  Row y of frame t is
// unpadded at (t H + y) W, padded at t frame + (y + PT) Wp + PL.
constexpr int kEwRows = 4;

__device__ __forceinline__ int64_t pic_row(const Layout& L, int t, int y) {
    return ((int64_t)t * L.H + y) * L.W;
}
__device__ __forceinline__ int64_t pad_row(const Layout& L, int t, int y) {
    return (int64_t)t * L.frame + (int64_t)(y + L.PT) * L.Wp + L.PL;
}
__device__ __forceinline__ uint32_t ew_block() { return blockIdx.y * gridDim.x + blockIdx.x; }

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
    // F == NULL reads S twice rather than branching inside the load group
    // (a branch there makes the compiler wait for each row's loads in turn)
    const float* __restrict__ Fv = F ? F : S;
    for (int t = blockIdx.y; t < L.T; t += gridDim.y) {
        for (int y0 = blockIdx.x * kEwRows; y0 < L.H; y0 += gridDim.x * kEwRows) {
            for (int x = threadIdx.x; x < L.W; x += blockDim.x) {
                float sv[kEwRows], fv[kEwRows];
#pragma unroll
                for (int u = 0; u < kEwRows; ++u) {
                    if (y0 + u < L.H) {
                        const int64_t i = pic_row(L, t, y0 + u) + x;
                        sv[u] = S[i];
                        fv[u] = Fv[i];
                    }
                }
#pragma unroll
                for (int u = 0; u < kEwRows; ++u) {
                    if (y0 + u >= L.H) continue;
                    if (!isfinite(sv[u]) || !isfinite(fv[u]) || (p > 0.f && sv[u] < 0.f)) badv = 1;
                    const float wv = (p == 0.f) ? 1.f : (sv[u] > 0.f ? powf(sv[u], p) : 0.f);
                    const int64_t d = pad_row(L, t, y0 + u) + x;
                    Stor<TS>::st(w, d, wv);
                    Stor<TS>::st(f, d, fv[u]);
                    Stor<TS>::st(s0, d, sv[u]);
                }
            }
        }
    }
    if (__any(badv) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

// Init: Y_0 = storage(x0), with each block's sum of Y_0^2 (float64 products
// of float32 values) and a non-finite flag in partials[2 b], partials[2 b + 1].
template <typename TS>
__global__ __launch_bounds__(256) void init_kernel(const void* __restrict__ src, int src_is_storage,
                                                   TS* __restrict__ y0, Layout L,
                                                   double* partials) {
    __shared__ double red[2][4];
    double ss = 0.0, bad = 0.0;
    for (int t = blockIdx.y; t < L.T; t += gridDim.y) {
        for (int r0 = blockIdx.x * kEwRows; r0 < L.H; r0 += gridDim.x * kEwRows) {
            for (int x = threadIdx.x; x < L.W; x += blockDim.x) {
                float v[kEwRows];
#pragma unroll
                for (int u = 0; u < kEwRows; ++u) {
                    if (r0 + u < L.H)
                        v[u] = src_is_storage ? Stor<TS>::ld((const TS*)src, pad_row(L, t, r0 + u) + x)
                                              : ((const float*)src)[pic_row(L, t, r0 + u) + x];
                }
#pragma unroll
                for (int u = 0; u < kEwRows; ++u) {
                    if (r0 + u >= L.H) continue;
                    const float q = Stor<TS>::rnd(v[u]);
                    if (!isfinite(q)) bad = 1.0;
                    Stor<TS>::st(y0, pad_row(L, t, r0 + u) + x, q);
                    ss = fma((double)q, (double)q, ss);
                }
            }
        }
    }
    ss = detail::wave_sum(ss);
    bad = detail::wave_sum(bad);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = ss;
        red[1][threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < (int)blockDim.x / 64; ++i) {
            a += red[0][i];
            b += red[1][i];
        }
        detail::agent_store(partials + 2 * ew_block(), a);
        detail::agent_store(partials + 2 * ew_block() + 1, b);
    }
}

// One block after init_kernel: s = 1/||Y_0|| from the block sums in a fixed
// order, and the rest of the iteration state reset.
__global__ __launch_bounds__(256) void init_finish(DevState* st, const double* partials,
                                                   uint32_t nb) {
    __shared__ double fin[256];
    const double tss = fixed_order_sum<256>(partials, nb, 0, fin);
    const double tbad = fixed_order_sum<256>(partials, nb, 1, fin);
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
    }
}

// out = s * Y_k (the unit iterate), float32, unpadded.
template <typename TS>
__global__ __launch_bounds__(256) void eigvec_kernel(const TS* __restrict__ y, const DevState* st,
                                                     float* __restrict__ out, Layout L) {
    const double s = st->s;
    for (int t = blockIdx.y; t < L.T; t += gridDim.y) {
        for (int r0 = blockIdx.x * kEwRows; r0 < L.H; r0 += gridDim.x * kEwRows) {
            for (int x = threadIdx.x; x < L.W; x += blockDim.x) {
                float v[kEwRows];
#pragma unroll
                for (int u = 0; u < kEwRows; ++u)
                    if (r0 + u < L.H) v[u] = Stor<TS>::ld(y, pad_row(L, t, r0 + u) + x);
#pragma unroll
                for (int u = 0; u < kEwRows; ++u)
                    if (r0 + u < L.H) out[pic_row(L, t, r0 + u) + x] = (float)((double)v[u] * s);
            }
        }
    }
}

template <typename TS>
__global__ __launch_bounds__(256) void to_storage_kernel(const float* __restrict__ src,
                                                         TS* __restrict__ dst, Layout L) {
    for (int t = blockIdx.y; t < L.T; t += gridDim.y) {
        for (int r0 = blockIdx.x * kEwRows; r0 < L.H; r0 += gridDim.x * kEwRows) {
            for (int x = threadIdx.x; x < L.W; x += blockDim.x) {
                float v[kEwRows];
#pragma unroll
                for (int u = 0; u < kEwRows; ++u)
                    if (r0 + u < L.H) v[u] = src[pic_row(L, t, r0 + u) + x];
#pragma unroll
                for (int u = 0; u < kEwRows; ++u)
                    if (r0 + u < L.H) Stor<TS>::st(dst, pad_row(L, t, r0 + u) + x, v[u]);
            }
        }
    }
}

template <typename TS>
__global__ __launch_bounds__(256) void from_storage_kernel(const TS* __restrict__ src,
                                                           float* __restrict__ dst, Layout L) {
    for (int t = blockIdx.y; t < L.T; t += gridDim.y) {
        for (int r0 = blockIdx.x * kEwRows; r0 < L.H; r0 += gridDim.x * kEwRows) {
            for (int x = threadIdx.x; x < L.W; x += blockDim.x) {
                float v[kEwRows];
#pragma unroll
                for (int u = 0; u < kEwRows; ++u)
                    if (r0 + u < L.H) v[u] = Stor<TS>::ld(src, pad_row(L, t, r0 + u) + x);
#pragma unroll
                for (int u = 0; u < kEwRows; ++u)
                    if (r0 + u < L.H) dst[pic_row(L, t, r0 + u) + x] = v[u];
            }
        }
    }
}

// One block: fold a step launch's pending partial sums into st2[slot] and copy
// the state into both slots (the host reads slot 0).
__global__ __launch_bounds__(256) void step_finish(DevState* st2, int slot, const double* part,
                                                   int nblocks) {
    __shared__ double red[2][4];
    const DevState s = detail::state_of_input<256>(st2 + slot, part, nblocks, red);
    if (threadIdx.x == 0) {
        st2[0] = s;
        st2[1] = s;
    }
}

// Block i: fold clip i's item partial sums into its state if it was iterating;
// block 0 also resets the work queues for the next batched step.
__global__ __launch_bounds__(256) void batch_finish(const BatchClip* clips, const double* partials,
                                                    uint32_t* queue) {
    __shared__ double red[2][4];
    const BatchClip& cl = clips[blockIdx.x];
    DevState* st = cl.st;
    if (blockIdx.x == 0 && threadIdx.x < 9) queue[threadIdx.x] = 0u;
    if (st->done) return;
    double syy, syx;
    detail::fold_partials<256>(partials + 2 * (int64_t)cl.first_item, cl.n_items, red, syy, syx);
    if (threadIdx.x == 0) detail::advance_state(st, syy, syx);
}

// 2D grid of at most `blocks` blocks for the element-wise kernels.
dim3 ew_dims(const Layout& L, int blocks) {
    const int gy = L.T < blocks ? L.T : blocks;
    int gx = blocks / gy;
    const int groups = (L.H + kEwRows - 1) / kEwRows;
    if (gx > groups) gx = groups;
    return dim3(gx < 1 ? 1 : gx, gy);
}

}  // namespace

// `shape` is a kernel variant (kernel_shape): 0..1 for every storage type,
// 2 (matrix-core spatial passes, r_t <= 2), 3 (two fused steps, r_s <= 5,
// r_t <= 2) and 4..5 (two feature channels) for float32 only.
static bool variant_ok(int dtype, int shape, int rs, int rt) {
    if (shape < 0 || shape >= KERNEL_VARIANTS || rs < 0 || rs > SFSEG_MAX_RS || rt < 0 ||
        rt > SFSEG_MAX_RT)
        return false;
    if (shape >= 2 && dtype != SFSEG_F32) return false;
    if (shape == SHAPE_MFMA && rt > MFMA_MAX_RT) return false;
    if (shape == SHAPE_FUSED2 && (rs > FUSED_MAX_RS || rt > FUSED_MAX_RT)) return false;
    return true;
}

hipError_t launch_step(int dtype, int shape, int rs, int rt, const StepParams& p, int grid,
                       hipStream_t s) {
    if (!variant_ok(dtype, shape, rs, rt)) return hipErrorInvalidValue;
    switch (dtype) {
        case SFSEG_F32: return launch_step_f32(shape, rs, rt, p, grid, s);
        case SFSEG_BF16: return launch_step_bf16(shape, rs, rt, p, grid, s);
        case SFSEG_F16: return launch_step_f16(shape, rs, rt, p, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_step(int dtype, int shape, int rs, int rt, const BatchParams& p, int grid,
                             hipStream_t s) {
    if (shape < 0 || shape >= 2 || rs < 0 || rs > SFSEG_MAX_RS || rt < 0 ||
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
    if (shape < 0 || shape >= 2 || rs < 0 || rs > SFSEG_MAX_RS || rt < 0 ||
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
    if (!variant_ok(dtype, shape, rs, rt)) return hipErrorInvalidValue;
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

hipError_t launch_batch_finish(const BatchClip* clips, int n_clips, const double* partials,
                               uint32_t* queue, hipStream_t stream) {
    if (n_clips < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_finish, dim3(n_clips), dim3(256), 0, stream, clips, partials, queue);
    return hipGetLastError();
}

hipError_t launch_step_finish(DevState* st2, int slot, const double* part, int nblocks,
                              hipStream_t stream) {
    if (slot < 0 || slot > 1 || nblocks < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(step_finish, dim3(1), dim3(256), 0, stream, st2, slot, part, nblocks);
    return hipGetLastError();
}

hipError_t launch_prep(int dtype, const float* S, const float* F, double p, void* w, void* f,
                       void* s0, const Layout& L, int32_t* bad, int grid, hipStream_t stream) {
    SFSEG_DISPATCH_DTYPE(dtype, TS,
                         hipLaunchKernelGGL((prep_kernel<TS>), ew_dims(L, grid), dim3(256), 0, stream, S,
                                            F, (float)p, (TS*)w, (TS*)f, (TS*)s0, L, bad));
    return hipGetLastError();
}

hipError_t launch_init(int dtype, const void* src, int src_is_storage, void* y0, const Layout& L,
                       DevState* st, double* partials, int grid, hipStream_t stream) {
    const dim3 g = ew_dims(L, grid);
    SFSEG_DISPATCH_DTYPE(dtype, TS,
                         hipLaunchKernelGGL((init_kernel<TS>), g, dim3(256), 0, stream,
                                            src, src_is_storage, (TS*)y0, L, partials));
    hipLaunchKernelGGL(init_finish, dim3(1), dim3(256), 0, stream, st, (const double*)partials,
                       (uint32_t)(g.x * g.y));
    return hipGetLastError();
}

hipError_t launch_eigvec(int dtype, const void* y, const DevState* st, float* out,
                         const Layout& L, int grid, hipStream_t stream) {
    SFSEG_DISPATCH_DTYPE(dtype, TS,
                         hipLaunchKernelGGL((eigvec_kernel<TS>), ew_dims(L, grid), dim3(256), 0, stream,
                                            (const TS*)y, st, out, L));
    return hipGetLastError();
}

hipError_t launch_to_storage(int dtype, const float* src, void* dst, const Layout& L, int grid,
                             hipStream_t stream) {
    SFSEG_DISPATCH_DTYPE(dtype, TS,
                         hipLaunchKernelGGL((to_storage_kernel<TS>), ew_dims(L, grid), dim3(256), 0,
                                            stream, src, (TS*)dst, L));
    return hipGetLastError();
}

hipError_t launch_from_storage(int dtype, const void* src, float* dst, const Layout& L, int grid,
                               hipStream_t stream) {
    SFSEG_DISPATCH_DTYPE(dtype, TS,
                         hipLaunchKernelGGL((from_storage_kernel<TS>), ew_dims(L, grid), dim3(256), 0,
                                            stream, (const TS*)src, dst, L));
    return hipGetLastError();
}

}  // namespace sfseg

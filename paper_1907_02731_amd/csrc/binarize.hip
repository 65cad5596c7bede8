// Binarisation of the solution (Sec. 4.1; Algorithm 1, step 3) on gfx950,
// and its C-ABI entry points (sfseg_project, sfseg_threshold, sfseg_segment).
//
// The projection maps the stored iterate Y through
//     P_i = 1 / (1 + exp(-(a Y_i - b))),  a = slope / max_j Y_j,  b = slope * threshold
// (the sigmoid of slope * (z_i - threshold) with z = Y / max Y) and the hard
// threshold writes mask_i = [Y_i > threshold * max_j Y_j].  Both need the
// maximum over the picture first, so each is two launches: a max reduction
// leaving one maximum per block, then the element-wise pass, whose blocks
// each reduce those maxima first.  The projection's pass also forms per-block
// sums of P^2 in float64 (products of float32 values), and a one-block launch
// adds them in a fixed order and installs the new scale s = 1 / ||P|| and
// step multiplier c = s * gain, so the next step treats P like any other
// iterate.
//
// All three kernels are bound by HBM: rows of the picture in groups of
// kRows per block and pass, each lane taking 4 consecutive voxels (a 16-byte
// float32 or 8-byte 16-bit access; row starts in the padded layout are
// 4-element aligned), with the loads of a group issued before any of its
// stores so that kRows accesses per lane are in flight.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "host_internal.h"
#include "step_kernel.h"

namespace sfseg {
namespace {
using detail::agent_load;
using detail::agent_store;
using detail::fixed_order_sum;
using detail::make_rsrc;
using detail::Stor;

constexpr int kNT = 256;
constexpr int kRows = 4;

// The grid is 2D: blockIdx.y strides over frames, blockIdx.x over groups of
// kRows rows of a frame, so a row's padded offset needs no integer division
// (a 64-bit division per row on the scalar unit, shared by the CU's waves,
// is what limits a row-linear loop).  Block b = y * gridDim.x + x of
// nblocks = gridDim.x * gridDim.y owns partial slot b.

// Byte offset of the first picture voxel of row y of frame t in the padded
// layout (the whole volume is below 2 GiB).
template <typename TS>
__device__ __forceinline__ int row_offset(const Layout& L, int t, int y) {
    return (t * (int)L.frame + (y + L.PT) * L.Wp + L.PL) * (int)sizeof(TS);
}

__device__ __forceinline__ uint32_t block_id() { return blockIdx.y * gridDim.x + blockIdx.x; }
__device__ __forceinline__ uint32_t block_count() { return gridDim.x * gridDim.y; }

__device__ __forceinline__ float block_max(float m, float* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = m;
    __syncthreads();
    float r = red[0];
#pragma unroll
    for (int i = 1; i < kNT / 64; ++i) r = fmaxf(r, red[i]);
    __syncthreads();
    return r;
}

// Maximum over all blocks of max_kernel (partials[2 b], b < nb), the same
// value in every block that calls it.
__device__ __forceinline__ float global_max(const double* partials, uint32_t nb, float* red) {
    float g = -INFINITY;
    for (uint32_t b = threadIdx.x; b < nb; b += kNT) g = fmaxf(g, (float)agent_load(partials + 2 * b));
    return block_max(g, red);
}

// Per-block maximum of the stored iterate over the picture into
// partials[2 b].  The consumers (the next launches) reduce the nb block
// maxima themselves: a kernel boundary makes them visible, where a
// last-block ticket would need an agent-scope fence per block, which on this
// multi-XCD part writes back and invalidates the XCD's L2 and costs more
// than the pass itself.  skip_if_done: return at once when the iteration
// has stopped (inside a run of Algorithm 1).
template <typename TS>
__global__ __launch_bounds__(kNT) void max_kernel(const TS* __restrict__ y, Layout L, DevState* st,
                                                  double* partials, int skip_if_done) {
    if (skip_if_done && st->done) return;
    __shared__ float red[kNT / 64];
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(y, (uint32_t)(L.total * (int64_t)sizeof(TS)));
    const int Q = (L.W + 3) >> 2;
    float m = -INFINITY;
    for (int t = blockIdx.y; t < L.T; t += gridDim.y) {
        for (int y0 = blockIdx.x * kRows; y0 < L.H; y0 += gridDim.x * kRows) {
            const int base = row_offset<TS>(L, t, y0);
            const int pitch = L.Wp * (int)sizeof(TS);
            for (int q = threadIdx.x; q < Q; q += kNT) {
                float v[kRows][4];
#pragma unroll
                for (int u = 0; u < kRows; ++u) {
                    if (y0 + u < L.H) {
                        Stor<TS>::template bloadn<4>(rs, base + u * pitch + 4 * q * (int)sizeof(TS), v[u]);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[u][e] = -INFINITY;
                    }
                }
#pragma unroll
                for (int u = 0; u < kRows; ++u)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (4 * q + e < L.W) m = fmaxf(m, v[u][e]);
            }
        }
    }
    m = block_max(m, red);
    if (threadIdx.x == 0) agent_store(partials + 2 * block_id(), (double)m);
}

// In-place projection of the stored iterate, given the block maxima of
// max_kernel on the same grid; each block's sum of P^2 (float64 products of
// float32 values) goes to partials[2 b + 1].  A maximum that is not positive
// or not finite leaves the iterate alone (project_finish reports it).
template <typename TS>
__global__ __launch_bounds__(kNT) void project_kernel(TS* __restrict__ y, Layout L, DevState* st,
                                                      double* partials, float slope, float thr,
                                                      int skip_if_done) {
    if (skip_if_done && st->done) return;
    __shared__ float red[kNT / 64];
    __shared__ double sred[kNT / 64];
    const uint32_t nb = block_count();
    const float m = global_max(partials, nb, red);
    const bool ok = isfinite(m) && m > 0.f;
    const float a = ok ? (float)((double)slope / (double)m) : 0.f;
    const float b = slope * thr;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(y, (uint32_t)(L.total * (int64_t)sizeof(TS)));
    const int Q = (L.W + 3) >> 2;
    const int T = ok ? L.T : 0;
    double ss = 0.0;
    for (int t = blockIdx.y; t < T; t += gridDim.y) {
        for (int y0 = blockIdx.x * kRows; y0 < L.H; y0 += gridDim.x * kRows) {
            const int base = row_offset<TS>(L, t, y0);
            const int pitch = L.Wp * (int)sizeof(TS);
            for (int q = threadIdx.x; q < Q; q += kNT) {
                const int off = base + 4 * q * (int)sizeof(TS);
                float v[kRows][4];
#pragma unroll
                for (int u = 0; u < kRows; ++u)
                    if (y0 + u < L.H) Stor<TS>::template bloadn<4>(rs, off + u * pitch, v[u]);
#pragma unroll
                for (int u = 0; u < kRows; ++u) {
                    if (y0 + u >= L.H) continue;
                    float pq[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        // voxels past the picture's right edge keep their zeros
                        const float p = __builtin_amdgcn_rcpf(1.0f + expf(b - a * v[u][e]));
                        pq[e] = 4 * q + e < L.W ? Stor<TS>::rnd(p) : 0.f;
                        ss = fma((double)pq[e], (double)pq[e], ss);
                    }
                    Stor<TS>::template bstoren<4>(rs, off + u * pitch, pq);
                }
            }
        }
    }
    ss = detail::wave_sum(ss);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < kNT / 64; ++i) acc += sred[i];
        agent_store(partials + 2 * block_id() + 1, acc);
    }
}

// One block: the fixed-order float64 sum of the projection's block sums, then
// s = 1 / ||P||, c = s * gain in both state slots st[0], st[1] (the next step
// reads the slot of the buffer that holds P); a maximum that is not positive
// or not finite stops the iteration with SFSEG_ERR_ZERO_NORM or
// SFSEG_ERR_NONFINITE.
__global__ __launch_bounds__(kNT) void project_finish(DevState* st, const double* partials,
                                                      uint32_t nb, int skip_if_done) {
    if (skip_if_done && st->done) return;
    __shared__ float red[kNT / 64];
    __shared__ double fin[kNT];
    const float m = global_max(partials, nb, red);
    const double tss = fixed_order_sum<kNT>(partials, nb, 1, fin);
    if (threadIdx.x == 0) {
        DevState s = st[0];
        const double n = sqrt(tss);
        if (!(isfinite(m) && m > 0.f) || !(n > 0.0) || !isfinite(n)) {
            s.status = isfinite(m) ? SFSEG_ERR_ZERO_NORM : SFSEG_ERR_NONFINITE;
            s.done = 1;
        } else {
            s.status = SFSEG_OK;
            s.s = 1.0 / n;
            s.c = (float)(s.s * s.gain);
        }
        st[0] = s;
        st[1] = s;
    }
}

// mask_i = [Y_i > thr * max Y] (the block maxima from max_kernel on the same
// grid); the product of two float32 values is exact in float64.
template <typename TS>
__global__ __launch_bounds__(kNT) void threshold_kernel(const TS* __restrict__ y, Layout L,
                                                        const double* partials, float thr,
                                                        uint8_t* __restrict__ mask) {
    __shared__ float red[kNT / 64];
    const double t_abs = (double)thr * (double)global_max(partials, block_count(), red);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(y, (uint32_t)(L.total * (int64_t)sizeof(TS)));
    const int Q = (L.W + 3) >> 2;
    for (int t = blockIdx.y; t < L.T; t += gridDim.y) {
        for (int y0 = blockIdx.x * kRows; y0 < L.H; y0 += gridDim.x * kRows) {
            const int base = row_offset<TS>(L, t, y0);
            const int pitch = L.Wp * (int)sizeof(TS);
            for (int q = threadIdx.x; q < Q; q += kNT) {
                float v[kRows][4];
#pragma unroll
                for (int u = 0; u < kRows; ++u)
                    if (y0 + u < L.H)
                        Stor<TS>::template bloadn<4>(rs, base + u * pitch + 4 * q * (int)sizeof(TS), v[u]);
#pragma unroll
                for (int u = 0; u < kRows; ++u) {
                    if (y0 + u >= L.H) continue;
                    uint8_t* row = mask + ((int64_t)t * L.H + y0 + u) * L.W;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (4 * q + e < L.W) row[4 * q + e] = (double)v[u][e] > t_abs ? 1 : 0;
                }
            }
        }
    }
}

}  // namespace

#define SFSEG_BIN_DISPATCH(dtype, ...)                 \
    switch (dtype) {                                   \
        case SFSEG_F32: {                              \
            using TS = float;                          \
            __VA_ARGS__;                               \
            break;                                     \
        }                                              \
        case SFSEG_BF16: {                             \
            using TS = __bf16;                         \
            __VA_ARGS__;                               \
            break;                                     \
        }                                              \
        case SFSEG_F16: {                              \
            using TS = _Float16;                       \
            __VA_ARGS__;                               \
            break;                                     \
        }                                              \
        default:                                       \
            return hipErrorInvalidValue;               \
    }

// 2D grid of at most `blocks` blocks: frames over y, row groups over x.
static dim3 bin_dims(const Layout& L, int blocks) {
    const int gy = L.T < blocks ? L.T : blocks;
    int gx = blocks / gy;
    const int groups = (L.H + kRows - 1) / kRows;
    if (gx > groups) gx = groups;
    return dim3(gx < 1 ? 1 : gx, gy);
}

// The max and element-wise launches share one grid of at most `blocks`
// blocks; partials must hold 2 * blocks doubles.
hipError_t launch_project(int dtype, void* y, const Layout& L, DevState* st, double* partials,
                          float slope, float thr, int skip_if_done, int blocks, hipStream_t s) {
    const dim3 g = bin_dims(L, blocks);
    SFSEG_BIN_DISPATCH(dtype,
        hipLaunchKernelGGL((max_kernel<TS>), g, dim3(kNT), 0, s, (const TS*)y, L, st,
                           partials, skip_if_done);
        hipLaunchKernelGGL((project_kernel<TS>), g, dim3(kNT), 0, s, (TS*)y, L, st,
                           partials, slope, thr, skip_if_done));
    hipLaunchKernelGGL(project_finish, dim3(1), dim3(kNT), 0, s, st, (const double*)partials,
                       (uint32_t)(g.x * g.y), skip_if_done);
    return hipGetLastError();
}

hipError_t launch_threshold(int dtype, const void* y, const Layout& L, DevState* st,
                            double* partials, float thr, uint8_t* mask, int blocks,
                            hipStream_t s) {
    const dim3 g = bin_dims(L, blocks);
    SFSEG_BIN_DISPATCH(dtype,
        hipLaunchKernelGGL((max_kernel<TS>), g, dim3(kNT), 0, s, (const TS*)y, L, st,
                           partials, 0);
        hipLaunchKernelGGL((threshold_kernel<TS>), g, dim3(kNT), 0, s, (const TS*)y, L,
                           partials, thr, mask));
    return hipGetLastError();
}

}  // namespace sfseg

using sfseg::DevState;
using namespace sfseg_host;

namespace {

// Grid of the binarisation kernels: at most half the element-wise grid (four
// 256-thread blocks per CU).
int bin_grid(const sfseg_ctx* ctx) {
    const int g = ctx->ew_grid / 2;
    return g < 1 ? 1 : g;
}

int check_ctx(sfseg_ctx* ctx) {
    if (!ctx) return fail(SFSEG_ERR_INVALID_ARG, "ctx is NULL");
    if (ctx->batch) return fail(SFSEG_ERR_STATE, "batch context: binarisation works on one clip");
    if (bin_grid(ctx) > ctx->partial_slots)
        return fail(SFSEG_ERR_STATE, "partials buffer too small");
    return SFSEG_OK;
}

int check_params(float slope, float threshold) {
    if (!(slope > 0.f) || !isfinite(slope))
        return fail(SFSEG_ERR_INVALID_ARG, "slope must be finite and > 0");
    if (!isfinite(threshold)) return fail(SFSEG_ERR_INVALID_ARG, "threshold must be finite");
    return SFSEG_OK;
}

int state_error(int status, int k) {
    return fail(status, status == SFSEG_ERR_ZERO_NORM
                            ? "zero norm or no positive entry (iteration %d)"
                            : "non-finite value (iteration %d)",
                k);
}

}  // namespace

extern "C" {

void sfseg_binarize_default(sfseg_binarize* b) {
    if (!b) return;
    b->iters = 5;
    b->project_from = 3;
    b->slope = 10.0f;
    b->threshold = 0.5f;
}

int sfseg_project(sfseg_ctx* ctx, float slope, float threshold) {
    int rc = check_ctx(ctx);
    if (rc != SFSEG_OK) return rc;
    rc = check_params(slope, threshold);
    if (rc != SFSEG_OK) return rc;
    if (!ctx->have_iterate) return fail(SFSEG_ERR_STATE, "no iterate: call sfseg_power_iterate first");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(sfseg::launch_project(ctx->cfg.storage, ctx->buf[ctx->cur], ctx->L, ctx->st,
                                  ctx->partials, slope, threshold, 0, bin_grid(ctx), ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->h_st, ctx->st, sizeof(DevState), hipMemcpyDeviceToHost,
                           ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (ctx->h_st->status != SFSEG_OK) return state_error(ctx->h_st->status, ctx->h_st->k);
    return SFSEG_OK;
}

int sfseg_threshold(sfseg_ctx* ctx, float threshold, uint8_t* mask) {
    int rc = check_ctx(ctx);
    if (rc != SFSEG_OK) return rc;
    if (!mask) return fail(SFSEG_ERR_INVALID_ARG, "mask is NULL");
    if (!isfinite(threshold)) return fail(SFSEG_ERR_INVALID_ARG, "threshold must be finite");
    if (!ctx->have_iterate) return fail(SFSEG_ERR_STATE, "no iterate: call sfseg_power_iterate first");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(sfseg::launch_threshold(ctx->cfg.storage, ctx->buf[ctx->cur], ctx->L, ctx->st,
                                    ctx->partials, threshold, mask, bin_grid(ctx), ctx->stream));
    return SFSEG_OK;
}

int sfseg_segment(sfseg_ctx* ctx, const float* x0, const sfseg_binarize* b, uint8_t* mask,
                  sfseg_result* res) {
    int rc = check_ctx(ctx);
    if (rc != SFSEG_OK) return rc;
    if (!b) return fail(SFSEG_ERR_INVALID_ARG, "b is NULL");
    if (b->iters < 1) return fail(SFSEG_ERR_INVALID_ARG, "iters must be >= 1");
    if (b->project_from < 1) return fail(SFSEG_ERR_INVALID_ARG, "project_from must be >= 1");
    rc = check_params(b->slope, b->threshold);
    if (rc != SFSEG_OK) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->have_iterate = false;

    HIP_TRY(hipEventRecord(ctx->ev[0], ctx->stream));
    rc = run_init(ctx->stream, ctx->cfg, ctx->L, ctx->n, x0 ? (const void*)x0 : ctx->s0, x0 ? 0 : 1,
                  ctx->buf[0], ctx->st, ctx->h_st, ctx->partials, ctx->ew_grid, b->iters, -1.0);
    if (rc != SFSEG_OK) return rc;
    HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));
    const int grid = bin_grid(ctx);
    for (int k = 1; k <= b->iters; ++k) {
        rc = launch_steps(ctx, (k - 1) & 1, 1, nullptr);
        if (rc != SFSEG_OK) return rc;
        if (b->project_from <= k && k < b->iters) {
            rc = launch_finish(ctx, k & 1);  // the projection needs the step's norm
            if (rc != SFSEG_OK) return rc;
            HIP_TRY(sfseg::launch_project(ctx->cfg.storage, ctx->buf[k & 1], ctx->L, ctx->st,
                                          ctx->partials, b->slope, b->threshold, 1, grid,
                                          ctx->stream));
        }
    }
    rc = launch_finish(ctx, b->iters & 1);
    if (rc != SFSEG_OK) return rc;
    if (mask)
        HIP_TRY(sfseg::launch_threshold(ctx->cfg.storage, ctx->buf[b->iters & 1], ctx->L, ctx->st,
                                        ctx->partials, b->threshold, mask, grid, ctx->stream));
    HIP_TRY(hipEventRecord(ctx->ev[2], ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->h_st, ctx->st, sizeof(DevState), hipMemcpyDeviceToHost,
                           ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    const DevState& s = *ctx->h_st;

    float t_init = 0.f, t_all = 0.f;
    HIP_TRY(hipEventElapsedTime(&t_init, ctx->ev[0], ctx->ev[1]));
    HIP_TRY(hipEventElapsedTime(&t_all, ctx->ev[0], ctx->ev[2]));
    ctx->timing.total_ms = t_all;
    ctx->timing.init_ms = t_init;
    ctx->timing.loop_ms = t_all - t_init;
    ctx->timing.iters = s.k;
    ctx->timing.launches = b->iters;

    if (res) {
        res->iters = s.k;
        res->converged = 0;
        res->delta = s.delta;
        res->lambda = s.lambda;
    }
    if (s.status != SFSEG_OK) return state_error(s.status, s.k);
    ctx->cur = b->iters & 1;
    ctx->have_iterate = true;
    return SFSEG_OK;
}

}  // extern "C"

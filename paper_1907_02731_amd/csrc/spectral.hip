// sfseg_spectral_grad: the training loss of the learned warm start on the
// error that survives k power-iteration steps, and its gradient.
//
// The network's estimate x^ replaces the start vector of Algorithm 1, so what
// matters is how much of its error the next k steps (Eq. (4) with the
// normalisation of Eq. (8)) leave.  With v = M^k x^ (M of Eq. (2)) the loss
// is L = 1 - cos(v, x*), scale-free in v, and since M is symmetric
//
//     dL/dx^ = M^k dL/dv,   dL/dv = -(x* / (|v| |x*|) - cos v / |v|^2).
//
// The k products run through the context's step kernel (sfseg_apply's path);
// each product's result is divided by its norm n_i (float64 sums), so the
// vectors stay near unit length, y_k = v / (n_1 ... n_k) = v / |v|, and the
// same divisions on the way back give dL/dv's share: g <- M g / n_i for
// i = k .. 1.  The loss's three sums are float64 and added on the host in a
// fixed order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "host_internal.h"

using sfseg_host::fail;

namespace {

constexpr int kBlocks = 512;

// Block b's share (grid-stride, fixed grid) of sum(x^2) in float64.
__global__ __launch_bounds__(256) void sumsq_part(const float* __restrict__ x, int64_t n,
                                                  double* __restrict__ part) {
    __shared__ double sm[256];
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = x[i];
        a = fma(v, v, a);
    }
    sm[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// One block: out = sqrt(sum of the nb block shares), in a fixed order.
__global__ __launch_bounds__(256) void norm_finish(const double* __restrict__ part, int nb,
                                                   double* __restrict__ out) {
    __shared__ double sm[256];
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) a += part[b];
    sm[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sqrt(sm[0]);
}

// out = in / *norm (in and out may be the same array).
__global__ __launch_bounds__(256) void scale_div(const float* in, float* out, int64_t n,
                                                 const double* __restrict__ norm) {
    const double inv = 1.0 / *norm;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = (float)((double)in[i] * inv);
}

// Block shares of sum(y t), sum(y^2), sum(t^2): part[3 b + 0..2].
__global__ __launch_bounds__(256) void loss_part(const float* __restrict__ y,
                                                 const float* __restrict__ t, int64_t n,
                                                 double* __restrict__ part) {
    __shared__ double sm[3][256];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double yv = y[i], tv = t[i];
        a = fma(yv, tv, a);
        b = fma(yv, yv, b);
        c = fma(tv, tv, c);
    }
    sm[0][threadIdx.x] = a;
    sm[1][threadIdx.x] = b;
    sm[2][threadIdx.x] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = sm[threadIdx.x][0];
}

// g = -(t c0 - y c1), with c0 = 1 / (|y| |t|), c1 = cos / |y|^2 (g may alias y).
__global__ __launch_bounds__(256) void cos_grad(const float* y, const float* __restrict__ t,
                                                int64_t n, double c0, double c1, float* g) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        g[i] = (float)-((double)t[i] * c0 - (double)y[i] * c1);
}

int grow_buffers(sfseg_ctx* ctx, int k) {
    const int64_t n = (int64_t)ctx->cfg.T * ctx->cfg.H * ctx->cfg.W;
    if (!ctx->spec_buf) HIP_TRY(hipMalloc((void**)&ctx->spec_buf, sizeof(float) * n));
    if (!ctx->spec_part) HIP_TRY(hipMalloc((void**)&ctx->spec_part, sizeof(double) * 3 * kBlocks));
    if (!ctx->h_spec)
        HIP_TRY(hipHostMalloc((void**)&ctx->h_spec, sizeof(double) * 3 * kBlocks, hipHostMallocDefault));
    if (k > ctx->spec_norms_cap) {
        if (ctx->spec_norms) HIP_TRY(hipFree(ctx->spec_norms));
        ctx->spec_norms = nullptr;
        HIP_TRY(hipMalloc((void**)&ctx->spec_norms, sizeof(double) * k));
        ctx->spec_norms_cap = k;
    }
    return SFSEG_OK;
}

}  // namespace

extern "C" {

int sfseg_spectral_grad(sfseg_ctx* ctx, const float* xhat, const float* target, int32_t k,
                        float* grad, double* loss) {
    if (!ctx || !xhat || !target || !grad)
        return fail(SFSEG_ERR_INVALID_ARG, "ctx, xhat, target or grad is NULL");
    if (ctx->batch) return fail(SFSEG_ERR_STATE, "batch context: sfseg_spectral_grad works on one clip");
    if (k < 0 || k > 4096) return fail(SFSEG_ERR_INVALID_ARG, "k must be 0..4096");
    if (grad == xhat || grad == target)
        return fail(SFSEG_ERR_INVALID_ARG, "grad may not alias xhat or target");
    HIP_TRY(hipSetDevice(ctx->device));
    if (int rc = grow_buffers(ctx, k > 0 ? k : 1)) return rc;
    hipStream_t s = ctx->stream;
    const int64_t n = (int64_t)ctx->cfg.T * ctx->cfg.H * ctx->cfg.W;
    const dim3 g(kBlocks), b(256);

    // forward: y_i = M y_{i-1} / n_i, y_0 = x^ (grad serves as the product's target)
    const float* y = xhat;
    for (int i = 0; i < k; ++i) {
        if (int rc = sfseg_host::apply_async(ctx, y, grad)) return rc;
        hipLaunchKernelGGL(sumsq_part, g, b, 0, s, (const float*)grad, n, ctx->spec_part);
        hipLaunchKernelGGL(norm_finish, dim3(1), b, 0, s, (const double*)ctx->spec_part, kBlocks,
                           ctx->spec_norms + i);
        hipLaunchKernelGGL(scale_div, g, b, 0, s, (const float*)grad, ctx->spec_buf, n,
                           (const double*)(ctx->spec_norms + i));
        HIP_TRY(hipGetLastError());
        y = ctx->spec_buf;
    }

    // loss and dL/dy_k
    hipLaunchKernelGGL(loss_part, g, b, 0, s, y, target, n, ctx->spec_part);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(ctx->h_spec, ctx->spec_part, sizeof(double) * 3 * kBlocks,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double dot = 0.0, yy = 0.0, tt = 0.0;
    for (int i = 0; i < kBlocks; ++i) {
        dot += ctx->h_spec[3 * i];
        yy += ctx->h_spec[3 * i + 1];
        tt += ctx->h_spec[3 * i + 2];
    }
    const double ny = sqrt(yy), nt = sqrt(tt);
    if (!(ny > 0.0) || !(nt > 0.0) || !isfinite(dot) || !isfinite(ny) || !isfinite(nt))
        return fail(ny > 0.0 && nt > 0.0 ? SFSEG_ERR_NONFINITE : SFSEG_ERR_ZERO_NORM,
                    "M^k xhat or the target has zero or non-finite norm");
    const double cosv = dot / (ny * nt);
    if (loss) *loss = 1.0 - cosv;
    float* cur = k > 0 ? ctx->spec_buf : grad;
    hipLaunchKernelGGL(cos_grad, g, b, 0, s, y, target, n, 1.0 / (ny * nt), cosv / (ny * ny), cur);
    HIP_TRY(hipGetLastError());

    // backward: g <- M g / n_i, i = k .. 1 (M symmetric)
    float* other = cur == grad ? ctx->spec_buf : grad;
    for (int i = k - 1; i >= 0; --i) {
        if (int rc = sfseg_host::apply_async(ctx, cur, other)) return rc;
        hipLaunchKernelGGL(scale_div, g, b, 0, s, (const float*)other, other, n,
                           (const double*)(ctx->spec_norms + i));
        HIP_TRY(hipGetLastError());
        float* tmp = cur;
        cur = other;
        other = tmp;
    }
    if (cur != grad)
        HIP_TRY(hipMemcpyAsync(grad, cur, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SFSEG_OK;
}

}  // extern "C"

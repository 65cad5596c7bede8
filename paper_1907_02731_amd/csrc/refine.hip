// sfseg_refine_frames: frame-wise Rayleigh-Ritz refinement of the current
// iterate, a start vector for the warm-started form (not part of the paper).
//
// Eq. (3) makes the principal eigenvector the maximiser of the Rayleigh
// quotient.  Over the subspace spanned by the frames of the iterate x
// (q_t = x on frame t, zero elsewhere) the maximiser is sum_t a_t q_t, with
// a the top eigenvector of the pencil B a = mu G a, B[i][j] = q_i^T M q_j and
// G = diag(||q_t||^2) (the q_t have disjoint supports).  M couples frames at
// most r_t apart, so B is a band matrix of half-width r_t.
//
// B is formed with 2 r_t + 1 products of M instead of one per frame: the
// frames of residue r modulo m = 2 r_t + 1 are at least m apart, so in
// y_r = M (x restricted to those frames) the frame i holds M q_j for the one
// frame j = i + d, |d| <= r_t, of that residue, and B[i][j] = <x_i, (y_r)_i>.
// Products run through the context's step kernel (one application, c = 1)
// on the stored iterate; the frame inner products are float64 block sums
// added on the host in a fixed order.  The small band problem is solved on
// the host in float64: the largest eigenvalue by bisection on inertia counts
// (Sylvester's law: the negative pivots of the LDL^T factors of A - sigma I,
// banded, no pivoting), its eigenvector by inverse iteration with a shift
// just above it, where A - sigma I is definite.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <vector>

#include "host_internal.h"

using sfseg::DevState;
using sfseg::StepParams;
using sfseg_host::fail;

namespace {

constexpr int kFrameBlocks = 16;  // blocks per frame in the frame sums

template <typename TS>
__device__ __forceinline__ float widen(TS v) {
    return (float)v;
}

// dst = src on the frames t with t % m == r, zeros on the others (padded
// volumes of `frame` elements per frame).  Block b works on frame
// b / kFrameBlocks.
template <typename TS>
__global__ __launch_bounds__(256) void mask_frames(const TS* __restrict__ src, TS* __restrict__ dst,
                                                   int64_t frame, int m, int r) {
    const int t = blockIdx.x / kFrameBlocks, sub = blockIdx.x % kFrameBlocks;
    const bool keep = t % m == r;
    const int64_t base = (int64_t)t * frame;
    for (int64_t i = (int64_t)sub * 256 + threadIdx.x; i < frame; i += (int64_t)kFrameBlocks * 256)
        dst[base + i] = keep ? src[base + i] : (TS)0.f;
}

// part[t * kFrameBlocks + b] = block b's share of sum_i a[t][i] * b[t][i]
// (float64; a product of two float32 values is exact in float64).
template <typename TS>
__global__ __launch_bounds__(256) void frame_dot_part(const TS* __restrict__ a,
                                                      const TS* __restrict__ b, int64_t frame,
                                                      double* __restrict__ part) {
    __shared__ double sm[256];
    const int t = blockIdx.x / kFrameBlocks, sub = blockIdx.x % kFrameBlocks;
    const int64_t base = (int64_t)t * frame;
    double acc = 0.0;
    for (int64_t i = (int64_t)sub * 256 + threadIdx.x; i < frame; i += (int64_t)kFrameBlocks * 256)
        acc = fma((double)widen(a[base + i]), (double)widen(b[base + i]), acc);
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// out (unpadded float32, T x H x W) = fac[t] * y (padded storage).
template <typename TS>
__global__ __launch_bounds__(256) void scaled_frames_out(const TS* __restrict__ y,
                                                         const double* __restrict__ fac,
                                                         float* __restrict__ out,
                                                         sfseg::Layout L) {
    const int64_t plane = (int64_t)L.H * L.W;
    const int64_t n = plane * L.T;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int t = (int)(i / plane);
        const int64_t rem = i - (int64_t)t * plane;
        const int yy = (int)(rem / L.W), xx = (int)(rem - (int64_t)yy * L.W);
        const float v = widen(y[(int64_t)t * L.frame + (int64_t)(yy + L.PT) * L.Wp + xx + L.PL]);
        out[i] = (float)(fac[t] * (double)v);
    }
}

template <typename TS>
hipError_t launch_mask(const void* src, void* dst, const sfseg::Layout& L, int m, int r,
                       hipStream_t s) {
    hipLaunchKernelGGL((mask_frames<TS>), dim3(kFrameBlocks * L.T), dim3(256), 0, s,
                       (const TS*)src, (TS*)dst, L.frame, m, r);
    return hipGetLastError();
}

template <typename TS>
hipError_t launch_dots(const void* a, const void* b, const sfseg::Layout& L, double* part,
                       hipStream_t s) {
    hipLaunchKernelGGL((frame_dot_part<TS>), dim3(kFrameBlocks * L.T), dim3(256), 0, s,
                       (const TS*)a, (const TS*)b, L.frame, part);
    return hipGetLastError();
}

template <typename TS>
hipError_t launch_out(const void* y, const double* fac, float* out, const sfseg::Layout& L,
                      int grid, hipStream_t s) {
    hipLaunchKernelGGL((scaled_frames_out<TS>), dim3(grid), dim3(256), 0, s, (const TS*)y, fac,
                       out, L);
    return hipGetLastError();
}

#define SFSEG_DISPATCH(dt, call)                                  \
    ((dt) == SFSEG_F32    ? call<float>                           \
     : (dt) == SFSEG_BF16 ? call<__bf16>                          \
                          : call<_Float16>)

// ---------------------------------------------------------------------------
// Host: the top eigenpair of a symmetric band matrix in float64
// ---------------------------------------------------------------------------
// A[i][i + d] = a[i * (p + 1) + d], d = 0 .. p (upper band; A symmetric).
struct Band {
    int n, p;
    std::vector<double> a;
    double at(int i, int j) const {
        if (i > j) {
            const int k = i;
            i = j;
            j = k;
        }
        return j - i <= p ? a[(size_t)i * (p + 1) + (j - i)] : 0.0;
    }
};

// LDL^T of A - sigma I without pivoting (L unit lower, band p): returns the
// number of negative pivots; l[i * (p + 1) + k] = L[i][i - k], piv[i] = D[i].
// A zero pivot is replaced by a tiny negative one.
int ldl_band(const Band& A, double sigma, double tiny, std::vector<double>& l,
             std::vector<double>& piv) {
    const int n = A.n, p = A.p;
    l.assign((size_t)n * (p + 1), 0.0);
    piv.assign(n, 0.0);
    int neg = 0;
    auto L = [&](int i, int j) -> double& { return l[(size_t)i * (p + 1) + (i - j)]; };
    for (int i = 0; i < n; ++i) {
        const int j0 = i - p > 0 ? i - p : 0;
        for (int j = j0; j < i; ++j) {
            double s = A.at(i, j);
            for (int k = (j - p > j0 ? j - p : j0); k < j; ++k) s -= L(i, k) * L(j, k) * piv[k];
            L(i, j) = s / piv[j];
        }
        double d = A.at(i, i) - sigma;
        for (int k = j0; k < i; ++k) d -= L(i, k) * L(i, k) * piv[k];
        if (d == 0.0) d = -tiny;
        piv[i] = d;
        if (d < 0.0) ++neg;
    }
    return neg;
}

// Solve (L D L^T) v = b in place with the factors of ldl_band.
void ldl_solve(int n, int p, const std::vector<double>& l, const std::vector<double>& piv,
               std::vector<double>& v) {
    auto L = [&](int i, int j) { return l[(size_t)i * (p + 1) + (i - j)]; };
    for (int i = 0; i < n; ++i)
        for (int j = (i - p > 0 ? i - p : 0); j < i; ++j) v[i] -= L(i, j) * v[j];
    for (int i = 0; i < n; ++i) v[i] /= piv[i];
    for (int i = n - 1; i >= 0; --i)
        for (int j = i + 1; j <= i + p && j < n; ++j) v[i] -= L(j, i) * v[j];
}

// Largest eigenvalue and a unit eigenvector of the symmetric band matrix A.
void top_eigenpair(const Band& A, double* lam, std::vector<double>& v) {
    const int n = A.n;
    double lo = INFINITY, hi = -INFINITY, scale = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = 0.0;
        for (int j = i - A.p; j <= i + A.p; ++j)
            if (j >= 0 && j < n && j != i) r += fabs(A.at(i, j));
        lo = fmin(lo, A.at(i, i) - r);
        hi = fmax(hi, A.at(i, i) + r);
        scale = fmax(scale, fabs(A.at(i, i)) + r);
    }
    const double tiny = 1e-300 + 1e-30 * scale;
    std::vector<double> l, piv;
    // every eigenvalue lies in [lo, hi]; keep count(A < hi) = n, count(A < lo) < n
    lo -= 1e-12 * scale + tiny;
    hi += 1e-12 * scale + tiny;
    for (int it = 0; it < 200 && hi - lo > 4e-16 * scale; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (ldl_band(A, mid, tiny, l, piv) == n)
            hi = mid;
        else
            lo = mid;
    }
    *lam = 0.5 * (lo + hi);
    // inverse iteration with a shift above the largest eigenvalue: A - sigma I
    // is negative definite, its factors are stable
    const double sigma = hi + 1e-10 * scale + tiny;
    ldl_band(A, sigma, tiny, l, piv);
    v.assign(n, 1.0);
    for (int it = 0; it < 6; ++it) {
        ldl_solve(n, A.p, l, piv, v);
        double nn = 0.0;
        for (double e : v) nn += e * e;
        nn = sqrt(nn);
        for (double& e : v) e /= nn;
    }
}

}  // namespace

extern "C" {

int sfseg_refine_frames(sfseg_ctx* ctx, float* x_out, double* ritz_value) {
    if (!ctx || !x_out) return fail(SFSEG_ERR_INVALID_ARG, "ctx or x_out is NULL");
    if (ctx->batch) return fail(SFSEG_ERR_STATE, "batch context: the refinement works on one clip");
    if (!ctx->have_iterate)
        return fail(SFSEG_ERR_STATE, "no iterate: call sfseg_power_iterate first");
    HIP_TRY(hipSetDevice(ctx->device));
    const sfseg::Layout& L = ctx->L;
    const int dt = ctx->cfg.storage;
    const int T = L.T, rt = ctx->cfg.r_t, m = 2 * rt + 1;
    const size_t bytes = (size_t)L.total * sfseg_host::dtype_size(dt);
    const size_t nsum = (size_t)(m + 1) * T * kFrameBlocks;  // m band products + the norms
    if (!ctx->apply_in) {
        HIP_TRY(hipMalloc(&ctx->apply_in, bytes));
        HIP_TRY(hipMemsetAsync(ctx->apply_in, 0, bytes, ctx->stream));
    }
    if (!ctx->apply_out) {
        HIP_TRY(hipMalloc(&ctx->apply_out, bytes));
        HIP_TRY(hipMemsetAsync(ctx->apply_out, 0, bytes, ctx->stream));
    }
    if (ctx->ritz_cap < nsum) {
        if (ctx->ritz_part) HIP_TRY(hipFree(ctx->ritz_part));
        if (ctx->h_ritz) HIP_TRY(hipHostFree(ctx->h_ritz));
        ctx->ritz_part = nullptr;
        ctx->h_ritz = nullptr;
        ctx->ritz_cap = 0;
        HIP_TRY(hipMalloc((void**)&ctx->ritz_part, nsum * sizeof(double)));
        HIP_TRY(hipHostMalloc((void**)&ctx->h_ritz, nsum * sizeof(double), hipHostMallocDefault));
        ctx->ritz_cap = nsum;
    }
    if (ctx->ritz_fac_cap < (size_t)T) {
        if (ctx->ritz_fac) HIP_TRY(hipFree(ctx->ritz_fac));
        ctx->ritz_fac = nullptr;
        ctx->ritz_fac_cap = 0;
        HIP_TRY(hipMalloc((void**)&ctx->ritz_fac, (size_t)T * sizeof(double)));
        ctx->ritz_fac_cap = T;
    }
    const void* Y = ctx->buf[ctx->cur];

    // One application of M per residue class of frames (c = 1, nothing pending).
    DevState h{};
    h.s = 1.0;
    h.c = 1.0f;
    h.gain = 1.0;
    h.tol = -1.0;
    h.max_iters = 1;
    ctx->h_st[0] = h;
    HIP_TRY(hipMemcpyAsync(ctx->st_apply, ctx->h_st, sizeof(DevState), hipMemcpyHostToDevice,
                           ctx->stream));
    HIP_TRY(SFSEG_DISPATCH(dt, launch_dots)(Y, Y, L, ctx->ritz_part + (size_t)m * T * kFrameBlocks,
                                            ctx->stream));
    for (int r = 0; r < m; ++r) {
        HIP_TRY(SFSEG_DISPATCH(dt, launch_mask)(Y, ctx->apply_in, L, m, r, ctx->stream));
        StepParams p = ctx->params[0];
        p.x = ctx->apply_in;
        p.y = ctx->apply_out;
        p.st_in = ctx->st_apply;
        p.st_out = ctx->st_apply + 1;
        p.half = 1;
        HIP_TRY(sfseg::launch_step(dt, sfseg::kernel_shape(ctx->shape, ctx->nf), ctx->cfg.r_s, rt,
                                   p, ctx->step_grid, ctx->stream));
        HIP_TRY(SFSEG_DISPATCH(dt, launch_dots)(Y, ctx->apply_out, L,
                                                ctx->ritz_part + (size_t)r * T * kFrameBlocks,
                                                ctx->stream));
    }
    HIP_TRY(hipMemcpyAsync(ctx->h_ritz, ctx->ritz_part, nsum * sizeof(double),
                           hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));

    // frame sums in a fixed order
    auto fsum = [&](int set, int t) {
        double s = 0.0;
        for (int b = 0; b < kFrameBlocks; ++b) s += ctx->h_ritz[((size_t)set * T + t) * kFrameBlocks + b];
        return s;
    };
    std::vector<double> G(T);
    std::vector<int> keep;
    for (int t = 0; t < T; ++t) {
        G[t] = fsum(m, t);
        if (!isfinite(G[t])) return fail(SFSEG_ERR_NONFINITE, "non-finite iterate");
        if (G[t] > 0.0) keep.push_back(t);
    }
    if (keep.empty()) return fail(SFSEG_ERR_ZERO_NORM, "the iterate is zero on every frame");
    // B[i][j] = <x_i, (M x_{j mod m})_i> for |i - j| <= r_t; symmetrised and
    // scaled by G^-1/2 on both sides, over the frames with G > 0
    const int n = (int)keep.size();
    Band A{n, rt, std::vector<double>((size_t)n * (rt + 1), 0.0)};
    auto Bij = [&](int i, int j) { return fsum(((j % m) + m) % m, i); };
    for (int a = 0; a < n; ++a)
        for (int b = a; b < n && keep[b] - keep[a] <= rt; ++b) {
            const int i = keep[a], j = keep[b];
            const double v = 0.5 * (Bij(i, j) + Bij(j, i)) / sqrt(G[i] * G[j]);
            if (!isfinite(v)) return fail(SFSEG_ERR_NONFINITE, "non-finite product");
            A.a[(size_t)a * (rt + 1) + (b - a)] = v;
        }
    double mu = 0.0;
    std::vector<double> z;
    top_eigenpair(A, &mu, z);
    // a_t = z / sqrt(G_t), signed for a positive overlap with x (sum a_t G_t > 0);
    // sum a_t^2 G_t = 1, so the output has unit norm
    double overlap = 0.0;
    for (int a = 0; a < n; ++a) overlap += z[a] * sqrt(G[keep[a]]);
    std::vector<double> fac(T, 0.0);
    for (int a = 0; a < n; ++a) fac[keep[a]] = (overlap < 0.0 ? -z[a] : z[a]) / sqrt(G[keep[a]]);
    // the host buffer is free again (the stream has passed its copy)
    for (int t = 0; t < T; ++t) ctx->h_ritz[t] = fac[t];
    HIP_TRY(hipMemcpyAsync(ctx->ritz_fac, ctx->h_ritz, (size_t)T * sizeof(double),
                           hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(SFSEG_DISPATCH(dt, launch_out)(Y, ctx->ritz_fac, x_out, L, ctx->ew_grid, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (ritz_value) *ritz_value = mu;
    return SFSEG_OK;
}

}  // extern "C"

// gfx950 kernels of the SFSeg power iteration.
//
// One power-iteration step (Eq. (4) then Eq. (8)) is one launch of the fused
// step kernel.  The adjacency of Eq. (2) is applied through its three-filter
// form (Eq. (7), multiplied out by alpha so that alpha = 0 needs no special
// case):
//
//     u = w * x,   A = G * u,   B = G * (F^2 u),   C = G * (F u)
//     y = w * [ A - alpha * (F * (F * A - 2 C) + B) ]
//
// with G the separable box-truncated Gaussian of Eq. (1) (Sec. 4.2: a 3D
// filter is three 1D filters) and zero padding at the volume faces, which
// is what makes the filtering equal the symmetric matrix M.
//
// Work layout of the step kernel: the volume is cut into 64 x 16 pixel
// tiles; the (tile, frame) units are laid out tile-major and split into equal
// contiguous ranges, one per block, so every block does the same work.  A
// block streams along time through its range: for each input frame it loads
// the tile plus an r_s halo, forms the three fields, filters them along y
// (LDS -> LDS) and x (LDS -> registers), and pushes the result into a
// register ring of 2 r_t + 1 frames; once the ring holds frames
// t - r_t .. t + r_t it filters along t, combines, stores frame t and
// accumulates sum(y^2) and sum(y * Y_k) in float64 on the stored values.  The
// block's partial sums go to memory; the last block to finish reduces all
// partials in a fixed order and advances the iteration state (norm, Rayleigh
// quotient, change, convergence flag), so results are bit-reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <utility>

#include "sfseg_internal.h"

namespace sfseg {
namespace detail {


// ---------------------------------------------------------------------------
// Storage precisions: float32, bfloat16, float16 (values are widened to
// float32 on load; float32 results are rounded to nearest-even on store).
// ---------------------------------------------------------------------------
template <typename TS>
struct Stor;
template <>
struct Stor<float> {
    static __device__ __forceinline__ float ld(const float* p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ float rnd(float v) { return v; }
    static __device__ __forceinline__ void st(float* p, int64_t i, float v) { p[i] = v; }
};
template <>
struct Stor<__bf16> {
    static __device__ __forceinline__ float ld(const __bf16* p, int64_t i) { return (float)p[i]; }
    static __device__ __forceinline__ float rnd(float v) { return (float)(__bf16)v; }
    static __device__ __forceinline__ void st(__bf16* p, int64_t i, float v) { p[i] = (__bf16)v; }
};
template <>
struct Stor<_Float16> {
    static __device__ __forceinline__ float ld(const _Float16* p, int64_t i) { return (float)p[i]; }
    static __device__ __forceinline__ float rnd(float v) { return (float)(_Float16)v; }
    static __device__ __forceinline__ void st(_Float16* p, int64_t i, float v) { p[i] = (_Float16)v; }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double agent_load(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void agent_store(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum nvals partial values (stride 2 starting at `first`) over nblocks blocks
// in a fixed order: thread i sums blocks i, i+NT, ...; then a fixed tree.
template <int NT>
__device__ double fixed_order_sum(const double* partials, int nblocks, int first, double* lds) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NT) acc += agent_load(partials + 2 * b + first);
    lds[threadIdx.x] = acc;
    __syncthreads();
#pragma unroll
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
        __syncthreads();
    }
    double r = lds[0];
    __syncthreads();
    return r;
}

// Block-wide sum of two doubles into partials[2*slot], partials[2*slot+1];
// returns true in every thread of the last block of the launch to arrive.
template <int NT>
__device__ bool block_partials_and_ticket(double a, double b, double* partials, int slot,
                                          uint32_t* ticket, uint32_t nblocks) {
    __shared__ double red[2][NT / 64];
    __shared__ int is_last;
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wid] = a;
        red[1][wid] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) {
            sa += red[0][i];
            sb += red[1][i];
        }
        agent_store(partials + 2 * slot, sa);
        agent_store(partials + 2 * slot + 1, sb);
        __threadfence();
        const uint32_t t = atomicAdd(ticket, 1u);
        is_last = (t == nblocks - 1);
    }
    __syncthreads();
    const bool last = is_last != 0;
    if (last) __threadfence();
    return last;
}

// Advance the iteration state after a step; run by thread 0 of the last block.
//   syy = sum(y_i^2), syx = sum(y_i * Y_k,i) over the stored values, where
//   y = c * M Y_k and x_k = s * Y_k.  Then
//   M x_k = (s / c) y            =>  lambda = x_k^T M x_k = s^2 syx / c
//   x_{k+1} = y / ||y||          =>  x_{k+1} . x_k = s syx / ||y||
//   delta = ||x_{k+1} - x_k|| = sqrt(2 - 2 x_{k+1} . x_k)   (both unit vectors)
__device__ inline void advance_state(DevState* st, double syy, double syx) {
    const double n = sqrt(syy);
    const double s = st->s;
    const double c = (double)st->c;
    st->k += 1;
    if (!isfinite(n) || !isfinite(syx)) {
        st->status = SFSEG_ERR_NONFINITE;
        st->done = 1;
        return;
    }
    if (!(n > 0.0)) {
        st->status = SFSEG_ERR_ZERO_NORM;
        st->done = 1;
        return;
    }
    st->lambda = s * s * syx / c;
    const double cosv = s * syx / n;
    st->delta = sqrt(fmax(0.0, 2.0 - 2.0 * cosv));
    st->s = 1.0 / n;
    st->c = (float)(st->s * st->gain);
    if (st->delta < st->tol) {
        st->converged = 1;
        st->done = 1;
    }
    if (st->k >= st->max_iters) st->done = 1;
}

// ---------------------------------------------------------------------------
// Fused step kernel
// ---------------------------------------------------------------------------
constexpr int NT = STEP_THREADS;
constexpr int TX = TILE_X, TY = TILE_Y;
constexpr int PX = 4;              // outputs per thread along x
constexpr int NSEG = TX / PX;      // 16 thread columns
constexpr int PY = 4;              // y-pass outputs per work item
static_assert(NSEG * TY == NT, "one output strip per thread");

template <typename TS, int RS, int RT>
__global__ __launch_bounds__(NT) void step_kernel(StepParams p) {
    constexpr int IW = TX + 2 * RS;  // input region (tile + halo) width
    constexpr int IH = TY + 2 * RS;
    constexpr int NIN = IW * IH;
    constexpr int NLD = (NIN + NT - 1) / NT;
    constexpr int MP = IW | 1;        // odd pitch of the y-filtered rows
    constexpr int NYI = IW * (TY / PY);
    constexpr int NYR = (NYI + NT - 1) / NT;
    constexpr int NR = 2 * RT + 1;    // frames in the time ring
    constexpr int XW = PX + 2 * RS;   // x-pass register window
    constexpr int YW = PY + 2 * RS;   // y-pass register window

    __shared__ float in3[3][NIN];     // fields u, F u, F^2 u of the input frame
    __shared__ float mid3[3][TY * MP];  // y-filtered fields
    __shared__ double fin[NT];

    DevState* st = p.st;
    if (st->done) return;

    const float c = st->c;
    const float alpha = p.alpha;
    float gs[RS + 1];
#pragma unroll
    for (int d = 0; d <= RS; ++d) gs[d] = p.gs[d];
    float gt[NR];
#pragma unroll
    for (int m = 0; m < NR; ++m) gt[m] = p.gt[m < RT ? RT - m : m - RT] * c;

    const TS* __restrict__ X = (const TS*)p.x;
    const TS* __restrict__ Wt = (const TS*)p.w;
    const TS* __restrict__ Fv = (const TS*)p.f;
    TS* __restrict__ Y = (TS*)p.y;
    const int T = p.T, H = p.H, W = p.W;
    const int64_t HW = (int64_t)H * W;

    const int tid = threadIdx.x;
    const int orow = tid / NSEG;          // output row inside the tile
    const int ocol = (tid % NSEG) * PX;   // first output column inside the tile

    // Blocks are dealt to the XCDs round-robin; give each XCD a contiguous
    // run of ranges so that neighbouring tiles share its L2.
    const int G = gridDim.x;
    const int lb = (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;
    const int64_t u0 = (int64_t)lb * p.n_units / G;
    const int64_t u1 = (int64_t)(lb + 1) * p.n_units / G;

    double syy = 0.0, syx = 0.0;

    for (int64_t u = u0; u < u1;) {
        const int tile = (int)(u / T);
        const int ta = (int)(u % T);
        const int tb = (int)((int64_t)ta + (u1 - u) < T ? (int64_t)ta + (u1 - u) : T);
        u += tb - ta;
        const int tx0 = (tile % p.tiles_x) * TX;
        const int ty0 = (tile / p.tiles_x) * TY;

        // In-frame offsets of this thread's input-region elements (-1: outside).
        int goff[NLD];
#pragma unroll
        for (int m = 0; m < NLD; ++m) {
            const int e = tid + m * NT;
            const int r = e / IW, cc = e - (e / IW) * IW;
            const int gy = ty0 - RS + r, gx = tx0 - RS + cc;
            goff[m] = (e < NIN && gy >= 0 && gy < H && gx >= 0 && gx < W) ? gy * W + gx : -1;
        }
        const int gyo = ty0 + orow;
        const int gxo = tx0 + ocol;
        const bool orow_ok = gyo < H;

        float pX[NLD], pW[NLD], pF[NLD];  // prefetched input region of the next frame
        float cX[PX], cW[PX], cF[PX];     // prefetched own outputs' x, w, F
        auto load_frame = [&](int t) {
            const bool tin = (t >= 0 && t < T);
            const int64_t base = (int64_t)t * HW;
#pragma unroll
            for (int m = 0; m < NLD; ++m) {
                const bool ok = tin && goff[m] >= 0;
                const int64_t i = base + (ok ? goff[m] : 0);
                pX[m] = ok ? Stor<TS>::ld(X, i) : 0.f;
                pW[m] = ok ? Stor<TS>::ld(Wt, i) : 0.f;
                pF[m] = ok ? Stor<TS>::ld(Fv, i) : 0.f;
            }
#pragma unroll
            for (int i = 0; i < PX; ++i) {
                const bool ok = tin && orow_ok && (gxo + i) < W;
                const int64_t j = base + (ok ? (int64_t)gyo * W + gxo + i : 0);
                cX[i] = ok ? Stor<TS>::ld(X, j) : 0.f;
                cW[i] = ok ? Stor<TS>::ld(Wt, j) : 0.f;
                cF[i] = ok ? Stor<TS>::ld(Fv, j) : 0.f;
            }
        };

        float ring[NR][3][PX];   // x/y-filtered fields of the last NR frames
        float cring[NR][3][PX];  // x, w, F of this thread's outputs, same frames
#pragma unroll
        for (int j = 0; j < NR; ++j)
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int i = 0; i < PX; ++i) ring[j][f][i] = cring[j][f][i] = 0.f;

        const int n_in = (tb - ta) + 2 * RT;  // input frames ta-RT .. tb+RT-1
        load_frame(ta - RT);

        for (int s0 = 0; s0 < n_in; s0 += NR) {
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const int s = s0 + j;
                if (s < n_in) {
                    const int t_in = ta - RT + s;
                    __syncthreads();  // previous frame's readers of in3 / mid3 are done
                    // (1) fields of frame t_in into LDS
#pragma unroll
                    for (int m = 0; m < NLD; ++m) {
                        const int e = tid + m * NT;
                        if (e < NIN) {
                            const float uu = pW[m] * pX[m];
                            const float vv = pF[m] * uu;
                            in3[0][e] = uu;
                            in3[1][e] = vv;
                            in3[2][e] = pF[m] * vv;
                        }
                    }
#pragma unroll
                    for (int i = 0; i < PX; ++i) {
                        cring[j][0][i] = cX[i];
                        cring[j][1][i] = cW[i];
                        cring[j][2][i] = cF[i];
                    }
                    // (2) prefetch the next frame while this one is filtered
                    if (s + 1 < n_in) load_frame(t_in + 1);
                    __syncthreads();
                    // (3) filter along y: in3 -> mid3
#pragma unroll
                    for (int m = 0; m < NYR; ++m) {
                        const int it = tid + m * NT;
                        if (it < NYI) {
                            const int col = it % IW;
                            const int r0 = (it / IW) * PY;
#pragma unroll
                            for (int f = 0; f < 3; ++f) {
                                float win[YW];
#pragma unroll
                                for (int k = 0; k < YW; ++k) win[k] = in3[f][(r0 + k) * IW + col];
#pragma unroll
                                for (int i = 0; i < PY; ++i) {
                                    float a = gs[0] * win[i + RS];
#pragma unroll
                                    for (int d = 1; d <= RS; ++d)
                                        a = fmaf(gs[d], win[i + RS - d] + win[i + RS + d], a);
                                    mid3[f][(r0 + i) * MP + col] = a;
                                }
                            }
                        }
                    }
                    __syncthreads();
                    // (4) filter along x: mid3 -> ring slot j
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        float win[XW];
#pragma unroll
                        for (int k = 0; k < XW; ++k) win[k] = mid3[f][orow * MP + ocol + k];
#pragma unroll
                        for (int i = 0; i < PX; ++i) {
                            float a = gs[0] * win[i + RS];
#pragma unroll
                            for (int d = 1; d <= RS; ++d)
                                a = fmaf(gs[d], win[i + RS - d] + win[i + RS + d], a);
                            ring[j][f][i] = a;
                        }
                    }
                    // (5) once frames t-RT..t+RT are in the ring: filter along t,
                    //     combine (Eq. (7)), store frame t = t_in - RT, reduce.
                    if (s >= 2 * RT) {
                        const int t_out = t_in - RT;
                        const int jc = (j + NR - RT) % NR;  // ring slot of frame t_out (constant once unrolled)
                        const int64_t obase = (int64_t)t_out * HW + (int64_t)gyo * W + gxo;
#pragma unroll
                        for (int i = 0; i < PX; ++i) {
                            float A = 0.f, B = 0.f, C = 0.f;
#pragma unroll
                            for (int m = 0; m < NR; ++m) {
                                const int slot = (j + 1 + m) % NR;
                                A = fmaf(gt[m], ring[slot][0][i], A);  // G * u
                                C = fmaf(gt[m], ring[slot][1][i], C);  // G * (F u)
                                B = fmaf(gt[m], ring[slot][2][i], B);  // G * (F^2 u)
                            }
                            const float xc = cring[jc][0][i];
                            const float wc = cring[jc][1][i];
                            const float fc = cring[jc][2][i];
                            const float E = fmaf(-alpha, fmaf(fc, fmaf(fc, A, -2.f * C), B), A);
                            const float yq = Stor<TS>::rnd(wc * E);
                            if (orow_ok && gxo + i < W) {
                                Stor<TS>::st(Y, obase + i, yq);
                                syy = fma((double)yq, (double)yq, syy);
                                syx = fma((double)yq, (double)xc, syx);
                            }
                        }
                    }
                }
            }
        }
    }

    if (block_partials_and_ticket<NT>(syy, syx, p.partials, lb, &st->ticket, (uint32_t)G)) {
        const double tyy = fixed_order_sum<NT>(p.partials, G, 0, fin);
        const double tyx = fixed_order_sum<NT>(p.partials, G, 1, fin);
        if (threadIdx.x == 0) {
            advance_state(st, tyy, tyx);
            __hip_atomic_store(&st->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}


// Launch / occupancy tables over (r_s, r_t) for one storage type.
template <typename TS, int RS, int RT>
hipError_t launch_step_t(const StepParams& p, int grid, hipStream_t s) {
    hipLaunchKernelGGL((step_kernel<TS, RS, RT>), dim3(grid), dim3(NT), 0, s, p);
    return hipGetLastError();
}
template <typename TS, int RS, int RT>
hipError_t occ_step_t(int* blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, step_kernel<TS, RS, RT>, NT, 0);
}

using LaunchFn = hipError_t (*)(const StepParams&, int, hipStream_t);
using OccFn = hipError_t (*)(int*);
constexpr int NCOMB = (SFSEG_MAX_RS + 1) * (SFSEG_MAX_RT + 1);

template <typename TS, int RS, int... RTs>
void fill_rt(LaunchFn* lt, OccFn* ot, std::integer_sequence<int, RTs...>) {
    ((lt[RS * (SFSEG_MAX_RT + 1) + RTs] = &launch_step_t<TS, RS, RTs>,
      ot[RS * (SFSEG_MAX_RT + 1) + RTs] = &occ_step_t<TS, RS, RTs>), ...);
}
template <typename TS, int... RSs>
void fill_rs(LaunchFn* lt, OccFn* ot, std::integer_sequence<int, RSs...>) {
    (fill_rt<TS, RSs>(lt, ot, std::make_integer_sequence<int, SFSEG_MAX_RT + 1>{}), ...);
}

template <typename TS>
struct StepTable {
    LaunchFn launch[NCOMB];
    OccFn occ[NCOMB];
    StepTable() { fill_rs<TS>(launch, occ, std::make_integer_sequence<int, SFSEG_MAX_RS + 1>{}); }
};

}  // namespace detail
}  // namespace sfseg

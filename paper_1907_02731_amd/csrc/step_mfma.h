// Fused power-iteration step with the spatial filtering on the matrix cores.
//
// The same step as step_kernel (Eq. (4) applied through the three-filter form
// of Eq. (7), then the float64 sums of Eq. (8)), for float32 storage and one
// pairwise feature channel, with the two spatial passes of the separable
// Gaussian done as small matrix products on v_mfma_f32_16x16x32_f16:
//
//   x pass  X[row][col] = sum_k U[row][k] Gx[k][col]   (k: 32 region columns)
//   y pass  Y[row][col] = sum_k Gy[row][k] X[k][col]   (k: 32 region rows)
//
// for each of the three fields U = u, F u, F^2 u (u = c w x, the step's
// scale c applied as the fields are formed, so their magnitude stays near 1).
// The band matrices Gx, Gy hold the taps of Eq. (1) (zero beyond the radius);
// the temporal pass and the combine stay in float32 on the vector ALUs.
//
// Precision.  A float32 operand v enters the matrix cores as two float16
// values, v = hi + lo + e with hi = fp16(v), lo = fp16(v - hi), |e| <= 2^-23 |v|
// (v - hi is exact in float32), and so do the taps (g = gh + gl up to
// 2^-22 |g|, a fixed perturbation of the operator well below the float32
// taps' own rounding for the nearest taps and about 6e-7 relative for the
// farthest ones).  Each product takes three matrix operations, lo x gh,
// hi x gl, hi x gh, accumulated in float32 smallest first; lo x gl (below
// 2^-22) is dropped.  The y-pass taps are scaled by 16 (exact) so that their
// low parts stay normal float16 numbers, and the temporal taps divide the 16
// back out.

// Range.  Only the matrix operands are float16: u and the x-pass results.
// In a power-iteration step |u| <= c ||Y|| = gain = sqrt(N) / sum(G) and the
// x-pass results stay below sum(G_x) gain = sqrt(N) / (sum(G_y) sum(G_t)),
// under the float16 maximum for every volume of fewer than 2^31 voxels.  A
// single application (c = 1) needs |w x| sum(G_x) below it.
//
// Work layout: one block owns a 64 x 16 tile over a run of frames, as in
// step_kernel (same work items, padded layout and partial sums), with four
// waves; wave jb owns tile columns 16 jb .. 16 jb + 15 for all 16 rows.  Its
// x pass reads the 32 region columns [16 jb - RSA, 16 jb + 32 - RSA) of the
// region rows 0..31 (two 16-row blocks; rows past the 16 + 2 r_s loaded ones
// are zero) straight from LDS in the matrix operand layout, and the x-pass
// results land in registers in exactly the layout the y pass takes as its
// second operand (the y pass's k index runs over region rows in the order
// 4q..4q+3, 16+4q..16+4q+3 of lane group q; the band matrix Gy is laid out in
// the same order), so nothing goes back through LDS between the passes.
//
// Operand layout of the 16x16x32 product (checked on the GPU): lane l holds
// A[i = l % 16][k = 8 (l / 16) + e] and B[k = 8 (l / 16) + e][j = l % 16] for
// e = 0..7; D[i][j] sits in lane j + 16 (i / 4), register i % 4.
#pragma once

#include "step_kernel.h"

namespace sfseg {
namespace detail {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// (a, b) -> packed float16 pairs hi, lo with a = hi.x + lo.x and b = hi.y +
// lo.y up to 2^-23 relative: hi rounds to nearest, v - hi is formed exactly
// by a mixed-precision FMA (the float16 half of hi widened exactly), and
// rounded again.
__device__ __forceinline__ void split_f16x2(float a, float b, uint32_t& hi, uint32_t& lo) {
    const f32x2_t v = {a, b};
    hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, half2_t));
    float ra, rb;
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(ra) : "v"(hi), "v"(a));
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
        : "=v"(rb)
        : "v"(hi), "v"(b));
    const f32x2_t r = {ra, rb};
    lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, half2_t));
}

// Eight float32 values -> two float16 operands (hi, lo).
__device__ __forceinline__ void split8(const float* v, half8_t& hi, half8_t& lo) {
    u32x4 h, l;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        uint32_t a, b;
        split_f16x2(v[2 * e], v[2 * e + 1], a, b);
        h[e] = a;
        l[e] = b;
    }
    hi = __builtin_bit_cast(half8_t, h);
    lo = __builtin_bit_cast(half8_t, l);
}

// A float32 constant as two float16 parts, g = h + l up to 2^-22 |g| (the
// taps of both spatial passes).
struct Tap2 {
    half8_t h, l;
};
__device__ __forceinline__ void split_taps(const float* v, Tap2& t) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const _Float16 h = (_Float16)v[e];
        t.h[e] = h;
        t.l[e] = (_Float16)(v[e] - (float)h);
    }
}

__device__ __forceinline__ f32x4_t mfma16(half8_t a, half8_t b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

constexpr float kTapScale = 16.f;  // y-pass taps; 1 / 16 in the temporal taps

template <int RS, int RT>
struct MGeom {
    static constexpr int NT = 256;                 // four waves
    static constexpr int RSA = round4(RS);         // region starts RSA columns left of the tile
    static constexpr int IH = TY + 2 * RS;         // region rows loaded (<= 32)
    static constexpr int ROWS = 32;                // region rows the x pass reads (rest zero)
    static constexpr int PITCH = 84;               // floats per LDS row: 80 read + 4 (banks)
    static constexpr int CPR = PITCH / 4;          // 16-byte chunks per row
    static constexpr int NCH = IH * CPR;           // chunks per region (one array)
    static constexpr int NDMA = (NCH + NT - 1) / NT;
    static constexpr int AREA = ROWS * PITCH;      // floats per array per buffer
    static constexpr int NR = 2 * RT + 1;
    static_assert(IH <= ROWS, "the y window of 32 rows covers the tile and its halo");
    static_assert(16 + 2 * RS <= 32 && RSA <= 16 - RS, "the x window covers 16 columns and halo");
};

template <int RS, int RT>
struct MfmaLds {
    float raw[2][3][MGeom<RS, RT>::AREA] __attribute__((aligned(16)));  // double-buffered region
};

// One work item (tile origin tx0, ty0; output frames [ta, tb)); see run_item.
template <int RS, int RT>
__device__ __forceinline__ void run_item_mfma(const float* __restrict__ X,
                                              const float* __restrict__ Wt,
                                              const float* __restrict__ Fv, float* __restrict__ Y,
                                              int T, int Wp, int PT, int PL, int64_t frame,
                                              int tx0, int ty0, int ta, int tb, float cscale,
                                              const Tap2& gx, const Tap2& gy, const float* gt,
                                              float alpha, MfmaLds<RS, RT>& lds, double& syy,
                                              double& syx) {
    using G = MGeom<RS, RT>;
    constexpr int NT = G::NT, RSA = G::RSA, CPR = G::CPR, NCH = G::NCH, NDMA = G::NDMA,
                  AREA = G::AREA, PITCH = G::PITCH, NR = G::NR;
    if (tb <= ta) return;
    const uint32_t frame_bytes = (uint32_t)(frame * 4);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int jb = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave: tile columns 16 jb ..
    const int li = lane & 15, q = lane >> 4;

    int doff[NDMA];
#pragma unroll
    for (int r = 0; r < NDMA; ++r) {
        const int cidx = r * NT + tid;
        const int row = cidx / CPR, cq = cidx - (cidx / CPR) * CPR;
        doff[r] = ((ty0 + row) * Wp + (tx0 + PL - RSA) + cq * 4) * 4;
    }
    auto load_region = [&](int t, int buf) {
        if (t < 0 || t >= T) return;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float* base = (a == 0 ? X : (a == 1 ? Wt : Fv)) + (int64_t)t * frame;
            const __amdgpu_buffer_rsrc_t rr = make_rsrc(base, frame_bytes);
#pragma unroll
            for (int r = 0; r < NDMA; ++r)
                if (r * NT + tid < NCH)
                    load_lds16(rr, &lds.raw[buf][a][(r * NT + jb * 64) * 4], doff[r]);
        }
    };

    // x-pass operand of lane (li, q): region row li (+ 16), columns 16 jb + 8 q ..
    const int xa_off = li * PITCH + 16 * jb + 8 * q;
    // own voxels: rows 4 q + r of the tile, column 16 jb + li
    const int own_off = (4 * q + RS) * PITCH + RSA + 16 * jb + li;
    int ooff[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) ooff[r] = ((ty0 + PT + 4 * q + r) * Wp + (tx0 + PL + 16 * jb + li)) * 4;

    float ring[NR][3][4];  // y/x-filtered fields (scaled by 16) of the last NR frames
    float own[NR][3][4];   // x, w, F of the own voxels, by input frame
#pragma unroll
    for (int m = 0; m < NR; ++m)
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) ring[m][f][r] = 0.f;
    float yv[4];
    int pending_t = -1;

    const int n_in = (tb - ta) + 2 * RT;
    const int n_steps = (n_in + NR - 1) / NR * NR;
    load_region(ta - RT, 0);

    for (int s0 = 0; s0 < n_steps; s0 += NR) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const int s = s0 + j;
            if (s >= n_in) break;  // uniform
            const int t_in = ta - RT + s;
            const int cur = s & 1;
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();  // raw[cur] holds frame t_in; raw[cur ^ 1] is free
            if (s + 1 < n_in) load_region(t_in + 1, cur ^ 1);
            if (pending_t >= 0) {
                const __amdgpu_buffer_rsrc_t ry = make_rsrc(Y + (int64_t)pending_t * frame, frame_bytes);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(yv[r]), ry, ooff[r], 0, 0);
                pending_t = -1;
            }
            const float* rx = lds.raw[cur][0];
            const float* rw = lds.raw[cur][1];
            const float* rf = lds.raw[cur][2];
            if (t_in >= ta && t_in < tb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    own[j][0][r] = rx[own_off + r * PITCH];
                    own[j][1][r] = rw[own_off + r * PITCH];
                    own[j][2][r] = rf[own_off + r * PITCH];
                }
            }
            if (t_in >= 0 && t_in < T) {
                // ---- x pass: two 16-row blocks of the region, three fields.
                // All six operands are formed and split first; the products
                // then go round-robin over the six independent accumulators,
                // smallest parts first. ----
                half8_t ah[2][3], al[2][3];
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    const int o = xa_off + rb * 16 * PITCH;
                    float fx[8], fw[8], ff[8];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const float4 a = *reinterpret_cast<const float4*>(rx + o + 4 * h);
                        const float4 b = *reinterpret_cast<const float4*>(rw + o + 4 * h);
                        const float4 c = *reinterpret_cast<const float4*>(rf + o + 4 * h);
                        fx[4 * h] = a.x; fx[4 * h + 1] = a.y; fx[4 * h + 2] = a.z; fx[4 * h + 3] = a.w;
                        fw[4 * h] = b.x; fw[4 * h + 1] = b.y; fw[4 * h + 2] = b.z; fw[4 * h + 3] = b.w;
                        ff[4 * h] = c.x; ff[4 * h + 1] = c.y; ff[4 * h + 2] = c.z; ff[4 * h + 3] = c.w;
                    }
                    float u[8], fu[8], f2u[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        u[e] = (cscale * fw[e]) * fx[e];
                        fu[e] = ff[e] * u[e];
                        f2u[e] = ff[e] * fu[e];
                    }
                    split8(u, ah[rb][0], al[rb][0]);
                    split8(fu, ah[rb][1], al[rb][1]);
                    split8(f2u, ah[rb][2], al[rb][2]);
                }
                const f32x4_t z4 = {0.f, 0.f, 0.f, 0.f};
                f32x4_t xacc[2][3];
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int f = 0; f < 3; ++f) xacc[rb][f] = mfma16(al[rb][f], gx.h, z4);
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int f = 0; f < 3; ++f) xacc[rb][f] = mfma16(ah[rb][f], gx.l, xacc[rb][f]);
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int f = 0; f < 3; ++f) xacc[rb][f] = mfma16(ah[rb][f], gx.h, xacc[rb][f]);
                // ---- y pass: the x-pass results are already the second operand ----
                half8_t bh[3], bl[3];
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const float v[8] = {xacc[0][f][0], xacc[0][f][1], xacc[0][f][2], xacc[0][f][3],
                                        xacc[1][f][0], xacc[1][f][1], xacc[1][f][2], xacc[1][f][3]};
                    split8(v, bh[f], bl[f]);
                }
                f32x4_t yacc[3];
#pragma unroll
                for (int f = 0; f < 3; ++f) yacc[f] = mfma16(gy.h, bl[f], z4);
#pragma unroll
                for (int f = 0; f < 3; ++f) yacc[f] = mfma16(gy.l, bh[f], yacc[f]);
#pragma unroll
                for (int f = 0; f < 3; ++f) yacc[f] = mfma16(gy.h, bh[f], yacc[f]);
#pragma unroll
                for (int f = 0; f < 3; ++f)
#pragma unroll
                    for (int r = 0; r < 4; ++r) ring[j][f][r] = yacc[f][r];
            } else {
#pragma unroll
                for (int f = 0; f < 3; ++f)
#pragma unroll
                    for (int r = 0; r < 4; ++r) ring[j][f][r] = 0.f;
            }
            // ---- t pass, combine (Eq. (7)), reduce: output frame t_in - r_t ----
            const int t_out = t_in - RT;
            if (t_out >= ta && t_out < tb) {
                const int jo = (j + NR - RT) % NR;  // own values of the output frame (constant)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float tf[3] = {0.f, 0.f, 0.f};
#pragma unroll
                    for (int m = 0; m < NR; ++m) {
                        const int slot = (j + 1 + m) % NR;
#pragma unroll
                        for (int f = 0; f < 3; ++f) tf[f] = fmaf(gt[m], ring[slot][f][r], tf[f]);
                    }
                    const float xo = own[jo][0][r], wo = own[jo][1][r], fo = own[jo][2][r];
                    const float qv = fmaf(fo, fmaf(fo, tf[0], -2.f * tf[1]), tf[2]);
                    const float E = fmaf(-alpha, qv, tf[0]);
                    const float yq = wo * E;
                    yv[r] = yq;
                    syy = fma((double)yq, (double)yq, syy);
                    syx = fma((double)yq, (double)xo, syx);
                }
                pending_t = t_out;
            }
        }
    }
    if (pending_t >= 0) {
        const __amdgpu_buffer_rsrc_t ry = make_rsrc(Y + (int64_t)pending_t * frame, frame_bytes);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(yv[r]), ry, ooff[r], 0, 0);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
}

template <int RS, int RT>
__global__ __launch_bounds__(256, 2) void step_mfma_kernel(StepParams p) {
    using G = MGeom<RS, RT>;
    constexpr int NR = G::NR, RSA = G::RSA;
    __shared__ MfmaLds<RS, RT> lds;
    __shared__ double fold_red[2][4];

    const DevState s = state_of_input<256>(p.st_in, p.part_in, gridDim.x, fold_red);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevState o = s;
        o.pending = s.done ? 0 : 1;
        *p.st_out = o;
    }
    if (s.done) return;

    // Rows past the loaded region read as zeros (both buffers, every array).
    if constexpr (G::IH < G::ROWS) {
        constexpr int per = (G::ROWS - G::IH) * G::PITCH;
        for (int i = threadIdx.x; i < 6 * per; i += 256) {
            const int ba = i / per, k = i - ba * per;
            lds.raw[ba / 3][ba % 3][G::IH * G::PITCH + k] = 0.f;
        }
    }

    // Band matrices of the spatial taps in the operand layouts (y taps scaled by 16).
    const int lane = threadIdx.x & 63, li = lane & 15, q = lane >> 4;
    Tap2 gx, gy;
    {
        float vx[8], vy[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            // x pass, B[k][j]: region column 8 q + e against output column li + RSA
            const int dx = 8 * q + e - li - RSA;
            vx[e] = (dx >= -RS && dx <= RS) ? p.gs[dx < 0 ? -dx : dx] : 0.f;
            // y pass, A[i][k]: region row rho(q, e) against output row li + RS
            const int rho = e < 4 ? 4 * q + e : 16 + 4 * q + (e - 4);
            const int dy = rho - li - RS;
            vy[e] = (dy >= -RS && dy <= RS) ? kTapScale * p.gs[dy < 0 ? -dy : dy] : 0.f;
        }
        split_taps(vx, gx);
        split_taps(vy, gy);
    }
    float gt[NR];
#pragma unroll
    for (int m = 0; m < NR; ++m)
        gt[m] = p.gt[m < RT ? RT - m : m - RT] * (1.f / kTapScale);

    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int4 item = p.items[lb];
    double syy = 0.0, syx = 0.0;
    run_item_mfma<RS, RT>((const float*)p.x, (const float*)p.w, (const float*)p.f, (float*)p.y,
                          p.T, p.Wp, p.PT, p.PL, p.frame, item.x, item.y, item.z, item.w, s.c,
                          gx, gy, gt, p.alpha, lds, syy, syx);
    block_partials<256>(syy, syx, p.part_out, lb);
}

template <int RS, int RT>
hipError_t launch_mfma_t(const StepParams& p, int grid, hipStream_t s) {
    hipLaunchKernelGGL((step_mfma_kernel<RS, RT>), dim3(grid), dim3(256), 0, s, p);
    return hipGetLastError();
}
template <int RS, int RT>
hipError_t occ_mfma_t(int* blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, step_mfma_kernel<RS, RT>, 256, 0);
}

// Temporal radii up to MFMA_MAX_RT: the two register rings (filtered fields
// and own values, 2 r_t + 1 frames each) stay within the 256 registers that
// two waves per SIMD allow.
template <int RS, int... RTs>
void fill_mfma_rt(StepFns* t, std::integer_sequence<int, RTs...>) {
    ((t[RS * (SFSEG_MAX_RT + 1) + RTs] =
          StepFns{&launch_mfma_t<RS, RTs>, &occ_mfma_t<RS, RTs>, nullptr, nullptr}),
     ...);
}
template <int... RSs>
void fill_mfma_rs(StepFns* t, std::integer_sequence<int, RSs...>) {
    (fill_mfma_rt<RSs>(t, std::make_integer_sequence<int, MFMA_MAX_RT + 1>{}), ...);
}
struct MfmaTable {
    StepFns fns[NCOMB] = {};
    MfmaTable() { fill_mfma_rs(fns, std::make_integer_sequence<int, SFSEG_MAX_RS + 1>{}); }
};

}  // namespace detail
}  // namespace sfseg

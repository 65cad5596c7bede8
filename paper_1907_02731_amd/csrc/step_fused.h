// Two power-iteration steps per pass over HBM (temporal blocking).
//
// One launch of step2_kernel computes Y2 = c M (c M Y0) for its tile: it
// reads x = Y0, w and F once and writes only Y2; the intermediate iterate
// Y1 = c M Y0 lives in LDS.  M is applied as in step_kernel (the three-field
// form of Eq. (7) with the separable box-truncated Gaussian of Eq. (1), zero
// padding at the faces), in float32 with the same taps.
//
// Halos.  Step 2 on a TW x TH tile over output frames [ta, tb) needs Y1 on
// the tile plus an r_s halo over frames [ta - r_t, tb + r_t); step 1 there
// needs Y0 on the tile plus 2 r_s over frames [ta - 2 r_t, tb + 2 r_t).  The
// block recomputes the halo part of Y1 (it belongs to neighbouring tiles) --
// the arithmetic that fusing trades for the HBM pass it saves.  Reads of the
// wider halo can fall outside the padded frame; those positions are zero
// (the zero padding of the method) and are not loaded.
//
// Scale.  Both steps use the multiplier c of the launch's input state (the
// previous fold's s times the storage gain): the norm of Y1 is not known
// until every block has finished, and c = 1 / lambda near the fixed point,
// so Y2 keeps the magnitude of Y1.  The block leaves two pairs of float64
// partial sums, (sum Y1^2, sum Y1 Y0) and (sum Y2^2, sum Y2 Y1) over its own
// voxels, and the state is marked pending = 2: the next fold advances it by
// the first pair with c, sets c back to the value the launch used and
// advances it by the second (see state_of_input).  With `half` set the
// launch stops after step 1 and writes Y1 (an odd last step, or a single
// application).
//
// Layout in LDS, one frame at a time (float32; fits 160 KB for r_s <= 5,
// r_t <= 2 with a 32 x 8 tile): the three fields of the input frame over the
// step-1 input region, their y-filtered rows, a ring of 2 r_t + 1 frames of
// fully filtered fields over the step-1 output region, the own x, w, F of
// r_t + 1 frames there, and the same three stages for step 2 over the tile.
#pragma once

#include "step_kernel.h"

namespace sfseg {
namespace detail {

template <int RS, int RT>
struct F2Geom {
    static constexpr int TW = FUSED_TILE_X, TH = FUSED_TILE_Y;  // step-2 output tile
    static constexpr int W1 = TW + 2 * RS, H1 = TH + 2 * RS;    // step-1 outputs
    static constexpr int W0 = TW + 4 * RS, H0 = TH + 4 * RS;    // step-1 inputs
    static constexpr int NR = 2 * RT + 1;
    static constexpr int NO = RT + 1;
    static constexpr int NT = 256;
    static constexpr int XSEG = 6;  // x-pass outputs per task
};

template <int RS, int RT>
struct F2Lds {
    using G = F2Geom<RS, RT>;
    float fld[3][G::H0 * G::W0];          // u = w x, F u, F^2 u of the input frame
    float mid1[3][G::H1 * G::W0];         // step 1 filtered along y
    float ring1[G::NR][3][G::H1 * G::W1];  // step 1 filtered along y and x
    float own1[G::NO][3][G::H1 * G::W1];   // x, w, F over the step-1 output region
    float fld2[3][G::H1 * G::W1];          // w Y1, F w Y1, F^2 w Y1
    float mid2[3][G::TH * G::W1];          // step 2 filtered along y
    float ring2[G::NR][3][G::TH * G::TW];  // step 2 filtered along y and x
    float own2[G::NO][3][G::TH * G::TW];   // Y1, w, F over the tile
};

// Column filter along y: out[i] = sum_d g[|d|] in[(i + RS + d) * stride] for
// NOUT outputs from NOUT + 2 RS inputs, streaming the inputs once.
template <int RS, int NOUT>
__device__ __forceinline__ void yfilter_column(const float* in, int stride, const float* g,
                                               float* out, int ostride) {
    float acc[NOUT];
#pragma unroll
    for (int i = 0; i < NOUT; ++i) acc[i] = 0.f;
#pragma unroll
    for (int k = 0; k < NOUT + 2 * RS; ++k) {
        const float v = in[k * stride];
#pragma unroll
        for (int i = 0; i < NOUT; ++i) {
            const int d = k - i - RS;
            if (d >= -RS && d <= RS) acc[i] = fmaf(g[d < 0 ? -d : d], v, acc[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < NOUT; ++i) out[i * ostride] = acc[i];
}

// Row filter along x: N outputs from N + 2 RS consecutive inputs.
template <int RS, int N>
__device__ __forceinline__ void xfilter_row(const float* in, const float* g, float* out) {
    float win[N + 2 * RS];
#pragma unroll
    for (int k = 0; k < N + 2 * RS; ++k) win[k] = in[k];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        float a = g[0] * win[i + RS];
#pragma unroll
        for (int d = 1; d <= RS; ++d) a = fmaf(g[d], win[i + RS - d] + win[i + RS + d], a);
        out[i] = a;
    }
}

template <int RS, int RT>
__global__ __launch_bounds__(256, 1) void step2_kernel(StepParams p) {
    using G = F2Geom<RS, RT>;
    constexpr int TW = G::TW, TH = G::TH, W1 = G::W1, H1 = G::H1, W0 = G::W0, H0 = G::H0,
                  NR = G::NR, NO = G::NO, NT = G::NT, XSEG = G::XSEG;
    __shared__ F2Lds<RS, RT> lds;
    __shared__ double fold_red[2][4];

    const DevState s = state_of_input<NT>(p.st_in, p.part_in, gridDim.x, fold_red);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevState o = s;
        o.pending = s.done ? 0 : (p.half ? 1 : 2);
        *p.st_out = o;
    }
    if (s.done) return;

    float g[RS + 1];
#pragma unroll
    for (int d = 0; d <= RS; ++d) g[d] = p.gs[d];
    float gt[NR];
#pragma unroll
    for (int m = 0; m < NR; ++m) gt[m] = p.gt[m < RT ? RT - m : m - RT] * s.c;
    const float alpha = p.alpha;

    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int4 item = p.items[lb];
    const int tx0 = item.x, ty0 = item.y, ta = item.z, tb = item.w;
    const int T = p.T, Wp = p.Wp, Hp = (int)(p.frame / p.Wp);
    const uint32_t frame_bytes = (uint32_t)(p.frame * 4);
    const float* X = (const float*)p.x;
    const float* Wt = (const float*)p.w;
    const float* Fv = (const float*)p.f;
    float* Y = (float*)p.y;
    const int tid = threadIdx.x;
    double syy1 = 0.0, syx1 = 0.0, syy2 = 0.0, syx2 = 0.0;

    if (tb > ta) {
        // input frames ta - 2 r_t .. tb + 2 r_t - 1 (ta - r_t .. tb + r_t - 1 for one step)
        const int lead = p.half ? RT : 2 * RT;
        const int n_in = (tb - ta) + 2 * lead;
        // padded row / column of region position (0, 0) of the step-1 inputs
        const int row0 = ty0 + p.PT - 2 * RS, col0 = tx0 + p.PL - 2 * RS;
        for (int s_ = 0; s_ < n_in; ++s_) {
            const int t = ta - lead + s_;
            const bool tin = t >= 0 && t < T;
            const int slot1 = s_ % NR, oslot1 = s_ % NO;
            // ---- (A) the input frame: fields over the step-1 input region, own x, w, F ----
            if (tin) {
                const __amdgpu_buffer_rsrc_t rx = make_rsrc(X + (int64_t)t * p.frame, frame_bytes);
                const __amdgpu_buffer_rsrc_t rw = make_rsrc(Wt + (int64_t)t * p.frame, frame_bytes);
                const __amdgpu_buffer_rsrc_t rf = make_rsrc(Fv + (int64_t)t * p.frame, frame_bytes);
                for (int i = tid; i < H0 * W0; i += NT) {
                    const int r = i / W0, c = i - (i / W0) * W0;
                    const int pr = row0 + r, pc = col0 + c;
                    // outside the padded frame the volume is zero
                    float xv = 0.f, wv = 0.f, fv = 0.f;
                    if (pr >= 0 && pr < Hp && pc >= 0 && pc < Wp) {
                        const int off = (pr * Wp + pc) * 4;
                        xv = Stor<float>::bload(rx, off);
                        wv = Stor<float>::bload(rw, off);
                        fv = Stor<float>::bload(rf, off);
                    }
                    const float u = wv * xv;
                    lds.fld[0][i] = u;
                    lds.fld[1][i] = fv * u;
                    lds.fld[2][i] = fv * (fv * u);
                    const int r1 = r - RS, c1 = c - RS;
                    if (r1 >= 0 && r1 < H1 && c1 >= 0 && c1 < W1) {
                        const int q = r1 * W1 + c1;
                        lds.own1[oslot1][0][q] = xv;
                        lds.own1[oslot1][1][q] = wv;
                        lds.own1[oslot1][2][q] = fv;
                    }
                }
            }
            __syncthreads();
            // ---- (B) step 1, y pass: one column of one field per thread ----
            if (tin) {
                for (int task = tid; task < 3 * W0; task += NT) {
                    const int f = task / W0, c = task - (task / W0) * W0;
                    yfilter_column<RS, H1>(&lds.fld[f][c], W0, g, &lds.mid1[f][c], W0);
                }
            }
            __syncthreads();
            // ---- (C) step 1, x pass into ring slot slot1 ----
            {
                constexpr int NSEG = (W1 + XSEG - 1) / XSEG;
                for (int task = tid; task < 3 * H1 * NSEG; task += NT) {
                    const int f = task / (H1 * NSEG);
                    const int rem = task - f * (H1 * NSEG);
                    const int r = rem / NSEG, sg = rem - (rem / NSEG) * NSEG;
                    const int c0 = sg * XSEG < W1 - XSEG ? sg * XSEG : W1 - XSEG;
                    float o[XSEG];
                    if (tin) {
                        xfilter_row<RS, XSEG>(&lds.mid1[f][r * W0 + c0], g, o);
                    } else {
#pragma unroll
                        for (int i = 0; i < XSEG; ++i) o[i] = 0.f;
                    }
#pragma unroll
                    for (int i = 0; i < XSEG; ++i) lds.ring1[slot1][f][r * W1 + c0 + i] = o[i];
                }
            }
            __syncthreads();
            if (s_ < 2 * RT) continue;  // the ring does not hold frame t - r_t's neighbours yet
            // ---- (D) step 1 output frame t1 = t - r_t over the step-1 output region ----
            const int t1 = t - RT;
            const bool t1in = t1 >= 0 && t1 < T;
            const int s1 = s_ - 2 * RT;  // index of t1 among the step-1 outputs
            const int oslot_t1 = (s_ - RT) % NO;
            if (t1in) {
                for (int q = tid; q < H1 * W1; q += NT) {
                    float tf[3] = {0.f, 0.f, 0.f};
#pragma unroll
                    for (int m = 0; m < NR; ++m) {
                        const int sl = (s_ - 2 * RT + m) % NR;
#pragma unroll
                        for (int f = 0; f < 3; ++f) tf[f] = fmaf(gt[m], lds.ring1[sl][f][q], tf[f]);
                    }
                    const float xo = lds.own1[oslot_t1][0][q], wo = lds.own1[oslot_t1][1][q],
                                fo = lds.own1[oslot_t1][2][q];
                    const float qv = fmaf(fo, fmaf(fo, tf[0], -2.f * tf[1]), tf[2]);
                    const float y1 = wo * fmaf(-alpha, qv, tf[0]);
                    const int r1 = q / W1, c1 = q - (q / W1) * W1;
                    const bool own = r1 >= RS && r1 < RS + TH && c1 >= RS && c1 < RS + TW;
                    if (own && t1 >= ta && t1 < tb) {
                        syy1 = fma((double)y1, (double)y1, syy1);
                        syx1 = fma((double)y1, (double)xo, syx1);
                        if (p.half) {
                            const int off = ((ty0 + p.PT + r1 - RS) * Wp + (tx0 + p.PL + c1 - RS)) * 4;
                            const __amdgpu_buffer_rsrc_t ry =
                                make_rsrc(Y + (int64_t)t1 * p.frame, frame_bytes);
                            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(y1), ry, off, 0, 0);
                        }
                    }
                    if (!p.half) {
                        const float u2 = wo * y1;
                        lds.fld2[0][q] = u2;
                        lds.fld2[1][q] = fo * u2;
                        lds.fld2[2][q] = fo * (fo * u2);
                        if (own) {
                            const int qq = (r1 - RS) * TW + (c1 - RS);
                            lds.own2[s1 % NO][0][qq] = y1;
                            lds.own2[s1 % NO][1][qq] = wo;
                            lds.own2[s1 % NO][2][qq] = fo;
                        }
                    }
                }
            }
            __syncthreads();
            if (p.half) continue;  // uniform: one step only
            // ---- (E) step 2 on frame t1: y pass, then x pass into ring slot s1 % NR ----
            const int slot2 = s1 % NR;
            if (t1in) {
                for (int task = tid; task < 3 * W1; task += NT) {
                    const int f = task / W1, c = task - (task / W1) * W1;
                    yfilter_column<RS, TH>(&lds.fld2[f][c], W1, g, &lds.mid2[f][c], W1);
                }
            }
            __syncthreads();
            {
                constexpr int SEG2 = 8;
                constexpr int NSEG2 = TW / SEG2;
                for (int task = tid; task < 3 * TH * NSEG2; task += NT) {
                    const int f = task / (TH * NSEG2);
                    const int rem = task - f * (TH * NSEG2);
                    const int r = rem / NSEG2, sg = rem - (rem / NSEG2) * NSEG2;
                    float o[SEG2];
                    if (t1in) {
                        xfilter_row<RS, SEG2>(&lds.mid2[f][r * W1 + sg * SEG2], g, o);
                    } else {
#pragma unroll
                        for (int i = 0; i < SEG2; ++i) o[i] = 0.f;
                    }
#pragma unroll
                    for (int i = 0; i < SEG2; ++i) lds.ring2[slot2][f][r * TW + sg * SEG2 + i] = o[i];
                }
            }
            __syncthreads();
            if (s1 < 2 * RT) continue;
            // ---- (F) step 2 output frame t2 = t1 - r_t over the tile ----
            const int t2 = t1 - RT;  // in [ta, tb)
            const int oslot_t2 = (s1 - RT) % NO;
            const __amdgpu_buffer_rsrc_t ry = make_rsrc(Y + (int64_t)t2 * p.frame, frame_bytes);
            for (int q = tid; q < TH * TW; q += NT) {
                float tf[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int m = 0; m < NR; ++m) {
                    const int sl = (s1 - 2 * RT + m) % NR;
#pragma unroll
                    for (int f = 0; f < 3; ++f) tf[f] = fmaf(gt[m], lds.ring2[sl][f][q], tf[f]);
                }
                const float yo = lds.own2[oslot_t2][0][q], wo = lds.own2[oslot_t2][1][q],
                            fo = lds.own2[oslot_t2][2][q];
                const float qv = fmaf(fo, fmaf(fo, tf[0], -2.f * tf[1]), tf[2]);
                const float y2 = wo * fmaf(-alpha, qv, tf[0]);
                syy2 = fma((double)y2, (double)y2, syy2);
                syx2 = fma((double)y2, (double)yo, syx2);
                const int r = q / TW, c = q - (q / TW) * TW;
                const int off = ((ty0 + p.PT + r) * Wp + (tx0 + p.PL + c)) * 4;
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(y2), ry, off, 0, 0);
            }
        }
    }
    block_partials<NT>(syy1, syx1, p.part_out, lb);
    if (!p.half) {
        __syncthreads();  // block_partials reuses its LDS
        block_partials<NT>(syy2, syx2, p.part_out + 2 * gridDim.x, lb);
    }
}

template <int RS, int RT>
hipError_t launch_fused_t(const StepParams& p, int grid, hipStream_t s) {
    hipLaunchKernelGGL((step2_kernel<RS, RT>), dim3(grid), dim3(256), 0, s, p);
    return hipGetLastError();
}
template <int RS, int RT>
hipError_t occ_fused_t(int* blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, step2_kernel<RS, RT>, 256, 0);
}

template <int RS, int... RTs>
void fill_fused_rt(StepFns* t, std::integer_sequence<int, RTs...>) {
    ((t[RS * (SFSEG_MAX_RT + 1) + RTs] =
          StepFns{&launch_fused_t<RS, RTs>, &occ_fused_t<RS, RTs>, nullptr, nullptr}),
     ...);
}
template <int... RSs>
void fill_fused_rs(StepFns* t, std::integer_sequence<int, RSs...>) {
    (fill_fused_rt<RSs>(t, std::make_integer_sequence<int, FUSED_MAX_RT + 1>{}), ...);
}
// Radii up to FUSED_MAX_RS, FUSED_MAX_RT: the LDS of one block stays within
// the 160 KB of a CU.
struct FusedTable {
    StepFns fns[NCOMB] = {};
    FusedTable() { fill_fused_rs(fns, std::make_integer_sequence<int, FUSED_MAX_RS + 1>{}); }
};

}  // namespace detail
}  // namespace sfseg

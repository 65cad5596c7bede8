// Kernels of the warm-start network (3D U-Net) for gfx950.
//
// The power iteration starts from a soft segmentation (Sec. 4, Algorithm 1);
// this network maps the input map S to an estimate of the principal
// eigenvector, and plain iterations then run to the same tolerance.
//
// Activations are bfloat16, channels-last: voxel v = (t * H + y) * W + x of a
// view holds its C channels at base[v * CS + c0 + c] (a view can be a channel
// slice of a wider buffer, which is how the skip concatenations are formed
// without copies).  Weights: FP32 master copies in the exchange layout
// (Cout, Cin, 3, 3, 3); the matrix cores read bfloat16 "fragments" prepared
// from them.  Accumulation is FP32; loss and bias/head reductions are FP64.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16:
//   forward      out[v][co] = b[co] + sum_k A[v][k] Wk[k][co],
//                k = tap * CIN + ci, A[v][k] = in[v + offset(tap)][ci]
//                (zero outside the volume), tap = (dt+1)*9 + (dy+1)*3 + (dx+1);
//   backward-data is the same product with CIN' = COUT, COUT' = CIN and the
//                taps mirrored (tap' = 26 - tap): it runs the forward kernel
//                on re-arranged fragments;
//   weight gradient gW[tap][co][ci] = sum_v gz[v][co] in[v + offset(tap)][ci]
//                with K = voxels (32 consecutive voxels of a row per step).
// MFMA operand layout (16x16x32): lane l holds A[i = l % 16][k = 8 (l / 16)
// + e] and B[k = 8 (l / 16) + e][j = l % 16] for e = 0..7; the result
// D[i][j] sits in lane j + 16 (i / 4), register i % 4.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <utility>

namespace sfseg {
namespace unet {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// A channels-last bfloat16 view.
struct View {
    __bf16* p;
    int32_t T, H, W;
    int32_t cs;  // channel stride of a voxel
    int32_t c0;  // first channel of the view
};

__device__ __forceinline__ bf16x8 load8(const __bf16* p) {
    const u32x4_t u = *reinterpret_cast<const u32x4_t*>(p);
    return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ bf16x8 zero8() {
    const u32x4_t u = {0u, 0u, 0u, 0u};
    return __builtin_bit_cast(bf16x8, u);
}

// ---------------------------------------------------------------------------
// Implicit-GEMM convolution (forward, or backward-data on mirrored fragments)
// ---------------------------------------------------------------------------
// The head's activation.
__device__ __forceinline__ float softplus(float z) { return z > 20.f ? z : log1pf(expf(z)); }

// frag[((q * NB + nb) * 64 + lane)] holds the 8 B-operand values of K chunk
// q (k = 32 q + 8 (lane / 16) + e) and output block nb (co = 16 nb + lane %
// 16).  mode 0: + bias, ReLU; mode 1: no bias, multiply by (mask > 0) if
// mask.p is set.
//
// The product runs with the input staged in LDS and streamed along t.  A
// block (four waves) owns RB output rows (y0 .. y0 + RB - 1) x XB voxels
// (x0 .. x0 + XB - 1) x all COUT channels over a run of output frames
// [ta, tb): NT = RB XB / 16 tiles of 16 voxels per frame, wave w taking the
// MT = NT / 4 consecutive tiles from w MT (row-major over the block's rows).
// LDS holds a ring of four frame slabs; slab slot s % 4 holds input frame s:
// rows y0-1 .. y0+RB, voxels x0-1 .. x0+XB, all CIN channels (zeros outside
// the volume), as 16-byte units of 8 channels laid out [row][channel
// group][voxel], so that the 16 lanes of a lane group, which read 16
// consecutive voxels of one channel group for one tap, read 256 contiguous
// bytes.  For output frame t the products read slots t-1, t, t+1 while the
// loads of frame t+2 are in flight into registers; they are written to slot
// t+2 (which held t-2) after the products, then one barrier.  Each input
// value thus leaves global memory about (RB + 2) / RB times per block row
// instead of once per tap.
// K chunk Q of the product (k = 32 Q .. 32 Q + 31, k = tap * CIN + channel):
// lane group g holds k = 32 Q + 8 g .. + 7.  The chunk starts on tap tl; lane
// groups g >= gs are on the next tap th (gs = 4: none).  For each of the two
// taps, the input frame f (0..2 for t-1 .. t+1) and the unit offset inside a
// frame slab relative to the lane's base ((row * NCG + g) * VOX + voxel):
// row shift dy, channel group, voxel shift dx.  Past the last tap the
// fragments hold zeros and the offsets point at loaded values of frame t.
template <int CIN, int NCG, int VOX, int Q>
struct ConvChunk {
    static constexpr int k0 = 32 * Q;
    static constexpr int tl = k0 / CIN, th = (k0 + 31) / CIN;
    static constexpr int gs = th == tl ? 4 : (CIN * th - k0) / 8;
    static constexpr int fl = tl < 27 ? tl / 9 : 1;
    static constexpr int ol = tl < 27 ? (((tl / 3) % 3) * NCG + (k0 - CIN * tl) / 8) * VOX + tl % 3 : 0;
    static constexpr int fh = th < 27 ? th / 9 : 1;
    static constexpr int oh = th < 27 ? (((th / 3) % 3) * NCG - gs) * VOX + th % 3 : -gs * VOX;
};

template <typename F, int... Qs>
__device__ __forceinline__ void for_each_chunk(F&& f, std::integer_sequence<int, Qs...>) {
    (f(std::integral_constant<int, Qs>{}), ...);
}

template <int CIN, int COUT, int RB, int XB>
struct ConvLds {
    static constexpr int NCG = CIN / 8;     // 8-channel groups
    static constexpr int ROWS = RB + 2;
    static constexpr int VOX = XB + 2;      // outputs plus one voxel each side
    static constexpr int UNITS = ROWS * NCG * VOX;  // 16-byte units per frame slab
    static constexpr int PER = (UNITS + 255) / 256; // units per thread
    static constexpr int TPR = XB / 16;     // tiles per row
    static constexpr int MT = RB * TPR / 4; // tiles per wave
    static_assert(MT >= 1 && TPR % MT == 0, "a wave's tiles lie in one row");
};

//
// With UP, input channels [0, cup) are the nearest-neighbour 2x upsampling
// of `up` (half resolution), read at the parent voxel while the slab is
// staged, and channels [cup, CIN) are channels 0 .. CIN - cup - 1 of `in`:
// the upsampled part of a concatenation is never written out (inference
// only; training keeps the concatenated tensor for the backward pass).
// With HEAD (COUT = 16, mode 0), the outputs are not stored: the 1x1x1 head
// of the network reads them, rounded to bfloat16 as a stored activation
// would be, and head_out[v] = softplus(head_w[16] + sum_c head_w[c] out[v][c])
// is written instead (the same arithmetic, in the same order, as head_fwd).
//
// With KS = 4 (split K), the four waves share the block's NT = RB XB / 16
// tiles and each takes every fourth K chunk (chunk q to wave q % 4); their
// partial sums meet in LDS and wave w adds the four, in wave order, for its
// own MT tiles.  The weight fragments, which do not fit in registers for the
// wide layers, are then read once per block and frame instead of once per
// wave and frame.
template <int CIN, int COUT, int RB, int XB, bool UP, bool HEAD = false, int KS = 1>
__global__ __launch_bounds__(256) void conv3_stream(View in, View up, int cup, View out,
                                                     const bf16x8* __restrict__ frag,
                                                     const float* __restrict__ bias, View mask,
                                                     int mode, int runs,
                                                     const float* __restrict__ head_w = nullptr,
                                                     float* __restrict__ head_out = nullptr) {
    using G = ConvLds<CIN, COUT, RB, XB>;
    constexpr int NB = COUT / 16;
    constexpr int NQ = (27 * CIN + 31) / 32;
    constexpr int NCG = G::NCG, VOX = G::VOX, MT = G::MT, UNITS = G::UNITS, PER = G::PER;
    static_assert(CIN % 8 == 0 && COUT % 16 == 0, "channel blocking");
    static_assert(KS == 1 || KS == 4, "split K over all four waves or none");
    // tiles in a wave's products: its own MT, or all of the block's with KS = 4
    constexpr int MP = KS == 1 ? MT : 4 * MT;
    __shared__ u32x4_t slab[4][UNITS];
    // Output staging: each wave's tiles as [tile][voxel][16 channels] bf16, so
    // that the stores to the channels-last output are 16 bytes per lane.
    __shared__ __bf16 obuf[4][MT * NB][16 * 16];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int T = out.T, H = out.H, W = out.W;
    const int tiles_x = (W + XB - 1) / XB;
    const int rows_y = (H + RB - 1) / RB;
    int b = blockIdx.x;
    const int tx = b % tiles_x;
    b /= tiles_x;
    const int ty = b % rows_y;
    const int run = b / rows_y;
    const int ta = (int)((int64_t)T * run / runs), tb = (int)((int64_t)T * (run + 1) / runs);
    const int x0 = tx * XB, y0 = ty * RB;
    const u32x4_t zero = {0u, 0u, 0u, 0u};

    // This thread's units of a frame slab, unit u = (r * NCG + cg) * VOX + v:
    // their element offsets inside an input frame of `in` or, for upsampled
    // channels, of `up` (-1 outside the picture).
    int64_t uoff[PER];
    bool fromup[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int u = j * 256 + threadIdx.x;
        const int v = u % VOX, rest = u / VOX;
        const int cg = rest % NCG, r = rest / NCG;
        const int ys = y0 + r - 1, xs = x0 + v - 1;
        const bool ok = u < UNITS && ys >= 0 && ys < H && xs >= 0 && xs < W;
        fromup[j] = UP && 8 * cg < cup;
        uoff[j] = !ok ? -1
                      : fromup[j] ? ((int64_t)(ys >> 1) * up.W + (xs >> 1)) * up.cs + up.c0 + 8 * cg
                                  : ((int64_t)ys * W + xs) * in.cs + in.c0 + 8 * cg - (UP ? cup : 0);
    }
    const int64_t fstride = (int64_t)H * W * in.cs;
    const int64_t ustride = (int64_t)up.H * up.W * up.cs;
    auto load_frame = [&](int ts, u32x4_t* reg) {
        const bool tin = ts >= 0 && ts < T;
        const __bf16* fb = in.p + (tin ? (int64_t)ts * fstride : 0);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            u32x4_t val = zero;
            if constexpr (UP) {
                const __bf16* ub = up.p + (tin ? (int64_t)(ts >> 1) * ustride : 0);
                if (tin && uoff[j] >= 0)
                    val = *reinterpret_cast<const u32x4_t*>((fromup[j] ? ub : fb) + uoff[j]);
            } else {
                if (tin && uoff[j] >= 0) val = *reinterpret_cast<const u32x4_t*>(fb + uoff[j]);
            }
            reg[j] = val;
        }
    };
    auto store_slot = [&](int ts, const u32x4_t* reg) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int u = j * 256 + threadIdx.x;
            if (u < UNITS) slab[ts & 3][u] = reg[j];
        }
    };
    {
        u32x4_t reg[PER];
        for (int ts = ta - 1; ts <= ta + 1; ++ts) {
            load_frame(ts, reg);
            store_slot(ts, reg);
        }
    }
    // Loads run PD frames ahead of their slot: with PD = 2 the values of frame
    // t + 2 arrive during frame t - 1 and wait in `ahead` (registers allowing).
    constexpr int PD = (NQ * NB <= 42 && NQ * NB > 28) ? 1 : 2;
    u32x4_t ahead[PD == 2 ? PER : 1];
    if constexpr (PD == 2) load_frame(ta + 2, ahead);
    __syncthreads();

    const int tile0 = wave * MT;
    const int row = tile0 / G::TPR;          // output row inside the block
    const int v0 = 16 * (tile0 % G::TPR);    // first output voxel of the wave in the row
    const int y = y0 + row;
    const int i = lane & 15, g = lane >> 4;
    // Weight fragments: held in registers for the whole run where they fit
    // (4 NQ NB registers), else re-read from L1 / L2 for every frame.
    constexpr bool BREG = KS == 1 && NQ * NB <= 42;
    bf16x8 breg[BREG ? NQ : 1][NB];
    if constexpr (BREG) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int n = 0; n < NB; ++n) breg[q][n] = frag[(q * NB + n) * 64 + lane];
    }
    for (int t = ta; t < tb; ++t) {
        u32x4_t next[PER];
        load_frame(t + 1 + PD, next);  // consumed after this frame's products (PD = 1)
                                       // or the next frame's (PD = 2)
        f32x4 acc[MP][NB];
#pragma unroll
        for (int m = 0; m < MP; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
        // the lane's base in the slabs of frames t-1, t, t+1 (all loaded): at
        // the wave's first tile, or at the block's first with KS = 4; tile m
        // of the products then sits at tile_off(m) units from it
        const int lane_off = KS == 1 ? (row * NCG + g) * VOX + v0 + i : g * VOX + i;
        auto tile_off = [](int m) {
            return KS == 1 ? 16 * m : (m / G::TPR) * NCG * VOX + 16 * (m % G::TPR);
        };
        const u32x4_t* fb[3] = {&slab[(t + 3) & 3][lane_off], &slab[t & 3][lane_off],
                                &slab[(t + 1) & 3][lane_off]};
        // A operands of chunk qc (one per tile) from the slabs, and the products
        auto reada = [&](auto qc, bf16x8* a) {
            using C = ConvChunk<CIN, NCG, VOX, decltype(qc)::value>;
            const u32x4_t* sp =
                (C::gs == 4 || g < C::gs) ? fb[C::fl] + C::ol : fb[C::fh] + C::oh;
#pragma unroll
            for (int m = 0; m < MP; ++m) a[m] = __builtin_bit_cast(bf16x8, sp[tile_off(m)]);
        };
        auto mma = [&](const bf16x8* a, const bf16x8* bf) {
#pragma unroll
            for (int m = 0; m < MP; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bf[n], acc[m][n], 0, 0, 0);
        };
        if constexpr (BREG && NQ * NB <= 14) {
            // the smallest layer: four waves per SIMD hide the slab reads,
            // which a read-ahead would cost (its registers allow three)
            for_each_chunk(
                [&](auto qc) {
                    bf16x8 a[MP];
                    reada(qc, a);
                    mma(a, breg[decltype(qc)::value]);
                },
                std::make_integer_sequence<int, NQ>{});
        } else if constexpr (BREG) {
            // the slab reads of chunk q + 1 issued before chunk q's products
            bf16x8 ab[2][MP];
            reada(std::integral_constant<int, 0>{}, ab[0]);
            for_each_chunk(
                [&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    if constexpr (q + 1 < NQ) reada(std::integral_constant<int, q + 1>{}, ab[(q + 1) & 1]);
                    __builtin_amdgcn_sched_barrier(0);
                    mma(ab[q & 1], breg[q]);
                },
                std::make_integer_sequence<int, NQ>{});
        } else {
            // re-read every frame, not hoisted out of the frame loop; the
            // pointer is cast back to the global address space after the
            // barrier, else the reads become flat loads, which the LDS
            // counter also tracks, and every one of them waits for the slab
            // reads in flight
            const bf16x8* fp = frag;
            asm volatile("" : "+s"(fp));
            const __attribute__((address_space(1))) bf16x8* fr =
                (const __attribute__((address_space(1))) bf16x8*)fp;
            // The wave's chunks W, W + KS, ... as straight-line code in a
            // software pipeline: step j issues the slab reads of chunk j + 1
            // and the fragment loads of chunk j + D (a ring of D fragment sets
            // in registers), then chunk j's products; the scheduling barrier
            // keeps the compiler from sinking the loads back to their uses.
            constexpr int D = NB <= 2 ? 4 : NB <= 4 ? 3 : 2;
            auto run = [&](auto wc) {
                constexpr int W = decltype(wc)::value;
                constexpr int L = (NQ - W + KS - 1) / KS;
                bf16x8 pf[D][NB];
                bf16x8 ab[2][MP];
                auto load = [&](bf16x8* dst, int q) {
#pragma unroll
                    for (int n = 0; n < NB; ++n) dst[n] = fr[(q * NB + n) * 64 + lane];
                };
                for_each_chunk(
                    [&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        if constexpr (j < L) load(pf[j], W + KS * j);
                    },
                    std::make_integer_sequence<int, D>{});
                reada(std::integral_constant<int, W>{}, ab[0]);
                for_each_chunk(
                    [&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        if constexpr (j + 1 < L)
                            reada(std::integral_constant<int, W + KS * (j + 1)>{}, ab[(j + 1) & 1]);
                        bf16x8 cur[NB];
#pragma unroll
                        for (int n = 0; n < NB; ++n) cur[n] = pf[j % D][n];
                        if constexpr (j + D < L) load(pf[j % D], W + KS * (j + D));
                        __builtin_amdgcn_sched_barrier(0);
                        mma(ab[j & 1], cur);
                    },
                    std::make_integer_sequence<int, L>{});
            };
            if constexpr (KS == 1) {
                run(std::integral_constant<int, 0>{});
            } else {
                switch (wave) {
                    case 0: run(std::integral_constant<int, 0>{}); break;
                    case 1: run(std::integral_constant<int, 1>{}); break;
                    case 2: run(std::integral_constant<int, 2>{}); break;
                    default: run(std::integral_constant<int, 3>{}); break;
                }
            }
        }
        if constexpr (KS > 1) {
            // the four waves' partial sums of this wave's tiles, in wave order;
            // red[wave][tile * NB + block of 16 channels][lane]
            __shared__ f32x4 red[4][MP * NB][64];
#pragma unroll
            for (int m = 0; m < MP; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n) red[wave][m * NB + n][lane] = acc[m][n];
            __syncthreads();
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n) {
                    f32x4 sum = red[0][(tile0 + m) * NB + n][lane];
#pragma unroll
                    for (int k = 1; k < 4; ++k) sum += red[k][(tile0 + m) * NB + n][lane];
                    acc[m][n] = sum;
                }
        }
        // bias and ReLU in the accumulator layout (lane: channel i, voxels
        // 4 g .. 4 g + 3), through LDS into [voxel][channel], then 16-byte
        // stores of 8 channels, the mask applied on those
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const float bco = mode == 0 ? bias[16 * n + i] : 0.f;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    float val = acc[m][n][rr];
                    if (mode == 0) val = fmaxf(val + bco, 0.f);
                    obuf[wave][m * NB + n][(4 * g + rr) * 16 + i] = (__bf16)val;
                }
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if constexpr (HEAD) {
            static_assert(NB == 1 && MT * 16 <= 64, "head: 16 channels, a voxel per lane");
            const int m = lane >> 4, vv = lane & 15;
            const int xo = x0 + v0 + 16 * m + vv;
            if (y < H && lane < MT * 16 && xo < W) {
                const bf16x8 lo = load8(&obuf[wave][m][vv * 16]);
                const bf16x8 hi = load8(&obuf[wave][m][vv * 16 + 8]);
                float z = head_w[16];
#pragma unroll
                for (int c = 0; c < 8; ++c) z = fmaf(head_w[c], (float)lo[c], z);
#pragma unroll
                for (int c = 0; c < 8; ++c) z = fmaf(head_w[8 + c], (float)hi[c], z);
                head_out[((int64_t)t * H + y) * W + xo] = softplus(z);
            }
        } else if (y < H) {
            const int64_t obase = ((int64_t)t * H + y) * W;
#pragma unroll
            for (int c0 = 0; c0 < MT * NB * 32; c0 += 64) {
                const int c = c0 + lane;
                const int tl = c >> 5, vv = (c & 31) >> 1, half = c & 1;
                const int m = tl / NB, n = tl - m * NB;
                const int xo = x0 + v0 + 16 * m + vv;
                if (c < MT * NB * 32 && xo < W) {
                    const int64_t v = obase + xo;
                    u32x4_t o = *reinterpret_cast<const u32x4_t*>(&obuf[wave][tl][vv * 16 + 8 * half]);
                    if (mode != 0 && mask.p) {
                        const bf16x8 mk = load8(mask.p + v * mask.cs + mask.c0 + 16 * n + 8 * half);
                        bf16x8 ov = __builtin_bit_cast(bf16x8, o);
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            if (!((float)mk[e] > 0.f)) ov[e] = (__bf16)0.f;
                        o = __builtin_bit_cast(u32x4_t, ov);
                    }
                    *reinterpret_cast<u32x4_t*>(out.p + v * out.cs + out.c0 + 16 * n + 8 * half) = o;
                }
            }
        }
        // slot of frame t - 2, read by no one now
        if constexpr (PD == 2) {
            store_slot(t + 2, ahead);
#pragma unroll
            for (int j = 0; j < PER; ++j) ahead[j] = next[j];
        } else {
            store_slot(t + 2, next);
        }
        __syncthreads();
    }
}

// First layer: one FP32 input channel, K = the 27 taps (one chunk of 32; the
// weights of k = 27 .. 31 are zero).  Streamed like conv3_stream: a block
// owns C1_RB rows x C1_XB voxels over a run of frames and keeps a ring of four
// FP32 frame slabs ((C1_RB + 2) rows x (C1_XB + 2) voxels, zeros outside the
// volume), the loads of frame t + 2 in registers during frame t.  Wave w
// computes row w; lane group g reads taps 8 g .. 8 g + 7 of its voxel from the
// slabs (a tap past the last reads the centre value, whose weight is zero).
constexpr int C1_RB = 4, C1_XB = 64;

template <int COUT>
__global__ __launch_bounds__(256) void conv3_c1_stream(const float* __restrict__ in, View out,
                                                        const bf16x8* __restrict__ frag,
                                                        const float* __restrict__ bias, int runs) {
    constexpr int NB = COUT / 16, MT = C1_XB / 16;
    constexpr int VOXS = C1_XB + 2, UNITS = (C1_RB + 2) * VOXS, SLOT = 512;
    constexpr int PER = (UNITS + 255) / 256;
    static_assert(UNITS <= SLOT && C1_RB == 4, "slab size, one row per wave");
    __shared__ float slab[4 * SLOT];
    __shared__ __bf16 obuf[4][MT * NB][16 * 16];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int T = out.T, H = out.H, W = out.W;
    const int tiles_x = (W + C1_XB - 1) / C1_XB;
    const int rows_y = (H + C1_RB - 1) / C1_RB;
    int b = blockIdx.x;
    const int tx = b % tiles_x;
    b /= tiles_x;
    const int ty = b % rows_y;
    const int run = b / rows_y;
    const int ta = (int)((int64_t)T * run / runs), tb = (int)((int64_t)T * (run + 1) / runs);
    const int x0 = tx * C1_XB, y0 = ty * C1_RB;

    // this thread's slab units u = r * VOXS + v: offsets inside an input frame
    int goff[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int u = j * 256 + threadIdx.x;
        const int r = u / VOXS, v = u - r * VOXS;
        const int ys = y0 + r - 1, xs = x0 + v - 1;
        goff[j] = (u < UNITS && ys >= 0 && ys < H && xs >= 0 && xs < W) ? ys * W + xs : -1;
    }
    const int64_t fstride = (int64_t)H * W;
    auto load_frame = [&](int ts, float* reg) {
        const bool tin = ts >= 0 && ts < T;
        const float* fb = in + (tin ? (int64_t)ts * fstride : 0);
#pragma unroll
        for (int j = 0; j < PER; ++j) reg[j] = (tin && goff[j] >= 0) ? fb[goff[j]] : 0.f;
    };
    auto store_slot = [&](int ts, const float* reg) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int u = j * 256 + threadIdx.x;
            if (u < UNITS) slab[(ts & 3) * SLOT + u] = reg[j];
        }
    };
    {
        float reg[PER];
        for (int ts = ta - 1; ts <= ta + 1; ++ts) {
            load_frame(ts, reg);
            store_slot(ts, reg);
        }
    }
    float ahead[PER];
    load_frame(ta + 2, ahead);
    __syncthreads();

    const int i = lane & 15, g = lane >> 4;
    const int y = y0 + wave;
    // the lane's taps: frame shift and offset inside a slab
    int tdt[8], toff[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int tap = 8 * g + e;
        const bool live = tap < 27;
        const int dt = live ? tap / 9 - 1 : 0, dy = live ? (tap / 3) % 3 - 1 : 0,
                  dx = live ? tap % 3 - 1 : 0;
        tdt[e] = dt;
        toff[e] = (wave + 1 + dy) * VOXS + 1 + dx + i;
    }
    bf16x8 breg[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) breg[n] = frag[n * 64 + lane];
    for (int t = ta; t < tb; ++t) {
        float next[PER];
        load_frame(t + 3, next);
        int base[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) base[e] = ((t + tdt[e]) & 3) * SLOT + toff[e];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            bf16x8 a;
#pragma unroll
            for (int e = 0; e < 8; ++e) a[e] = (__bf16)slab[base[e] + 16 * m];
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    a, breg[n], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                const float bco = bias[16 * n + i];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    obuf[wave][m * NB + n][(4 * g + r) * 16 + i] = (__bf16)fmaxf(acc[r] + bco, 0.f);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (y < H) {
            const int64_t obase = ((int64_t)t * H + y) * W;
#pragma unroll
            for (int c0 = 0; c0 < MT * NB * 32; c0 += 64) {
                const int c = c0 + lane;
                const int tl = c >> 5, vv = (c & 31) >> 1, half = c & 1;
                const int m = tl / NB, n = tl - m * NB;
                const int xo = x0 + 16 * m + vv;
                if (xo < W)
                    *reinterpret_cast<u32x4_t*>(out.p + (obase + xo) * out.cs + out.c0 + 16 * n +
                                                8 * half) =
                        *reinterpret_cast<const u32x4_t*>(&obuf[wave][tl][vv * 16 + 8 * half]);
            }
        }
        // slot of frame t - 2, read by no one now
        store_slot(t + 2, ahead);
#pragma unroll
        for (int j = 0; j < PER; ++j) ahead[j] = next[j];
        __syncthreads();
    }
}

// B-operand fragments from FP32 weights w[(co * cin + ci) * 27 + tap].
// mirrored = 0: forward fragments of a (cin -> cout) conv;
// mirrored = 1: backward-data fragments, i.e. forward fragments of the
//               (cout -> cin) conv with W'[co' = ci][ci' = co][tap] =
//               W[co][ci][26 - tap].
__global__ void make_fragments(const float* __restrict__ w, int cin, int cout, int mirrored,
                               bf16x8* __restrict__ frag) {
    const int fin = mirrored ? cout : cin;    // input channels of the product
    const int fout = mirrored ? cin : cout;   // output channels of the product
    const int nb_all = fout / 16;
    const int nq = (27 * fin + 31) / 32;
    const int total = nq * nb_all * 64;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int lane = idx & 63;
        const int nb = (idx >> 6) % nb_all;
        const int q = (idx >> 6) / nb_all;
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 32 * q + 8 * (lane >> 4) + e;
            const int tap = k / fin, c = k - tap * fin;  // c: input channel of the product
            const int o = 16 * nb + (lane & 15);         // output channel of the product
            float x = 0.f;
            if (tap < 27)
                x = mirrored ? w[((int64_t)c * cin + o) * 27 + (26 - tap)]
                             : w[((int64_t)o * cin + c) * 27 + tap];
            v[e] = (__bf16)x;
        }
        frag[idx] = v;
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: per (chunk of rows, tap) block partial sums
// ---------------------------------------------------------------------------
// gW[tap][co][ci] = sum_v gz[v][co] in[v + offset(tap)][ci].  M = co, N = ci,
// K = 32 consecutive voxels of a row.  Block (blockIdx.x = chunk, blockIdx.y =
// tap) covers units [u0, u1) of (row, 32-voxel segment); its four waves split
// the units, then add their accumulators through LDS in a fixed order.
// part[((chunk * 27 + tap) * COUT + co) * CIN + ci].
template <int CIN, int COUT, bool IN_F32>
__global__ __launch_bounds__(256) void conv3_wgrad(View gz, View in, const float* __restrict__ in32,
                                                    int units_per_chunk, float* __restrict__ part) {
    constexpr int MB = COUT / 16;
    constexpr int NBC = IN_F32 ? 1 : CIN / 16;
    constexpr int CI = IN_F32 ? 1 : CIN;
    __shared__ float red[4][MB * NBC * 4 * 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int T = gz.T, H = gz.H, W = gz.W;
    const int segs = (W + 31) / 32;
    const int64_t units = (int64_t)T * H * segs;
    const int tap = blockIdx.y;
    const int dt = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int j = lane & 15, g = lane >> 4;
    f32x4 acc[MB][NBC];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < NBC; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int64_t u0 = (int64_t)blockIdx.x * units_per_chunk;
    int64_t u1 = u0 + units_per_chunk;
    if (u1 > units) u1 = units;
    for (int64_t u = u0 + wave; u < u1; u += 4) {
        const int row = (int)(u / segs);
        const int xb = (int)(u - (int64_t)row * segs) * 32 + 8 * g;
        const int t = row / H, y = row - t * H;
        const int ts = t + dt, ys = y + dy;
        const bool rowok = ts >= 0 && ts < T && ys >= 0 && ys < H;
        const int64_t gbase = ((int64_t)t * H + y) * W;
        const int64_t sbase = ((int64_t)ts * H + ys) * W;
        bf16x8 a[MB], b[NBC];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int x = xb + e;
                a[m][e] = x < W ? gz.p[(gbase + x) * gz.cs + gz.c0 + 16 * m + j] : (__bf16)0.f;
            }
        }
#pragma unroll
        for (int n = 0; n < NBC; ++n) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int x = xb + e, xs = x + dx;
                const bool ok = rowok && x < W && xs >= 0 && xs < W;
                if constexpr (IN_F32) {
                    b[n][e] = (ok && j == 0) ? (__bf16)in32[sbase + xs] : (__bf16)0.f;
                } else {
                    b[n][e] = ok ? in.p[(sbase + xs) * in.cs + in.c0 + 16 * n + j] : (__bf16)0.f;
                }
            }
        }
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int n = 0; n < NBC; ++n)
                acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[n], acc[m][n], 0, 0, 0);
    }
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < NBC; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wave][((m * NBC + n) * 4 + r) * 64 + lane] = acc[m][n][r];
    __syncthreads();
    float* dst = part + ((int64_t)blockIdx.x * 27 + tap) * COUT * CI;
    for (int idx = threadIdx.x; idx < MB * NBC * 4 * 64; idx += 256) {
        const float s = ((red[0][idx] + red[1][idx]) + red[2][idx]) + red[3][idx];
        const int l = idx & 63, r = (idx >> 6) & 3, mn = idx >> 8;
        const int m = mn / NBC, n = mn - m * NBC;
        const int co = 16 * m + 4 * (l >> 4) + r, ci = 16 * n + (l & 15);
        if (ci < CI) dst[co * CI + ci] = s;
    }
}

// gW (exchange layout (co, ci, tap)) = sum over chunks, in chunk order.
__global__ void wgrad_reduce(const float* __restrict__ part, int chunks, int cin, int cout,
                             float* __restrict__ gw) {
    const int n = cout * cin * 27;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += gridDim.x * blockDim.x) {
        const int tap = idx % 27;
        const int ci = (idx / 27) % cin;
        const int co = idx / (27 * cin);
        double s = 0.0;
        for (int c = 0; c < chunks; ++c)
            s += part[(((int64_t)c * 27 + tap) * cout + co) * cin + ci];
        gw[idx] = (float)s;
    }
}

// Per-channel sums of a view over its voxels: block partials (FP64), one row
// per block, part[block * C + c].
__global__ void channel_sums(View v, int C, double* __restrict__ part) {
    extern __shared__ double cs_sm[];
    const int64_t nvox = (int64_t)v.T * v.H * v.W;
    const int lanes_per_c = blockDim.x / C;
    const int c = threadIdx.x % C, sub = threadIdx.x / C;
    double s = 0.0;
    if (sub < lanes_per_c) {
        for (int64_t p = (int64_t)blockIdx.x * lanes_per_c + sub; p < nvox;
             p += (int64_t)gridDim.x * lanes_per_c)
            s += (double)(float)v.p[p * v.cs + v.c0 + c];
    }
    cs_sm[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < C) {
        double tot = 0.0;
        for (int k = 0; k < lanes_per_c; ++k) tot += cs_sm[k * C + threadIdx.x];
        part[(int64_t)blockIdx.x * C + threadIdx.x] = tot;
    }
}

// out[c] = sum over blocks of part[block * C + c], in block order.
__global__ void sum_partials(const double* __restrict__ part, int blocks, int C,
                             float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += part[(int64_t)b * C + c];
    out[c] = (float)s;
}

// ---------------------------------------------------------------------------
// Pooling and upsampling
// ---------------------------------------------------------------------------
// out (ceil sizes) = 2x2x2 average of in over a zero-padded window.
__global__ void pool2_fwd(View in, View out, int C) {
    // one thread per (output voxel, 8 channels): 16-byte loads and stores
    const int C8 = C / 8;
    const int64_t n = (int64_t)out.T * out.H * out.W * C8;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int c = 8 * (int)(idx % C8);
        const int64_t v = idx / C8;
        const int xo = (int)(v % out.W), yo = (int)((v / out.W) % out.H), to = (int)(v / ((int64_t)out.W * out.H));
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int d = 0; d < 2; ++d) {
                    const int t = 2 * to + a, y = 2 * yo + b, x = 2 * xo + d;
                    if (t < in.T && y < in.H && x < in.W) {
                        const bf16x8 q = load8(in.p + (((int64_t)t * in.H + y) * in.W + x) * in.cs + in.c0 + c);
#pragma unroll
                        for (int e = 0; e < 8; ++e) s[e] += (float)q[e];
                    }
                }
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = (__bf16)(s[e] * 0.125f);
        *reinterpret_cast<u32x4_t*>(out.p + v * out.cs + out.c0 + c) = __builtin_bit_cast(u32x4_t, o);
    }
}

// g_in[v] = g_out[parent(v)] / 8 + skip[v], then zero where act[v] <= 0.
__global__ void pool2_bwd(View gout, View skip, View act, View gin, int C) {
    const int64_t n = (int64_t)gin.T * gin.H * gin.W * C;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(idx % C);
        const int64_t v = idx / C;
        const int x = (int)(v % gin.W), y = (int)((v / gin.W) % gin.H), t = (int)(v / ((int64_t)gin.W * gin.H));
        const int64_t pv = ((int64_t)(t >> 1) * gout.H + (y >> 1)) * gout.W + (x >> 1);
        float s = (float)gout.p[pv * gout.cs + gout.c0 + c] * 0.125f;
        s += (float)skip.p[v * skip.cs + skip.c0 + c];
        if (!((float)act.p[v * act.cs + act.c0 + c] > 0.f)) s = 0.f;
        gin.p[v * gin.cs + gin.c0 + c] = (__bf16)s;
    }
}

// out[v] = in[parent(v)] (nearest 2x, cropped to out's size).
template <typename I>
__device__ __forceinline__ void up2_body(const View& in, const View& out, int C8, I n) {
    for (I idx = (I)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (I)gridDim.x * blockDim.x) {
        const int c = 8 * (int)(idx % (I)C8);
        const I v = idx / (I)C8;
        const I hw = (I)out.H * (I)out.W;
        const int t = (int)(v / hw);
        const I rem = v - (I)t * hw;
        const int y = (int)(rem / (I)out.W), x = (int)(rem - (I)y * (I)out.W);
        const int64_t pv = ((int64_t)(t >> 1) * in.H + (y >> 1)) * in.W + (x >> 1);
        *reinterpret_cast<u32x4_t*>(out.p + (int64_t)v * out.cs + out.c0 + c) =
            *reinterpret_cast<const u32x4_t*>(in.p + pv * in.cs + in.c0 + c);
    }
}

__global__ void up2_fwd(View in, View out, int C) {
    // one thread per (output voxel, 8 channels): 16-byte loads and stores;
    // index arithmetic in 32 bits where the index range allows
    const int C8 = C / 8;
    const int64_t n = (int64_t)out.T * out.H * out.W * C8;
    if (n < ((int64_t)1 << 32))
        up2_body<uint32_t>(in, out, C8, (uint32_t)n);
    else
        up2_body<uint64_t>(in, out, C8, (uint64_t)n);
}

// g_in[p] = sum of g_out over p's children inside g_out, zero where act[p] <= 0.
__global__ void up2_bwd(View gout, View act, View gin, int C) {
    const int64_t n = (int64_t)gin.T * gin.H * gin.W * C;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(idx % C);
        const int64_t v = idx / C;
        const int xp = (int)(v % gin.W), yp = (int)((v / gin.W) % gin.H), tp = (int)(v / ((int64_t)gin.W * gin.H));
        float s = 0.f;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int d = 0; d < 2; ++d) {
                    const int t = 2 * tp + a, y = 2 * yp + b, x = 2 * xp + d;
                    if (t < gout.T && y < gout.H && x < gout.W)
                        s += (float)gout.p[(((int64_t)t * gout.H + y) * gout.W + x) * gout.cs + gout.c0 + c];
                }
        if (!((float)act.p[v * act.cs + act.c0 + c] > 0.f)) s = 0.f;
        gin.p[v * gin.cs + gin.c0 + c] = (__bf16)s;
    }
}

// ---------------------------------------------------------------------------
// Head (1x1x1 conv, softplus), loss and their gradients
// ---------------------------------------------------------------------------
// z[v] = sum_c wh[c] d1[v][c] + bh;  xh[v] = softplus(z[v]).
__global__ void head_fwd(View d1, const float* __restrict__ wh, float* __restrict__ z,
                         float* __restrict__ xh) {
    const int64_t n = (int64_t)d1.T * d1.H * d1.W;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        float s = wh[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) s = fmaf(wh[c], (float)d1.p[v * d1.cs + d1.c0 + c], s);
        z[v] = s;
        xh[v] = softplus(s);
    }
}

// Block partials (FP64) of sum(xh t), sum(xh^2), sum(t^2): part[3 block + k].
__global__ void loss_sums(const float* __restrict__ xh, const float* __restrict__ tg, int64_t n,
                          double* __restrict__ part) {
    __shared__ double sm[3][256];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const double x = xh[v], t = tg[v];
        a += x * t;
        b += x * x;
        c += t * t;
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

// Gradient through loss, softplus and head.  dL/dxh is gext[v] when gext is
// given, else that of the cosine loss with coef = (1 / (|xh| |t|), cos / |xh|^2):
//   dL/dxh = -(t coef0 - xh coef1);  gz = dL/dxh * sigmoid(z);
//   g_d1[v][c] = gz wh[c] (d1 > 0);  head partials (FP64): sum gz d1[c], sum gz
//   in hp[block * 17 + c].
__global__ void head_bwd(View d1, const float* __restrict__ wh, const float* __restrict__ z,
                         const float* __restrict__ xh, const float* __restrict__ tg,
                         const float* __restrict__ gext, double coef0, double coef1, View gd1,
                         double* __restrict__ hp) {
    __shared__ double sm[17][256];
    double acc[17];
#pragma unroll
    for (int c = 0; c < 17; ++c) acc[c] = 0.0;
    const int64_t n = (int64_t)d1.T * d1.H * d1.W;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const float gx = gext ? gext[v] : (float)(-(tg[v] * coef0 - xh[v] * coef1));
        const float gz = gx / (1.f + expf(-z[v]));
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const float a = (float)d1.p[v * d1.cs + d1.c0 + c];
            acc[c] += (double)gz * (double)a;
            gd1.p[v * gd1.cs + gd1.c0 + c] = (__bf16)(a > 0.f ? gz * wh[c] : 0.f);
        }
        acc[16] += (double)gz;
    }
#pragma unroll
    for (int c = 0; c < 17; ++c) sm[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int c = 0; c < 17; ++c) sm[c][threadIdx.x] += sm[c][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 17) hp[17 * blockIdx.x + threadIdx.x] = sm[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Adam (FP32 master weights)
// ---------------------------------------------------------------------------
__global__ void adam_step(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                          float c1, float c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

}  // namespace unet
}  // namespace sfseg

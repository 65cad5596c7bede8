// Fused power-iteration step for gfx950.
//
// One power-iteration step (Eq. (4) then Eq. (8)) is one launch of this
// kernel.  The adjacency of Eq. (2) is applied through its three-filter form
// (Eq. (7), multiplied out by alpha so that alpha = 0 needs no special case):
//
//     u = w * x,   A = G * u,   B = G * (F^2 u),   C = G * (F u)
//     y = w * [ A - alpha * (F * (F * A - 2 C) + B) ]
//
// with G the separable box-truncated Gaussian of Eq. (1) (Sec. 4.2: a 3D
// filter is three 1D filters) and zero padding at the volume faces, which is
// what makes the filtering equal the symmetric matrix M.
//
// Memory layout.  Every volume the kernel touches is stored zero-padded: each
// frame is Hp x Wp with the H x W picture at row PT = r_s, column PL (a
// multiple of 4 >= r_s), so that a tile's halo never leaves the frame and
// needs no bounds test.  Outputs that fall in the padding are exactly zero
// (w = 0 there), so they are stored and summed like any other.
//
// Work layout.  A block owns one 64 x 16 pixel tile over a run of frames (one
// work item).  Items are ordered chunk by chunk and, inside a chunk, tile row
// by tile row; blocks are dealt to the 8 XCDs round-robin, so the block index
// is remapped to give each XCD a contiguous run of items: neighbouring tiles
// then stream the same frames at the same time on the same L2, and the halo
// each one loads is the neighbour's interior, already cached.
//
// Per input frame a block loads the tile plus an r_s halo straight into LDS
// (16-byte direct-to-LDS buffer loads, one frame ahead), forms the three
// fields in registers from column strips of it, filters them along y into LDS
// and along x back into registers, and pushes the result into a register ring
// of 2 r_t + 1 frames; once the ring holds frames t - r_t .. t + r_t it filters
// along t, combines, stores frame t and accumulates sum(y^2) and sum(y * Y_k)
// in float64 on the stored values.  The
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

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufferFlags = 0x00020000;  // raw (untyped) buffer, 32-bit lanes

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             kBufferFlags);
}

// 16 bytes per lane from a buffer straight into LDS (buffer_load_dwordx4 ...
// lds): lane i's bytes land at dst + 16 i, dst being the same LDS address in
// every lane of the wave.  The data never passes through registers.
__device__ __forceinline__ void load_lds16(__amdgpu_buffer_rsrc_t rsrc, void* dst, int voff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void*)dst,
                                             16, voff, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Storage precisions: float32, bfloat16, float16.  Values are widened to
// float32 on load; float32 results are rounded to nearest-even on store.
// ---------------------------------------------------------------------------
// N (2 or 4) consecutive 16-bit values: loads of 2N bytes; stores take values
// already rounded to the storage type.
#define SFSEG_HALF_VECTOR_IO                                                                  \
    template <int N>                                                                          \
    static __device__ __forceinline__ void bloadn(__amdgpu_buffer_rsrc_t r, int off, float* v) { \
        if constexpr (N == 4) {                                                               \
            const u32x2 d = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);               \
            v[0] = widen(d.x & 0xffffu); v[1] = widen(d.x >> 16);                             \
            v[2] = widen(d.y & 0xffffu); v[3] = widen(d.y >> 16);                             \
        } else {                                                                              \
            const uint32_t d = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);            \
            v[0] = widen(d & 0xffffu); v[1] = widen(d >> 16);                                 \
        }                                                                                     \
    }                                                                                         \
    template <int N>                                                                          \
    static __device__ __forceinline__ void bstoren(__amdgpu_buffer_rsrc_t r, int off,         \
                                                   const float* v) {                          \
        if constexpr (N == 4) {                                                               \
            u32x2 d = {bits(v[0]) | (bits(v[1]) << 16), bits(v[2]) | (bits(v[3]) << 16)};     \
            __builtin_amdgcn_raw_buffer_store_b64(d, r, off, 0, 0);                           \
        } else {                                                                              \
            __builtin_amdgcn_raw_buffer_store_b32(bits(v[0]) | (bits(v[1]) << 16), r, off, 0, 0); \
        }                                                                                     \
    }

template <typename TS>
struct Stor;
template <>
struct Stor<float> {
    static __device__ __forceinline__ float ld(const float* p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ float rnd(float v) { return v; }
    static __device__ __forceinline__ void st(float* p, int64_t i, float v) { p[i] = v; }
    static __device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int off) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    // voffset (per lane) + soffset (uniform) addressing
    static __device__ __forceinline__ float bload_s(__amdgpu_buffer_rsrc_t r, int off, int soff) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
    }
    // N (2 or 4) consecutive values; off is 4N-byte aligned.
    template <int N>
    static __device__ __forceinline__ void bloadn(__amdgpu_buffer_rsrc_t r, int off, float* v) {
        if constexpr (N == 4) {
            const u32x4 d = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
            v[0] = __uint_as_float(d.x); v[1] = __uint_as_float(d.y);
            v[2] = __uint_as_float(d.z); v[3] = __uint_as_float(d.w);
        } else {
            const u32x2 d = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
            v[0] = __uint_as_float(d.x); v[1] = __uint_as_float(d.y);
        }
    }
    template <int N>
    static __device__ __forceinline__ void bstoren(__amdgpu_buffer_rsrc_t r, int off,
                                                   const float* v) {
        if constexpr (N == 4) {
            u32x4 d = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                       __float_as_uint(v[3])};
            __builtin_amdgcn_raw_buffer_store_b128(d, r, off, 0, 0);
        } else {
            u32x2 d = {__float_as_uint(v[0]), __float_as_uint(v[1])};
            __builtin_amdgcn_raw_buffer_store_b64(d, r, off, 0, 0);
        }
    }
};
template <>
struct Stor<__bf16> {
    static __device__ __forceinline__ float ld(const __bf16* p, int64_t i) { return (float)p[i]; }
    static __device__ __forceinline__ float rnd(float v) { return (float)(__bf16)v; }
    static __device__ __forceinline__ void st(__bf16* p, int64_t i, float v) { p[i] = (__bf16)v; }
    static __device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int off) {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        return __uint_as_float((uint32_t)h << 16);
    }
    static __device__ __forceinline__ float bload_s(__amdgpu_buffer_rsrc_t r, int off, int soff) {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0);
        return __uint_as_float((uint32_t)h << 16);
    }
    static __device__ __forceinline__ uint32_t bits(float v) {
        return (uint32_t)__builtin_bit_cast(unsigned short, (__bf16)v);
    }
    static __device__ __forceinline__ float widen(uint32_t h) { return __uint_as_float(h << 16); }
    SFSEG_HALF_VECTOR_IO
};
template <>
struct Stor<_Float16> {
    static __device__ __forceinline__ float ld(const _Float16* p, int64_t i) { return (float)p[i]; }
    static __device__ __forceinline__ float rnd(float v) { return (float)(_Float16)v; }
    static __device__ __forceinline__ void st(_Float16* p, int64_t i, float v) { p[i] = (_Float16)v; }
    static __device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int off) {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        return (float)__builtin_bit_cast(_Float16, h);
    }
    static __device__ __forceinline__ float bload_s(__amdgpu_buffer_rsrc_t r, int off, int soff) {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0);
        return (float)__builtin_bit_cast(_Float16, h);
    }
    static __device__ __forceinline__ uint32_t bits(float v) {
        return (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)v);
    }
    static __device__ __forceinline__ float widen(uint32_t h) {
        return (float)__builtin_bit_cast(_Float16, (unsigned short)h);
    }
    SFSEG_HALF_VECTOR_IO
};

// ---------------------------------------------------------------------------
// Reductions shared by the step and start-vector kernels
// ---------------------------------------------------------------------------
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

// Sum value `first` (0 or 1) of the nblocks partial pairs in a fixed order:
// thread i sums blocks i, i+NT, ...; then a fixed tree over the threads.
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

// Block-wide sums of a and b written to partials[2*slot], partials[2*slot+1];
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

// XCD-aware block order: hardware deals block b to XCD b % 8; give XCD x the
// contiguous logical range [x * G/8, (x+1) * G/8).  G must be a multiple of 8.
__device__ __forceinline__ int xcd_logical_block(int b, int G) {
    return (b & 7) * (G >> 3) + (b >> 3);
}

// ---------------------------------------------------------------------------
// Fused step kernel
// ---------------------------------------------------------------------------
constexpr int TX = TILE_X, TY = TILE_Y;
constexpr int round4(int v) { return (v + 3) / 4 * 4; }

// Block shapes: PX outputs per thread along x (so TX / PX thread columns and
// NT = 16 * TX / PX threads), PY rows per y-pass column strip.
template <int PX_, int PY_>
struct Shape {
    static constexpr int PX = PX_, PY = PY_;
    static constexpr int NSEG = TX / PX;
    static constexpr int NT = NSEG * TY;
    // Minimum waves per SIMD (the second launch-bounds argument): 256-thread
    // blocks at 2 per CU need 2 (<= 256 VGPRs); 512-thread blocks at 2 per CU
    // need 4 (<= 128 VGPRs).
    static constexpr int MINW = NT / 128;
};
using ShapeWide = Shape<4, 8>;    // 256 threads
using ShapeDeep = Shape<2, 4>;    // 512 threads

// Per input frame a block runs two phases, software-pipelined so that the y
// phase of frame t+1 shares a barrier interval with the x phase of frame t:
//   Y: each column strip of the tile-plus-halo (64 + 2 r_s columns, 16 / PY
//      strips per column) loads PY + 2 r_s rows of x, w, F straight from L2
//      (prefetched one frame ahead), forms the fields u, F u, F^2 u in
//      registers and filters them along y into LDS;
//   X: each thread filters a PX-pixel row segment along x (8- or 16-byte LDS
//      reads that cover the 32 banks without conflicts), pushes it into its
//      register ring of 2 r_t + 1 frames and, once frame t - r_t's neighbours
//      are in, filters along t, combines with its own x, w, F (loaded from L2,
//      prefetched), stores and reduces.
template <typename TS, int RS, int RT, typename SH>
struct Geom {
    static constexpr int NT = SH::NT, PX = SH::PX, PY = SH::PY, NSEG = SH::NSEG;
    static constexpr int ES = (int)sizeof(TS);
    static constexpr int RSA = round4(RS);           // halo rounded to 16-byte columns
    static constexpr int IW = TX + 2 * RS;           // y-pass strips: tile columns plus halo
    static constexpr int IH = TY + 2 * RS;           // raw region rows
    static constexpr int IWA = TX + 2 * RSA;         // raw region columns (16-byte aligned)
    static constexpr int CPR = IWA * ES / 16;        // 16-byte chunks per region row
    static constexpr int NCH = IH * CPR;             // chunks per region (one array)
    static constexpr int NDMA = (NCH + NT - 1) / NT; // direct-to-LDS rounds per array
    static constexpr int RAWE = IH * IWA;            // elements per region (one array)
    static constexpr int NYS = TY / PY;              // strips per column
    static constexpr int NYI = IW * NYS;             // y-pass strips per frame
    static constexpr int YW = PY + 2 * RS;           // rows per strip
    static constexpr int XWA = round4(PX + 2 * RS);  // x-pass window, whole 8/16-byte reads
    static constexpr int MP = TX - PX + XWA + (PX == 2 ? 2 : 0);  // y-filtered row pitch
    static constexpr int NR = 2 * RT + 1;            // frames in the register ring
    static_assert(NYI <= NT, "one strip per thread");
    static_assert(TY % PY == 0, "whole strips per tile");
    static_assert(MP % 4 == 0, "aligned rows");
    static_assert((IWA * ES) % 16 == 0, "whole 16-byte chunks per row");
};

// LDS of one block: the raw x, w, F of the tile plus halo for two frames
// (filled by direct-to-LDS loads, one frame ahead) and the y-filtered fields.
template <typename TS, int RS, int RT, typename SH>
struct StepLds {
    using G = Geom<TS, RS, RT, SH>;
    TS raw[2][3][G::RAWE] __attribute__((aligned(16)));
    float mid3[3][TY * G::MP] __attribute__((aligned(16)));
};

// One work item: the 64 x 16 tile at picture origin (tx0, ty0) of one clip,
// output frames [ta, tb).  Accumulates the item's sum(y^2) and sum(y * Y_k)
// into syy, syx (per thread).
//
// Per input frame:  wait for this frame's region (loaded one frame ago) and
// barrier; store the previous frame's outputs; start the next frame's region
// loads straight into LDS (16 bytes per lane, no registers); Y phase: each
// column strip reads its x, w, F from LDS, forms u, F u, F^2 u and filters
// them along y into mid3; barrier; X phase: each thread filters its PX-pixel
// row segment along x, pushes it into the register ring, and once frames
// t - r_t .. t + r_t are in filters along t, combines with its own x, w, F and
// reduces.  Stores are deferred by one frame so that the wait for the region
// loads never waits for a store that was just issued.
template <typename TS, int RS, int RT, typename SH>
__device__ __forceinline__ void run_item(const TS* __restrict__ X, const TS* __restrict__ Wt,
                                         const TS* __restrict__ Fv, TS* __restrict__ Y, int T,
                                         int Wp, int PT, int PL, int64_t frame, int tx0, int ty0,
                                         int ta, int tb, const float* gs,
                                         const float* gt, float alpha,
                                         StepLds<TS, RS, RT, SH>& lds, double& syy, double& syx) {
    using G = Geom<TS, RS, RT, SH>;
    constexpr int NT = G::NT, PX = G::PX, PY = G::PY, NSEG = G::NSEG, NYI = G::NYI,
                  IW = G::IW, YW = G::YW, XWA = G::XWA, MP = G::MP, NR = G::NR, RSA = G::RSA,
                  IWA = G::IWA, CPR = G::CPR, NCH = G::NCH, NDMA = G::NDMA, RAWE = G::RAWE;
    constexpr int ES = (int)sizeof(TS);
    if (tb <= ta) return;
    const uint32_t frame_bytes = (uint32_t)(frame * ES);
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int orow = tid / NSEG;         // output row inside the tile
    const int ocol = (tid % NSEG) * PX;  // first output column inside the tile

    // Direct-to-LDS chunks of this thread: chunk c = r * NT + tid covers
    // region row c / CPR, 16 bytes at column (c % CPR) * 16 / ES.  The region
    // starts at padded row ty0 (PT = r_s) and column tx0 + PL - RSA = tx0.
    int doff[NDMA];
#pragma unroll
    for (int r = 0; r < NDMA; ++r) {
        const int cidx = r * NT + tid;
        const int row = cidx / CPR, cq = cidx - (cidx / CPR) * CPR;
        doff[r] = ((ty0 + row) * Wp + (tx0 + PL - RSA) + cq * (16 / ES)) * ES;
    }
    auto rsrc = [&](const TS* base, int t) {
        const bool tin = t >= 0 && t < T;
        return make_rsrc(base + (tin ? (int64_t)t * frame : 0), tin ? frame_bytes : 0u);
    };
    // Region of frame t into raw[buf]; frames outside the clip are zeros.
    auto load_region = [&](int t, int buf) {
        if (t >= 0 && t < T) {
            const TS* src[3] = {X, Wt, Fv};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const __amdgpu_buffer_rsrc_t rr = rsrc(src[a], t);
#pragma unroll
                for (int r = 0; r < NDMA; ++r) {
                    if (r * NT + tid < NCH) {
                        TS* dst = &lds.raw[buf][a][(r * NT + wave * 64) * (16 / ES)];
                        load_lds16(rr, dst, doff[r]);
                    }
                }
            }
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                for (int e = tid; e < RAWE; e += NT) lds.raw[buf][a][e] = (TS)0.f;
        }
    };

    // This thread's y-pass strip: region column ycol + RSA - RS, rows yseg*PY .. +YW.
    const bool yact = tid < NYI;
    const int ycol = yact ? tid % IW : 0;
    const int yseg = yact ? tid / IW : 0;
    const int ybase = (yseg * PY) * IWA + ycol + (RSA - RS);
    const int ooff = ((ty0 + PT + orow) * Wp + (tx0 + PL + ocol)) * ES;

    float qX[PX], qW[PX], qF[PX];  // own x, w, F of the output frame
    auto load_own = [&](int t) {
        const __amdgpu_buffer_rsrc_t rx = rsrc(X, t), rw = rsrc(Wt, t), rf = rsrc(Fv, t);
        Stor<TS>::template bloadn<PX>(rx, ooff, qX);
        Stor<TS>::template bloadn<PX>(rw, ooff, qW);
        Stor<TS>::template bloadn<PX>(rf, ooff, qF);
    };

    float ring[NR][3][PX];  // x/y-filtered fields of the last NR frames
#pragma unroll
    for (int j = 0; j < NR; ++j)
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int i = 0; i < PX; ++i) ring[j][f][i] = 0.f;
    float yv[PX];          // outputs waiting to be stored
    int pending_t = -1;    // their frame (-1: none)

    // Input frames ta-RT .. tb+RT-1, rounded up to whole ring turns; the
    // extra steps read frames past the run and store nothing.
    const int n_in = (tb - ta) + 2 * RT;
    const int n_steps = (n_in + NR - 1) / NR * NR;
    load_region(ta - RT, 0);

    for (int s0 = 0; s0 < n_steps; s0 += NR) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const int s = s0 + j;
            const int t_in = ta - RT + s;
            const int cur = s & 1;
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();  // raw[cur] is complete; mid3 and raw[cur ^ 1] are free
            if (pending_t >= 0) {
                const __amdgpu_buffer_rsrc_t ry = make_rsrc(Y + (int64_t)pending_t * frame, frame_bytes);
                Stor<TS>::template bstoren<PX>(ry, ooff, yv);
                pending_t = -1;
            }
            const int t_out = t_in - RT;
            const bool emit = t_out >= ta && t_out < tb;
            if (emit) load_own(t_out);
            load_region(t_in + 1, cur ^ 1);
            // ---- Y phase: fields and filter along y ----
            if (yact) {
                const TS* rx = &lds.raw[cur][0][ybase];
                const TS* rw = &lds.raw[cur][1][ybase];
                const TS* rf = &lds.raw[cur][2][ybase];
                float fu[YW], fv[YW], fz[YW];
#pragma unroll
                for (int k = 0; k < YW; ++k) {
                    const float xv = (float)rx[k * IWA], wv = (float)rw[k * IWA],
                                fvv = (float)rf[k * IWA];
                    fu[k] = wv * xv;
                    fv[k] = fvv * fu[k];
                    fz[k] = fvv * fv[k];
                }
#pragma unroll
                for (int i = 0; i < PY; ++i) {
                    float a0 = gs[0] * fu[i + RS], a1 = gs[0] * fv[i + RS], a2 = gs[0] * fz[i + RS];
#pragma unroll
                    for (int d = 1; d <= RS; ++d) {
                        a0 = fmaf(gs[d], fu[i + RS - d] + fu[i + RS + d], a0);
                        a1 = fmaf(gs[d], fv[i + RS - d] + fv[i + RS + d], a1);
                        a2 = fmaf(gs[d], fz[i + RS - d] + fz[i + RS + d], a2);
                    }
                    const int o = (yseg * PY + i) * MP + ycol;
                    lds.mid3[0][o] = a0;
                    lds.mid3[1][o] = a1;
                    lds.mid3[2][o] = a2;
                }
            }
            __syncthreads();  // mid3 is complete
            // ---- X phase: filter along x into ring slot j ----
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                float win[XWA];
                const float* src = &lds.mid3[f][orow * MP + ocol];
                if constexpr (PX % 4 == 0) {
#pragma unroll
                    for (int q = 0; q < XWA / 4; ++q) {
                        const float4 v4 = reinterpret_cast<const float4*>(src)[q];
                        win[4 * q + 0] = v4.x;
                        win[4 * q + 1] = v4.y;
                        win[4 * q + 2] = v4.z;
                        win[4 * q + 3] = v4.w;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < XWA / 2; ++q) {
                        const float2 v2 = reinterpret_cast<const float2*>(src)[q];
                        win[2 * q + 0] = v2.x;
                        win[2 * q + 1] = v2.y;
                    }
                }
#pragma unroll
                for (int i = 0; i < PX; ++i) {
                    float a = gs[0] * win[i + RS];
#pragma unroll
                    for (int d = 1; d <= RS; ++d)
                        a = fmaf(gs[d], win[i + RS - d] + win[i + RS + d], a);
                    ring[j][f][i] = a;
                }
            }
            // ---- filter along t, combine (Eq. (7)), reduce frame t_out ----
            if (emit) {
#pragma unroll
                for (int i = 0; i < PX; ++i) {
                    float A = 0.f, B = 0.f, C = 0.f;
#pragma unroll
                    for (int m = 0; m < NR; ++m) {
                        const int slot = (j + 1 + m) % NR;  // constant once unrolled
                        A = fmaf(gt[m], ring[slot][0][i], A);  // G * u
                        C = fmaf(gt[m], ring[slot][1][i], C);  // G * (F u)
                        B = fmaf(gt[m], ring[slot][2][i], B);  // G * (F^2 u)
                    }
                    const float E = fmaf(-alpha, fmaf(qF[i], fmaf(qF[i], A, -2.f * C), B), A);
                    const float yq = Stor<TS>::rnd(qW[i] * E);
                    yv[i] = yq;
                    syy = fma((double)yq, (double)yq, syy);
                    syx = fma((double)yq, (double)qX[i], syx);
                }
                pending_t = t_out;
            }
        }
    }
    if (pending_t >= 0) {
        const __amdgpu_buffer_rsrc_t ry = make_rsrc(Y + (int64_t)pending_t * frame, frame_bytes);
        Stor<TS>::template bstoren<PX>(ry, ooff, yv);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();  // the last region loads have landed before LDS is reused
}

template <typename TS, int RS, int RT, typename SH>
__global__ __launch_bounds__(SH::NT, SH::MINW) void step_kernel(StepParams p) {
    using G = Geom<TS, RS, RT, SH>;
    constexpr int NT = G::NT, NR = G::NR;
    __shared__ StepLds<TS, RS, RT, SH> lds;
    __shared__ double fin[NT];

    DevState* st = p.st;
    if (st->done) return;

    const float c = st->c;
    float gs[RS + 1];
#pragma unroll
    for (int d = 0; d <= RS; ++d) gs[d] = p.gs[d];
    float gt[NR];
#pragma unroll
    for (int m = 0; m < NR; ++m) gt[m] = p.gt[m < RT ? RT - m : m - RT] * c;

    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int4 item = p.items[lb];  // tile origin (picture coords) and frame range
    double syy = 0.0, syx = 0.0;
    run_item<TS, RS, RT, SH>((const TS*)p.x, (const TS*)p.w, (const TS*)p.f, (TS*)p.y, p.T, p.Wp,
                             p.PT, p.PL, p.frame, item.x, item.y, item.z, item.w, gs, gt, p.alpha,
                             lds, syy, syx);

    if (block_partials_and_ticket<NT>(syy, syx, p.partials, lb, &st->ticket, (uint32_t)gridDim.x)) {
        const double tyy = fixed_order_sum<NT>(p.partials, gridDim.x, 0, fin);
        const double tyx = fixed_order_sum<NT>(p.partials, gridDim.x, 1, fin);
        if (threadIdx.x == 0) {
            advance_state(st, tyy, tyx);
            __hip_atomic_store(&st->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// Batched persistent step: many clips, one launch
// ---------------------------------------------------------------------------
// Work items of all clips that are still iterating are handed out through 8
// queues, one per XCD: queue x holds a contiguous run of items (neighbouring
// tiles of one clip, so their halos meet in that XCD's L2).  A block drains
// the queue of its own XCD first, then takes leftovers from the others.  Each
// item writes its partial sums to its own slot; the last item of a clip to
// finish reduces that clip's slots in a fixed order and advances only that
// clip's state, so a converged clip drops out of the next launch.
template <typename TS, int RS, int RT, typename SH>
__global__ __launch_bounds__(SH::NT, SH::MINW) void batch_step_kernel(BatchParams p) {
    using G = Geom<TS, RS, RT, SH>;
    constexpr int NT = G::NT, NR = G::NR;
    __shared__ StepLds<TS, RS, RT, SH> lds;
    __shared__ double fin[NT];
    __shared__ int s_item;

    float gs[RS + 1];
#pragma unroll
    for (int d = 0; d <= RS; ++d) gs[d] = p.gs[d];
    const int home = blockIdx.x & 7;
    int q = home;  // queue being drained
    int tried = 0;

    for (;;) {
        if (threadIdx.x == 0) {
            int it = -1;
            while (tried < 8) {
                const uint32_t k = atomicAdd(&p.queue[q], 1u);
                if ((int)k < p.qcount[q]) {
                    it = p.qfirst[q] + (int)k;
                    break;
                }
                q = (q + 1) & 7;
                ++tried;
            }
            s_item = it;
        }
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it < 0) break;

        const int4 item = p.items[it];  // clip, x0 | y0 << 16, t0, t1
        const BatchClip* cl = p.clips + item.x;
        DevState* st = cl->st;
        if (st->done) continue;  // converged or stopped: nothing to do for this clip

        const float c = st->c;
        float gt[NR];
#pragma unroll
        for (int m = 0; m < NR; ++m) gt[m] = p.gt[m < RT ? RT - m : m - RT] * c;
        double syy = 0.0, syx = 0.0;
        run_item<TS, RS, RT, SH>((const TS*)cl->buf[p.parity], (const TS*)cl->w,
                                 (const TS*)cl->f, (TS*)cl->buf[1 - p.parity], cl->T, cl->Wp,
                                 cl->PT, cl->PL, cl->frame, item.y & 0xffff, item.y >> 16, item.z,
                                 item.w, gs, gt, p.alpha, lds, syy, syx);
        if (block_partials_and_ticket<NT>(syy, syx, p.partials, it, &st->ticket,
                                          (uint32_t)cl->n_items)) {
            const double* part = p.partials + 2 * cl->first_item;
            const double tyy = fixed_order_sum<NT>(part, cl->n_items, 0, fin);
            const double tyx = fixed_order_sum<NT>(part, cl->n_items, 1, fin);
            if (threadIdx.x == 0) {
                advance_state(st, tyy, tyx);
                __hip_atomic_store(&st->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    // The last block to leave resets the queues for the next launch.
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&p.queue[8], 1u) == gridDim.x - 1) {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                __hip_atomic_store(&p.queue[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <typename TS, int RS, int RT, typename SH>
hipError_t launch_batch_t(const BatchParams& p, int grid, hipStream_t s) {
    hipLaunchKernelGGL((batch_step_kernel<TS, RS, RT, SH>), dim3(grid), dim3(SH::NT), 0, s, p);
    return hipGetLastError();
}
template <typename TS, int RS, int RT, typename SH>
hipError_t occ_batch_t(int* blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, batch_step_kernel<TS, RS, RT, SH>,
                                                        SH::NT, 0);
}

// Launch / occupancy tables over (shape, r_s, r_t) for one storage type.
template <typename TS, int RS, int RT, typename SH>
hipError_t launch_step_t(const StepParams& p, int grid, hipStream_t s) {
    hipLaunchKernelGGL((step_kernel<TS, RS, RT, SH>), dim3(grid), dim3(SH::NT), 0, s, p);
    return hipGetLastError();
}
template <typename TS, int RS, int RT, typename SH>
hipError_t occ_step_t(int* blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, step_kernel<TS, RS, RT, SH>,
                                                        SH::NT, 0);
}

using LaunchFn = hipError_t (*)(const StepParams&, int, hipStream_t);
using BatchFn = hipError_t (*)(const BatchParams&, int, hipStream_t);
using OccFn = hipError_t (*)(int*);
constexpr int NSHAPES = 2;  // 0: ShapeWide (256 threads), 1: ShapeDeep (512 threads)
constexpr int NCOMB = (SFSEG_MAX_RS + 1) * (SFSEG_MAX_RT + 1);

struct StepFns {
    LaunchFn launch;
    OccFn occ;
    BatchFn batch;
    OccFn batch_occ;
};

template <typename TS, typename SH, int RS, int... RTs>
void fill_rt(StepFns* t, std::integer_sequence<int, RTs...>) {
    ((t[RS * (SFSEG_MAX_RT + 1) + RTs] =
          StepFns{&launch_step_t<TS, RS, RTs, SH>, &occ_step_t<TS, RS, RTs, SH>,
                  &launch_batch_t<TS, RS, RTs, SH>, &occ_batch_t<TS, RS, RTs, SH>}),
     ...);
}
template <typename TS, typename SH, int... RSs>
void fill_rs(StepFns* t, std::integer_sequence<int, RSs...>) {
    (fill_rt<TS, SH, RSs>(t, std::make_integer_sequence<int, SFSEG_MAX_RT + 1>{}), ...);
}

template <typename TS>
struct StepTable {
    StepFns fns[NSHAPES][NCOMB];
    StepTable() {
        fill_rs<TS, ShapeWide>(fns[0], std::make_integer_sequence<int, SFSEG_MAX_RS + 1>{});
        fill_rs<TS, ShapeDeep>(fns[1], std::make_integer_sequence<int, SFSEG_MAX_RS + 1>{});
    }
};

}  // namespace detail
}  // namespace sfseg

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
// work item).  Items are ordered run by run and, inside a run, tile row by
// tile row; blocks are dealt to the 8 XCDs round-robin, so the block index is
// remapped to give each XCD a contiguous range of items: neighbouring tiles
// then stream the same frames at about the same time on the same L2, and the
// halo each one loads is mostly the neighbour's interior, already cached.
//
// Per input frame a block loads the tile plus an r_s halo straight into LDS
// (16-byte direct-to-LDS buffer loads, one frame ahead), forms the three
// fields in registers from column strips of it, filters them along y into LDS
// and along x back into registers, and pushes the result into a register ring
// of 2 r_t + 1 frames; once the ring holds frames t - r_t .. t + r_t it filters
// along t, combines, stores frame t and accumulates sum(y^2) and sum(y * Y_k)
// in float64 on the stored values.  The block's partial sums go to memory.
// The next launch's blocks each add all of them in a fixed order and advance
// the iteration state (norm, Rayleigh quotient, change, convergence flag) in
// registers -- identical bits in every block -- before they start, so
// results are bit-reproducible and no block ever waits on another: a
// last-block ticket would need an agent-scope release fence in every block,
// which on this multi-XCD part writes back the XCD's L2 each time.
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
    // The float32 value is rounded: the empty asm keeps the compiler from
    // fusing the product that produced v with this rounding (one rounding
    // of the exact product instead of two), which it does or not depending
    // on the surrounding code.
    static __device__ __forceinline__ float rnd(float v) {
        asm volatile("" : "+v"(v));
        return (float)(_Float16)v;
    }
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

// Advance the iteration state after a step.
//   syy = sum(y_i^2), syx = sum(y_i * Y_k,i) over the stored values, where
//   y = c * M Y_k and x_k = s * Y_k.  Then
//   M x_k = (s / c) y            =>  lambda = x_k^T M x_k = s^2 syx / c
//   x_{k+1} = y / ||y||          =>  x_{k+1} . x_k = s syx / ||y||
//   delta = ||x_{k+1} - x_k|| = sqrt(2 - 2 x_{k+1} . x_k)   (both unit vectors)
__device__ inline void advance_values(DevState& st, double syy, double syx) {
    const double n = sqrt(syy);
    const double s = st.s;
    const double c = (double)st.c;
    st.k += 1;
    if (!isfinite(n) || !isfinite(syx)) {
        st.status = SFSEG_ERR_NONFINITE;
        st.done = 1;
        return;
    }
    if (!(n > 0.0)) {
        st.status = SFSEG_ERR_ZERO_NORM;
        st.done = 1;
        return;
    }
    st.lambda = s * s * syx / c;
    const double cosv = s * syx / n;
    st.delta = sqrt(fmax(0.0, 2.0 - 2.0 * cosv));
    st.s = 1.0 / n;
    st.c = (float)(st.s * st.gain);
    if (st.delta < st.tol) {
        st.converged = 1;
        st.done = 1;
    }
    if (st.k >= st.max_iters) st.done = 1;
}

// The same on a state in memory (one thread of a finish launch).
__device__ inline void advance_state(DevState* st, double syy, double syx) {
    advance_values(*st, syy, syx);
}

// Block-wide sums of a and b (each wave in a fixed butterfly, then the waves
// in order) written to part[2*slot], part[2*slot+1].
template <int NT>
__device__ void block_partials(double a, double b, double* part, int slot) {
    __shared__ double red[2][NT / 64];
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
        agent_store(part + 2 * slot, sa);
        agent_store(part + 2 * slot + 1, sb);
    }
}

// Fixed-order sums of the nblocks partial pairs of a step launch, the same
// bits in every block of any size >= 256: lanes 0..255 add blocks i, i + 256,
// ... in turn, each of the first four waves reduces its lanes, and the four
// wave sums are added in order.  Every thread gets both sums.
template <int NT>
__device__ void fold_partials(const double* part, int nblocks, double (*red)[4], double& a,
                              double& b) {
    static_assert(NT >= 256, "the fold needs four full waves");
    double sa = 0.0, sb = 0.0;
    if (threadIdx.x < 256) {
        for (int i = threadIdx.x; i < nblocks; i += 256) {
            sa += agent_load(part + 2 * i);
            sb += agent_load(part + 2 * i + 1);
        }
    }
    sa = wave_sum(sa);
    sb = wave_sum(sb);
    if (threadIdx.x < 256 && (threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sa;
        red[1][threadIdx.x >> 6] = sb;
    }
    __syncthreads();
    a = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    b = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    __syncthreads();
}

// The state of a step launch's input: the slot as written, with the partial
// sums of the launch that wrote the input folded in if they are pending.  A
// launch of two fused steps (pending = 2) leaves a second set of sums after
// the first (part + 2 nblocks); both of its steps used the multiplier c of
// its own input, so the second advance starts from that c again.  The pair
// is always taken whole: if the first step already met the tolerance, the
// state still ends at the second, which is the iterate in the buffer.
template <int NT>
__device__ DevState state_of_input(const DevState* slot, const double* part, int nblocks,
                                   double (*red)[4]) {
    DevState s = *slot;
    if (s.pending) {
        const int np = s.pending;
        const float c_used = s.c;
        double syy, syx;
        fold_partials<NT>(part, nblocks, red, syy, syx);
        s.pending = 0;
        advance_values(s, syy, syx);
        if (np == 2 && s.status == SFSEG_OK) {
            const int conv = s.converged;
            fold_partials<NT>(part + 2 * nblocks, nblocks, red, syy, syx);
            s.c = c_used;
            s.done = 0;
            advance_values(s, syy, syx);
            if (conv) {
                s.converged = 1;
                s.done = 1;
            }
        }
    }
    return s;
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

// Block shapes: PX outputs per thread along x, so TX / PX thread columns and
// NT = 16 * TX / PX threads; NF pairwise feature channels (Sec. 3.3): the
// filter then carries 1 + 2 NF fields, u and F_c u, F_c^2 u per channel.
template <int PX_, int NF_ = 1>
struct Shape {
    static constexpr int PX = PX_;
    static constexpr int NF = NF_;
    static constexpr int NSEG = TX / PX;
    static constexpr int NT = NSEG * TY;
    static constexpr int NWAVES = NT / 64;
};
using ShapeWide = Shape<4>;  // 256 threads
using ShapeDeep = Shape<2>;  // 512 threads
using ShapeWide2 = Shape<4, 2>;
using ShapeDeep2 = Shape<2, 2>;

// Per input frame a block runs two phases separated by a barrier:
//   Y: the y pass over the tile plus its x halo (64 + 2 r_s columns).  Every
//      column is cut into NS row segments of PY rows (the last one shifted up
//      to end at row 16), one segment per lane: waves 0 .. NS-1 take columns
//      0..63 of segment 0 .. NS-1, wave NS takes the 2 r_s halo columns of
//      all segments, so every SIMD gets an equal share.  A lane walks the
//      PY + 2 r_s region rows of its column once, forms u, F u, F^2 u from the
//      raw x, w, F in LDS and accumulates each into the PY outputs it touches.
//   X: each thread filters its PX-pixel row segment along x from 16-byte LDS
//      reads, pushes it into its register ring of 2 r_t + 1 frames and, once
//      frame t - r_t's neighbours are in, filters along t, combines with its
//      own x, w, F, rounds to the storage type and reduces.
// The raw region of the next frame is loaded straight into LDS while the X
// phase runs: the Y phase is its only reader and has finished.
constexpr int kLdsThreeBlocks = 53 * 1024;  // three blocks share a CU's 160 KB
template <typename TS, int RS, int RT, typename SH>
struct Geom {
    static constexpr int NT = SH::NT, PX = SH::PX, NSEG = SH::NSEG, NWAVES = SH::NWAVES;
    static constexpr int NF = SH::NF;                // pairwise feature channels
    static constexpr int NFLD = 1 + 2 * NF;          // filtered fields
    static constexpr int NARR = 2 + NF;              // arrays read: x, w, F_1..F_NF
    static constexpr int ES = (int)sizeof(TS);
    static constexpr int RSA = round4(RS);           // halo rounded to 16-byte columns
    static constexpr int IW = TX + 2 * RS;           // y-pass columns: tile plus halo
    static constexpr int IH = TY + 2 * RS;           // raw region rows
    static constexpr int IWA = TX + 2 * RSA;         // raw region columns (16-byte aligned)
    static constexpr int CPR = IWA * ES / 16;        // 16-byte chunks per region row
    static constexpr int NCH = IH * CPR;             // chunks per region (one array)
    static constexpr int NDMA = (NCH + NT - 1) / NT; // direct-to-LDS rounds per array
    static constexpr int RAWE = IH * IWA;            // elements per region (one array)
    static constexpr int EXT = IW - TX;              // halo columns (taken by wave NS)
    static constexpr int NS_W = NWAVES - 1;          // segments the waves allow
    static constexpr int NS_E = EXT > 0 ? 64 / EXT : TY;  // segments the halo wave can hold
    static constexpr int NS = NS_W < NS_E ? (NS_W < TY ? NS_W : TY) : (NS_E < TY ? NS_E : TY);
    static constexpr int PY = (TY + NS - 1) / NS;    // rows per segment
    static constexpr int YW = PY + 2 * RS;           // region rows a segment reads
    static constexpr int XWA = round4(PX + 2 * RS);  // x-pass window, whole 8/16-byte reads
    static constexpr int MP = TX - PX + XWA + (PX == 2 ? 2 : 0);  // y-filtered row pitch
    static constexpr int NR = 2 * RT + 1;            // frames in the register ring
    // The tile's own x, w, F of the last r_t + 1 frames (taken from the
    // region while it is in LDS) ride in a register shift ring.
    static constexpr int RT1 = RT + 1;                // frames in the own-value ring
    static constexpr int LDS_BASE = NARR * RAWE * ES + NFLD * TY * MP * 4;
    // Waves per SIMD the register budget is set for (the second launch-bounds
    // argument): three when three blocks fit the LDS and the register ring is
    // small enough; otherwise two (two blocks share a CU).
    static constexpr int RING = NR * NFLD * PX;
    static constexpr int MINW = LDS_BASE <= kLdsThreeBlocks && RING <= 84 ? 3 : 2;
    static_assert(NS >= 1 && NS * EXT <= 64 && NS + 1 <= NWAVES, "y-pass lane mapping");
    static_assert(NS * PY >= TY && PY <= TY, "segments cover the tile rows");
    static_assert(MP % 4 == 0, "aligned rows");
    static_assert((IWA * ES) % 16 == 0, "whole 16-byte chunks per row");
};

// LDS of one block: the raw x, w, F of the tile plus halo for one frame
// (filled by direct-to-LDS loads) and the y-filtered fields.
template <typename TS, int RS, int RT, typename SH>
struct StepLds {
    using G = Geom<TS, RS, RT, SH>;
    TS raw[G::NARR][G::RAWE] __attribute__((aligned(16)));
    float mid3[G::NFLD][TY * G::MP] __attribute__((aligned(16)));
};

// One work item: the 64 x 16 tile at picture origin (tx0, ty0) of one clip,
// output frames [ta, tb).  Accumulates the item's sum(y^2) and sum(y * Y_k)
// into syy, syx (per thread).
//
// Per input frame t:  wait for frame t's region and barrier; store frame
// t - r_t - 1's outputs (deferred by one frame, so that the wait above never
// waits for a store just issued); keep the tile's own x, w, F of frame t in
// the own ring; Y phase; barrier; X phase, with the region loads of frame
// t + 1 (16 bytes per lane straight into LDS) issued one array per field; t
// filter, combine with the own x, w, F of frame t - r_t, and reduce.  A frame
// outside the clip skips the Y and X phases and clears its ring slot.
template <typename TS, int RS, int RT, typename SH>
__device__ __forceinline__ void run_item(const TS* __restrict__ X, const TS* __restrict__ Wt,
                                         const TS* __restrict__ Fv, int64_t fstride,
                                         TS* __restrict__ Y, int T, int Wp, int PT, int PL,
                                         int64_t frame, int tx0, int ty0, int ta, int tb,
                                         const float* gs, const float* gt, float alpha,
                                         StepLds<TS, RS, RT, SH>& lds, double& syy,
                                         double& syx) {
    using G = Geom<TS, RS, RT, SH>;
    constexpr int NT = G::NT, PX = G::PX, NSEG = G::NSEG, IW = G::IW, EXT = G::EXT,
                  NS = G::NS, PY = G::PY, YW = G::YW, XWA = G::XWA, MP = G::MP, NR = G::NR,
                  RSA = G::RSA, IWA = G::IWA, CPR = G::CPR, NCH = G::NCH, NDMA = G::NDMA,
                  RAWE = G::RAWE, NF = G::NF, NFLD = G::NFLD, NARR = G::NARR;
    constexpr int ES = (int)sizeof(TS);
    if (tb <= ta) return;
    const uint32_t frame_bytes = (uint32_t)(frame * ES);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar branches
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
    // Array a (x, w or F) of the region of frame t into raw.  Frames outside
    // the clip are zeros: nothing reads raw for them (their steps skip the y
    // and x passes), so nothing is loaded.
    auto load_region_array = [&](int t, int a) {
        if (t >= 0 && t < T) {
            const __amdgpu_buffer_rsrc_t rr =
                rsrc(a == 0 ? X : (a == 1 ? Wt : Fv + (int64_t)(a - 2) * fstride), t);
#pragma unroll
            for (int r = 0; r < NDMA; ++r) {
                if (r * NT + tid < NCH)
                    load_lds16(rr, &lds.raw[a][(r * NT + wave * 64) * (16 / ES)], doff[r]);
            }
        }
    };

    // This lane's y-pass column and segment (see Geom).
    bool yact;
    int ycol, yseg;
    if (wave < NS) {
        yact = true;
        ycol = lane;
        yseg = wave;
    } else {
        yact = wave == NS && lane < NS * EXT;
        yseg = yact ? lane / EXT : 0;
        ycol = yact ? TX + (lane - yseg * EXT) : 0;
    }
    const int ys = min(yseg * PY, TY - PY);     // first row of the segment
    const int yskip = yseg * PY - ys;           // leading rows another segment writes
    const int ybase = ys * IWA + ycol + (RSA - RS);
    const int ooff = ((ty0 + PT + orow) * Wp + (tx0 + PL + ocol)) * ES;

    // Own x, w, F of this thread's PX pixels: copied from the region while
    // the frame is in LDS into a register shift ring of r_t + 1 frames
    // (oR[0] is the output frame's).
    const int rown = (orow + RS) * IWA + RSA + ocol;  // own pixels inside the region
    float qX[PX], qW[PX], qF[NF][PX];  // own x, w, F_c of the output frame
    float oR[G::RT1][NARR][PX];  // own x, w, F_c of frames t_in - r_t .. t_in

    float ring[NR][NFLD][PX];  // x/y-filtered fields of the last NR frames
#pragma unroll
    for (int j = 0; j < NR; ++j)
#pragma unroll
        for (int f = 0; f < NFLD; ++f)
#pragma unroll
            for (int i = 0; i < PX; ++i) ring[j][f][i] = 0.f;
    float yv[PX];          // outputs waiting to be stored
    int pending_t = -1;    // their frame (-1: none)

    // Input frames ta-RT .. tb+RT-1.  The loop runs in whole ring turns (the
    // ring slot is then a compile-time index) and leaves the last turn as
    // soon as the run's input frames are done.
    const int n_in = (tb - ta) + 2 * RT;
    const int n_steps = (n_in + NR - 1) / NR * NR;
#pragma unroll
    for (int a = 0; a < NARR; ++a) load_region_array(ta - RT, a);

    for (int s0 = 0; s0 < n_steps; s0 += NR) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (s0 + j >= n_in) break;  // uniform over the block
            const int t_in = ta - RT + s0 + j;
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();  // raw holds frame t_in; mid3 is free
            if (pending_t >= 0) {
                const __amdgpu_buffer_rsrc_t ry = make_rsrc(Y + (int64_t)pending_t * frame, frame_bytes);
                Stor<TS>::template bstoren<PX>(ry, ooff, yv);
                pending_t = -1;
            }
            const int t_out = t_in - RT;
            const bool emit = t_out >= ta && t_out < tb;
            // shift the own-value ring down one frame; frame t_in's own values
            // (needed only if it is an output frame) come from the region
#pragma unroll
            for (int q = 0; q < RT; ++q)
#pragma unroll
                for (int ar = 0; ar < NARR; ++ar)
#pragma unroll
                    for (int i = 0; i < PX; ++i) oR[q][ar][i] = oR[q + 1][ar][i];
            if (t_in >= ta && t_in < tb) {
#pragma unroll
                for (int ar = 0; ar < NARR; ++ar)
#pragma unroll
                    for (int i = 0; i < PX; ++i) oR[RT][ar][i] = (float)lds.raw[ar][rown + i];
            }
            // A frame outside the clip is all zeros, and so are its filtered
            // fields: its ring slot is cleared instead of running the y and x
            // passes (uniform over the block, like every branch around a
            // barrier here).
            const bool zero = t_in < 0 || t_in >= T;
            const bool more = s0 + j + 1 < n_in;  // the run reads frame t_in + 1
            if (!zero) {
                // ---- Y phase: fields, filtered along y, into mid3 ----
                if (yact) {
                    const TS* rx = &lds.raw[0][ybase];
                    const TS* rw = &lds.raw[1][ybase];
                    float acc[NFLD][PY];
#pragma unroll
                    for (int f = 0; f < NFLD; ++f)
#pragma unroll
                        for (int i = 0; i < PY; ++i) acc[f][i] = 0.f;
#pragma unroll
                    for (int k = 0; k < YW; ++k) {
                        // fields: u, then F_c u and F_c^2 u for each channel c
                        float fld[NFLD];
                        fld[0] = (float)rw[k * IWA] * (float)rx[k * IWA];
#pragma unroll
                        for (int c = 0; c < NF; ++c) {
                            const float fv = (float)lds.raw[2 + c][ybase + k * IWA];
                            fld[1 + 2 * c] = fv * fld[0];
                            fld[2 + 2 * c] = fv * fld[1 + 2 * c];
                        }
#pragma unroll
                        for (int i = 0; i < PY; ++i) {
                            const int d = k - i - RS;  // tap offset, constant once unrolled
                            if (d >= -RS && d <= RS) {
                                const float g = gs[d < 0 ? -d : d];
#pragma unroll
                                for (int f = 0; f < NFLD; ++f) acc[f][i] = fmaf(g, fld[f], acc[f][i]);
                            }
                        }
                    }
#pragma unroll
                    for (int i = 0; i < PY; ++i) {
                        if (i >= yskip) {
                            const int o = (ys + i) * MP + ycol;
#pragma unroll
                            for (int f = 0; f < NFLD; ++f) lds.mid3[f][o] = acc[f][i];
                        }
                    }
                }
                __syncthreads();  // mid3 is complete; raw is free
                // ---- X phase: filter along x into ring slot j; the region loads
                // of frame t_in + 1 (if the run reads it) are issued one array per
                // field ----
#pragma unroll
                for (int f = 0; f < NFLD; ++f) {
                    if (f < NARR && more) load_region_array(t_in + 1, f);
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
            } else {
                // raw is free (nothing reads it for this frame): load the next
                // region now
#pragma unroll
                for (int f = 0; f < NARR; ++f)
                    if (more) load_region_array(t_in + 1, f);
#pragma unroll
                for (int f = 0; f < NFLD; ++f)
#pragma unroll
                    for (int i = 0; i < PX; ++i) ring[j][f][i] = 0.f;
            }
            // ---- filter along t, combine (Eq. (7)), reduce frame t_out ----
            if (emit) {
#pragma unroll
                for (int i = 0; i < PX; ++i) {
                    qX[i] = oR[0][0][i];
                    qW[i] = oR[0][1][i];
#pragma unroll
                    for (int c = 0; c < NF; ++c) qF[c][i] = oR[0][2 + c][i];
                }
#pragma unroll
                for (int i = 0; i < PX; ++i) {
                    float tf[NFLD];  // A = G * u, then C_c = G * (F_c u), B_c = G * (F_c^2 u)
#pragma unroll
                    for (int f = 0; f < NFLD; ++f) tf[f] = 0.f;
#pragma unroll
                    for (int m = 0; m < NR; ++m) {
                        const int slot = (j + 1 + m) % NR;  // constant once unrolled
#pragma unroll
                        for (int f = 0; f < NFLD; ++f) tf[f] = fmaf(gt[m], ring[slot][f][i], tf[f]);
                    }
                    const float A = tf[0];
                    float q = 0.f;  // sum_c F_c (F_c A - 2 C_c) + B_c
#pragma unroll
                    for (int c = 0; c < NF; ++c) {
                        const float t_c = fmaf(qF[c][i], fmaf(qF[c][i], A, -2.f * tf[1 + 2 * c]),
                                               tf[2 + 2 * c]);
                        q = c == 0 ? t_c : q + t_c;
                    }
                    const float E = fmaf(-alpha, q, (float)NF * A);
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
__global__ __launch_bounds__(SH::NT, (Geom<TS, RS, RT, SH>::MINW))
void step_kernel(StepParams p) {
    using G = Geom<TS, RS, RT, SH>;
    constexpr int NT = G::NT, NR = G::NR;
    __shared__ StepLds<TS, RS, RT, SH> lds;
    __shared__ double fold_red[2][4];

    // Fold the previous step's partial sums (every block, same bits), record
    // the state for this launch's output, and stop if the iteration has.
    const DevState s = state_of_input<NT>(p.st_in, p.part_in, gridDim.x, fold_red);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevState o = s;
        o.pending = s.done ? 0 : 1;
        *p.st_out = o;
    }
    if (s.done) return;

    const float c = s.c;
    float gs[RS + 1];
#pragma unroll
    for (int d = 0; d <= RS; ++d) gs[d] = p.gs[d];
    float gt[NR];
#pragma unroll
    for (int m = 0; m < NR; ++m) gt[m] = p.gt[m < RT ? RT - m : m - RT] * c;

    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int4 item = p.items[lb];  // tile origin (picture coords) and frame range
    double syy = 0.0, syx = 0.0;
    run_item<TS, RS, RT, SH>((const TS*)p.x, (const TS*)p.w, (const TS*)p.f,
                                           p.fstride, (TS*)p.y, p.T, p.Wp, p.PT, p.PL, p.frame,
                                           item.x, item.y, item.z, item.w, gs, gt, p.alpha, lds,
                                           syy, syx);
    block_partials<NT>(syy, syx, p.part_out, lb);
}

// ---------------------------------------------------------------------------
// Batched persistent step: many clips, one launch
// ---------------------------------------------------------------------------
// Work items of all clips that are still iterating are handed out through 8
// queues, one per XCD: queue x holds a contiguous run of items (neighbouring
// tiles of one clip, so their halos meet in that XCD's L2).  A block drains
// the queue of its own XCD first, then takes leftovers from the others.  Each
// item writes its partial sums to its own slot and nothing else; the
// one-block-per-clip finish launch that follows folds each iterating clip's
// slots in a fixed order, advances only that clip's state (so a converged
// clip drops out of the next launch) and resets the queues.
template <typename TS, int RS, int RT, typename SH>
__global__ __launch_bounds__(SH::NT, (Geom<TS, RS, RT, SH>::MINW)) void batch_step_kernel(BatchParams p) {
    using G = Geom<TS, RS, RT, SH>;
    constexpr int NT = G::NT, NR = G::NR;
    __shared__ StepLds<TS, RS, RT, SH> lds;
    __shared__ int s_item;

    float gs[RS + 1];
#pragma unroll
    for (int d = 0; d <= RS; ++d) gs[d] = p.gs[d];
    int q = blockIdx.x & 7;  // queue being drained: the block's own XCD's first

    for (;;) {
        // Wave 0 takes the next item: an atomic on queue q; once q has run
        // dry, one look at all eight counters at once (lanes 0-7) moves it to
        // the first queue after q that still has items, so the end of a
        // launch costs one round trip per block instead of eight.  A failed
        // atomic leaves its queue dry for good (counters only grow), so at
        // most eight attempts fail before every queue reads empty.
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            int it = -1;
            for (int attempt = 0; attempt < 9; ++attempt) {
                if (lane == 0) {
                    const uint32_t k = atomicAdd(&p.queue[q], 1u);
                    it = (int)k < p.qcount[q] ? p.qfirst[q] + (int)k : -1;
                }
                it = __shfl(it, 0, 64);
                if (it >= 0) break;
                int left = 0;
                if (lane < 8) {
                    const int qq = (q + 1 + lane) & 7;
                    left = __hip_atomic_load(&p.queue[qq], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) < (uint32_t)p.qcount[qq];
                }
                const uint64_t m = __ballot(left);
                if (m == 0) break;  // every queue is empty
                q = (q + 1 + __builtin_ctzll(m)) & 7;
            }
            if (lane == 0) s_item = it;
        }
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it < 0) break;

        const int4 item = p.items[it];  // clip, x0 | y0 << 16, t0, t1
        const BatchClip* cl = p.clips + item.x;
        const DevState* st = cl->st;
        if (st->done) continue;  // converged or stopped: nothing to do for this clip

        const float c = st->c;
        float gt[NR];
#pragma unroll
        for (int m = 0; m < NR; ++m) gt[m] = p.gt[m < RT ? RT - m : m - RT] * c;
        double syy = 0.0, syx = 0.0;
        run_item<TS, RS, RT, SH>((const TS*)cl->buf[p.parity], (const TS*)cl->w,
                                 (const TS*)cl->f, 0, (TS*)cl->buf[1 - p.parity], cl->T, cl->Wp,
                                 cl->PT, cl->PL, cl->frame, item.y & 0xffff, item.y >> 16, item.z,
                                 item.w, gs, gt, p.alpha, lds, syy, syx);
        block_partials<NT>(syy, syx, p.partials, it);
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

// Step kernels only (no batched form) for two feature channels.
template <typename TS, typename SH, int RS, int... RTs>
void fill_rt_step(StepFns* t, std::integer_sequence<int, RTs...>) {
    ((t[RS * (SFSEG_MAX_RT + 1) + RTs] =
          StepFns{&launch_step_t<TS, RS, RTs, SH>, &occ_step_t<TS, RS, RTs, SH>, nullptr, nullptr}),
     ...);
}
template <typename TS, typename SH, int... RSs>
void fill_rs_step(StepFns* t, std::integer_sequence<int, RSs...>) {
    (fill_rt_step<TS, SH, RSs>(t, std::make_integer_sequence<int, SFSEG_MAX_RT + 1>{}), ...);
}
template <typename TS>
struct StepTable2 {
    StepFns fns[NSHAPES][NCOMB];
    StepTable2() {
        fill_rs_step<TS, ShapeWide2>(fns[0], std::make_integer_sequence<int, SFSEG_MAX_RS + 1>{});
        fill_rs_step<TS, ShapeDeep2>(fns[1], std::make_integer_sequence<int, SFSEG_MAX_RS + 1>{});
    }
};

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

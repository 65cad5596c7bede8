// Warm-start network: host side of the C-ABI (sfseg_unet_*).
//
// The network maps the input map S to an estimate of the principal
// eigenvector; its output is the start vector of the power iteration, which
// then runs to the requested tolerance (the start vector of Algorithm 1 is a
// soft segmentation provided by another method).  Training, inference and the
// gradients all run in the kernels of unet_kernels.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "host_internal.h"
#include "sfseg.h"
#include "unet_kernels.h"

using namespace sfseg_host;
using sfseg::unet::View;
using sfseg::unet::bf16x8;

namespace {

// Layers in the exchange order: (Cin, Cout); the last is the 1x1x1 head.
struct LayerDef {
    int cin, cout, k;
};
constexpr LayerDef kLayers[11] = {{1, 16, 3},  {16, 16, 3}, {16, 32, 3}, {32, 32, 3},
                                  {32, 64, 3}, {64, 64, 3}, {96, 32, 3}, {32, 32, 3},
                                  {48, 16, 3}, {16, 16, 3}, {16, 1, 1}};
enum { ENC1A, ENC1B, ENC2A, ENC2B, BOTA, BOTB, DEC2A, DEC2B, DEC1A, DEC1B, HEAD };

int64_t layer_weights(int l) {
    return (int64_t)kLayers[l].cout * kLayers[l].cin * (kLayers[l].k == 3 ? 27 : 1);
}
int64_t layer_offset(int l) {
    int64_t o = 0;
    for (int i = 0; i < l; ++i) o += layer_weights(i) + kLayers[i].cout;
    return o;
}
int64_t param_total() { return layer_offset(11); }
int64_t frag_elems(int fin, int fout) { return (int64_t)((27 * fin + 31) / 32) * (fout / 16) * 64; }

constexpr int kWChunks = 128;  // row chunks of the weight-gradient kernel
constexpr int kRedBlocks = 512;

int64_t ceil2(int64_t n) { return (n + 1) / 2; }

}  // namespace

struct sfseg_unet {
    int device = 0;
    hipStream_t stream = nullptr;
    int maxT = 0, maxH = 0, maxW = 0;
    int training = 0;
    int T = 0, H = 0, W = 0;  // size of the last forward pass
    bool have_forward = false;
    float* w = nullptr;  // FP32 master weights (exchange layout)
    float* g = nullptr;  // gradients
    float* m = nullptr;
    float* v = nullptr;
    bf16x8* ffwd[10] = {};
    bf16x8* fbwd[10] = {};
    // activations
    float* in32 = nullptr;
    float* z = nullptr;
    float* xh = nullptr;
    __bf16 *e1a = nullptr, *cat1 = nullptr, *p1 = nullptr, *e2a = nullptr, *cat2 = nullptr,
           *p2 = nullptr, *ba = nullptr, *bb = nullptr, *d2a = nullptr, *d2 = nullptr,
           *d1a = nullptr, *d1 = nullptr;
    // gradient buffers
    __bf16 *gA = nullptr, *gB = nullptr, *gC = nullptr;        // full: 16, 16, 48 ch
    __bf16 *gD = nullptr, *gE = nullptr, *gF = nullptr, *gG = nullptr;  // half: 32, 32, 96, 16
    __bf16 *gH = nullptr, *gI = nullptr, *gJ = nullptr;        // quarter: 64, 64, 32
    float* wpart = nullptr;
    double* dpart = nullptr;
    double* h_dpart = nullptr;  // pinned
    std::vector<void*> allocs;
};

namespace {

template <typename T>
int dalloc(sfseg_unet* n, T** p, int64_t count) {
    HIP_TRY(hipMalloc((void**)p, sizeof(T) * (size_t)std::max<int64_t>(count, 1)));
    n->allocs.push_back((void*)*p);
    return SFSEG_OK;
}

View view(__bf16* p, int T, int H, int W, int cs, int c0) { return View{p, T, H, W, cs, c0}; }

int grid_for(int64_t n, int per = 256) {
    const int64_t b = (n + per - 1) / per;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 65535 * 8);
}

// Block shape of the streamed convolution (rows RB x voxels XB): a frame
// slab, (RB + 2) rows x (XB + 2) voxels x CIN channels of 2 bytes, is 6.5 KB
// for 16 channels, 13 KB for 32 and 48 (a ring of four: three blocks per CU),
// 17 KB for 64 and 26 KB for 96.  Frame runs per tile: enough blocks to give every
// CU several.
constexpr int conv_rows(int cin) { return cin <= 32 ? 4 : 2; }
// Split K over the four waves (see conv3_stream) where the weight fragments
// would otherwise be read by every wave for one tile each: the 96 -> 32 layer.
constexpr int conv_ks(int cin, int cout) { return cin == 96 && cout == 32 ? 4 : 1; }
constexpr int conv_xb(int) { return 32; }
int conv_runs(int64_t tiles, int T) {
    const int64_t want = 2048;
    int64_t r = (want + tiles - 1) / tiles;
    if (r > T) r = T;
    return (int)(r < 1 ? 1 : r);
}

// up.p set: input channels [0, cup) are the 2x upsampling of `up` and
// channels [cup, cin) are the first cin - cup channels of `in` (see
// conv3_stream); otherwise `in` holds every input channel.
hipError_t conv_fwd_up(int cin, int cout, View in, View up, int cup, View out,
                       const bf16x8* frag, const float* bias, View mask, int mode,
                       hipStream_t s) {
    using namespace sfseg::unet;
#define SFSEG_CONV_CASE(CI, CO)                                                                   \
    if (cin == CI && cout == CO) {                                                                \
        constexpr int RB = conv_rows(CI), XB = conv_xb(CI), KS = conv_ks(CI, CO);                 \
        const int64_t tiles = (int64_t)((out.H + RB - 1) / RB) * ((out.W + XB - 1) / XB);         \
        const int runs = conv_runs(tiles, out.T);                                                 \
        if (up.p)                                                                                 \
            hipLaunchKernelGGL((conv3_stream<CI, CO, RB, XB, true, false, KS>),                   \
                               dim3((unsigned)(tiles * runs)), dim3(256), 0, s, in, up, cup, out, \
                               frag, bias, mask, mode, runs, nullptr, nullptr);                   \
        else                                                                                      \
            hipLaunchKernelGGL((conv3_stream<CI, CO, RB, XB, false, false, KS>),                  \
                               dim3((unsigned)(tiles * runs)), dim3(256), 0, s, in, up, cup, out, \
                               frag, bias, mask, mode, runs, nullptr, nullptr);                   \
        return hipGetLastError();                                                                 \
    }
    SFSEG_CONV_CASE(16, 16)
    SFSEG_CONV_CASE(16, 32)
    SFSEG_CONV_CASE(32, 32)
    SFSEG_CONV_CASE(32, 64)
    SFSEG_CONV_CASE(64, 64)
    SFSEG_CONV_CASE(96, 32)
    SFSEG_CONV_CASE(48, 16)
    SFSEG_CONV_CASE(32, 16)
    SFSEG_CONV_CASE(64, 32)
    SFSEG_CONV_CASE(32, 96)
    SFSEG_CONV_CASE(16, 48)
#undef SFSEG_CONV_CASE
    return hipErrorInvalidValue;
}

hipError_t conv_fwd(int cin, int cout, View in, View out, const bf16x8* frag, const float* bias,
                    View mask, int mode, hipStream_t s) {
    const View none{nullptr, 0, 0, 0, 0, 0};
    return conv_fwd_up(cin, cout, in, none, 0, out, frag, bias, mask, mode, s);
}

// The last 16 -> 16 convolution with the 1x1x1 head fused (inference): the
// network's output xh (FP32, T x H x W of `dims`) is written, the
// convolution's activations are not.
hipError_t conv_fwd_head(View in, View dims, const bf16x8* frag, const float* bias,
                         const float* head_w, float* xh, hipStream_t s) {
    using namespace sfseg::unet;
    constexpr int RB = conv_rows(16), XB = conv_xb(16);
    const View none{nullptr, 0, 0, 0, 0, 0};
    const int64_t tiles = (int64_t)((dims.H + RB - 1) / RB) * ((dims.W + XB - 1) / XB);
    const int runs = conv_runs(tiles, dims.T);
    hipLaunchKernelGGL((conv3_stream<16, 16, RB, XB, false, true>), dim3((unsigned)(tiles * runs)),
                       dim3(256), 0, s, in, none, 0, dims, frag, bias, none, 0, runs, head_w, xh);
    return hipGetLastError();
}

// The first layer (one FP32 input channel).
hipError_t conv_fwd_c1(const float* in, View out, const bf16x8* frag, const float* bias,
                       hipStream_t s) {
    using namespace sfseg::unet;
    const int64_t tiles = (int64_t)((out.H + C1_RB - 1) / C1_RB) * ((out.W + C1_XB - 1) / C1_XB);
    const int runs = conv_runs(tiles, out.T);
    hipLaunchKernelGGL(conv3_c1_stream<16>, dim3((unsigned)(tiles * runs)), dim3(256), 0, s, in,
                       out, frag, bias, runs);
    return hipGetLastError();
}

hipError_t conv_wgrad(int cin, int cout, View gz, View in, const float* in32, float* part,
                      hipStream_t s) {
    using namespace sfseg::unet;
    const int64_t units = (int64_t)gz.T * gz.H * ((gz.W + 31) / 32);
    const int per = (int)((units + kWChunks - 1) / kWChunks);
    const int chunks = (int)((units + per - 1) / per);
    const dim3 grid(chunks, 27), block(256);
#define SFSEG_WG_CASE(CI, CO, F32)                                                               \
    if (cin == CI && cout == CO) {                                                               \
        hipLaunchKernelGGL((conv3_wgrad<CI, CO, F32>), grid, block, 0, s, gz, in, in32, per,    \
                           part);                                                                \
        return hipGetLastError();                                                                \
    }
    SFSEG_WG_CASE(1, 16, true)
    SFSEG_WG_CASE(16, 16, false)
    SFSEG_WG_CASE(16, 32, false)
    SFSEG_WG_CASE(32, 32, false)
    SFSEG_WG_CASE(32, 64, false)
    SFSEG_WG_CASE(64, 64, false)
    SFSEG_WG_CASE(96, 32, false)
    SFSEG_WG_CASE(48, 16, false)
#undef SFSEG_WG_CASE
    return hipErrorInvalidValue;
}

int wgrad_chunks(View gz) {
    const int64_t units = (int64_t)gz.T * gz.H * ((gz.W + 31) / 32);
    const int per = (int)((units + kWChunks - 1) / kWChunks);
    return (int)((units + per - 1) / per);
}

// Weight and bias gradients of a 3x3x3 layer from its output gradient gz
// (already through the ReLU) and its input.
int layer_grads(sfseg_unet* n, int l, View gz, View in, const float* in32) {
    const LayerDef& L = kLayers[l];
    const int64_t off = layer_offset(l);
    HIP_TRY(conv_wgrad(L.cin, L.cout, gz, in, in32, n->wpart, n->stream));
    hipLaunchKernelGGL(sfseg::unet::wgrad_reduce, dim3(grid_for(layer_weights(l))), dim3(256), 0,
                       n->stream, n->wpart, wgrad_chunks(gz), L.cin, L.cout, n->g + off);
    HIP_TRY(hipGetLastError());
    const int threads = 256 / L.cout * L.cout;
    hipLaunchKernelGGL(sfseg::unet::channel_sums, dim3(kRedBlocks), dim3(threads),
                       threads * sizeof(double), n->stream, gz, L.cout, n->dpart);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(sfseg::unet::sum_partials, dim3(1), dim3(64), 0, n->stream, n->dpart,
                       kRedBlocks, L.cout, n->g + off + layer_weights(l));
    HIP_TRY(hipGetLastError());
    return SFSEG_OK;
}

int refresh_fragments(sfseg_unet* n) {
    for (int l = 0; l < 10; ++l) {
        const LayerDef& L = kLayers[l];
        const float* w = n->w + layer_offset(l);
        hipLaunchKernelGGL(sfseg::unet::make_fragments, dim3(64), dim3(256), 0, n->stream, w, L.cin,
                           L.cout, 0, n->ffwd[l]);
        HIP_TRY(hipGetLastError());
        if (l != ENC1A) {
            hipLaunchKernelGGL(sfseg::unet::make_fragments, dim3(64), dim3(256), 0, n->stream, w,
                               L.cin, L.cout, 1, n->fbwd[l]);
            HIP_TRY(hipGetLastError());
        }
    }
    return SFSEG_OK;
}

int check_net(const sfseg_unet* n) {
    if (!n) return fail(SFSEG_ERR_INVALID_ARG, "net is NULL");
    return SFSEG_OK;
}

}  // namespace

extern "C" {

int64_t sfseg_unet_param_count(void) { return param_total(); }

void sfseg_unet_destroy(sfseg_unet* n) {
    if (!n) return;
    (void)hipSetDevice(n->device);
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    for (void* p : n->allocs) (void)hipFree(p);
    if (n->h_dpart) (void)hipHostFree(n->h_dpart);
    delete n;
}

int sfseg_unet_create(int32_t max_T, int32_t max_H, int32_t max_W, int32_t training,
                      void* stream, sfseg_unet** out) {
    if (!out) return fail(SFSEG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (max_T < 1 || max_H < 1 || max_W < 1)
        return fail(SFSEG_ERR_INVALID_ARG, "max sizes must be >= 1");
    const int64_t nfull = (int64_t)max_T * max_H * max_W;
    if (nfull * 48 >= ((int64_t)1 << 31))
        return fail(SFSEG_ERR_INVALID_ARG, "volume too large for 32-bit channel-slab indexing");
    sfseg_unet* n = new (std::nothrow) sfseg_unet();
    if (!n) return fail(SFSEG_ERR_OOM, "host allocation failed");
    int rc = SFSEG_OK;
    do {
        if (hipGetDevice(&n->device) != hipSuccess) {
            rc = fail(SFSEG_ERR_HIP, "hipGetDevice failed");
            break;
        }
        n->stream = (hipStream_t)stream;
        n->maxT = max_T;
        n->maxH = max_H;
        n->maxW = max_W;
        n->training = training ? 1 : 0;
        const int64_t nh = ceil2(max_T) * ceil2(max_H) * ceil2(max_W);
        const int64_t nq = ceil2(ceil2(max_T)) * ceil2(ceil2(max_H)) * ceil2(ceil2(max_W));
        const int64_t np = param_total();
        if ((rc = dalloc(n, &n->w, np)) || (rc = dalloc(n, &n->g, np)) || (rc = dalloc(n, &n->m, np)) ||
            (rc = dalloc(n, &n->v, np)))
            break;
        for (int l = 0; l < 10 && !rc; ++l) {
            rc = dalloc(n, &n->ffwd[l], frag_elems(kLayers[l].cin, kLayers[l].cout));
            if (!rc && l != ENC1A) rc = dalloc(n, &n->fbwd[l], frag_elems(kLayers[l].cout, kLayers[l].cin));
        }
        if (rc) break;
        // Inference keeps only what the forward pass reads: the first layer
        // reads S itself, the skip tensors have their own channels alone (the
        // upsampled halves of the concatenations are never formed) and the
        // head is fused into the last convolution.
        const int64_t cat1_ch = n->training ? 48 : 16, cat2_ch = n->training ? 96 : 32;
        if ((rc = dalloc(n, &n->e1a, nfull * 16)) || (rc = dalloc(n, &n->cat1, nfull * cat1_ch)) ||
            (rc = dalloc(n, &n->p1, nh * 16)) || (rc = dalloc(n, &n->e2a, nh * 32)) ||
            (rc = dalloc(n, &n->cat2, nh * cat2_ch)) || (rc = dalloc(n, &n->p2, nq * 32)) ||
            (rc = dalloc(n, &n->ba, nq * 64)) || (rc = dalloc(n, &n->bb, nq * 64)) ||
            (rc = dalloc(n, &n->d2a, nh * 32)) || (rc = dalloc(n, &n->d2, nh * 32)) ||
            (rc = dalloc(n, &n->d1a, nfull * 16)))
            break;
        if (n->training) {
            if ((rc = dalloc(n, &n->in32, nfull)) || (rc = dalloc(n, &n->z, nfull)) ||
                (rc = dalloc(n, &n->xh, nfull)) || (rc = dalloc(n, &n->d1, nfull * 16)))
                break;
            if ((rc = dalloc(n, &n->gA, nfull * 16)) || (rc = dalloc(n, &n->gB, nfull * 16)) ||
                (rc = dalloc(n, &n->gC, nfull * 48)) || (rc = dalloc(n, &n->gD, nh * 32)) ||
                (rc = dalloc(n, &n->gE, nh * 32)) || (rc = dalloc(n, &n->gF, nh * 96)) ||
                (rc = dalloc(n, &n->gG, nh * 16)) || (rc = dalloc(n, &n->gH, nq * 64)) ||
                (rc = dalloc(n, &n->gI, nq * 64)) || (rc = dalloc(n, &n->gJ, nq * 32)))
                break;
            int64_t wp = 0;
            for (int l = 0; l < 10; ++l)
                wp = std::max<int64_t>(wp, (int64_t)kWChunks * 27 * kLayers[l].cin * kLayers[l].cout);
            if ((rc = dalloc(n, &n->wpart, wp))) break;
        }
        if ((rc = dalloc(n, &n->dpart, (int64_t)kRedBlocks * 64))) break;
        if (hipHostMalloc((void**)&n->h_dpart, sizeof(double) * kRedBlocks * 17) != hipSuccess) {
            rc = fail(SFSEG_ERR_OOM, "pinned host allocation failed");
            break;
        }
        if (hipMemsetAsync(n->m, 0, sizeof(float) * np, n->stream) != hipSuccess ||
            hipMemsetAsync(n->v, 0, sizeof(float) * np, n->stream) != hipSuccess ||
            hipMemsetAsync(n->w, 0, sizeof(float) * np, n->stream) != hipSuccess ||
            hipMemsetAsync(n->g, 0, sizeof(float) * np, n->stream) != hipSuccess) {
            rc = fail(SFSEG_ERR_HIP, "hipMemsetAsync failed");
            break;
        }
        rc = refresh_fragments(n);
        if (rc) break;
        if (hipStreamSynchronize(n->stream) != hipSuccess) {
            rc = fail(SFSEG_ERR_HIP, "hipStreamSynchronize failed");
            break;
        }
    } while (0);
    if (rc) {
        sfseg_unet_destroy(n);
        return rc;
    }
    *out = n;
    return SFSEG_OK;
}

int sfseg_unet_set_params(sfseg_unet* n, const float* host, int64_t count) {
    int rc = check_net(n);
    if (rc) return rc;
    if (!host || count != param_total())
        return fail(SFSEG_ERR_INVALID_ARG, "expected %lld parameters", (long long)param_total());
    HIP_TRY(hipSetDevice(n->device));
    HIP_TRY(hipMemcpyAsync(n->w, host, sizeof(float) * count, hipMemcpyHostToDevice, n->stream));
    HIP_TRY(hipMemsetAsync(n->m, 0, sizeof(float) * count, n->stream));
    HIP_TRY(hipMemsetAsync(n->v, 0, sizeof(float) * count, n->stream));
    rc = refresh_fragments(n);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(n->stream));
    return SFSEG_OK;
}

int sfseg_unet_get_params(const sfseg_unet* n, float* host, int64_t count) {
    int rc = check_net(n);
    if (rc) return rc;
    if (!host || count != param_total())
        return fail(SFSEG_ERR_INVALID_ARG, "expected %lld parameters", (long long)param_total());
    HIP_TRY(hipSetDevice(n->device));
    HIP_TRY(hipMemcpyAsync(host, n->w, sizeof(float) * count, hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    return SFSEG_OK;
}

int sfseg_unet_get_grads(const sfseg_unet* n, float* host, int64_t count) {
    int rc = check_net(n);
    if (rc) return rc;
    if (!n->training) return fail(SFSEG_ERR_STATE, "network was created without training buffers");
    if (!host || count != param_total())
        return fail(SFSEG_ERR_INVALID_ARG, "expected %lld parameters", (long long)param_total());
    HIP_TRY(hipSetDevice(n->device));
    HIP_TRY(hipMemcpyAsync(host, n->g, sizeof(float) * count, hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    return SFSEG_OK;
}

int sfseg_unet_forward(sfseg_unet* n, const float* S, int32_t T, int32_t H, int32_t W, float* out) {
    int rc = check_net(n);
    if (rc) return rc;
    if (!S || !out) return fail(SFSEG_ERR_INVALID_ARG, "S or out is NULL");
    if (T < 1 || H < 1 || W < 1 || T > n->maxT || H > n->maxH || W > n->maxW)
        return fail(SFSEG_ERR_INVALID_ARG, "size %dx%dx%d outside 1..%dx%dx%d", T, H, W, n->maxT,
                    n->maxH, n->maxW);
    HIP_TRY(hipSetDevice(n->device));
    hipStream_t s = n->stream;
    const int64_t nv = (int64_t)T * H * W;
    const int Th = (int)ceil2(T), Hh = (int)ceil2(H), Wh = (int)ceil2(W);
    const int Tq = (int)ceil2(Th), Hq = (int)ceil2(Hh), Wq = (int)ceil2(Wh);
    const bool tr = n->training != 0;
    if (tr) HIP_TRY(hipMemcpyAsync(n->in32, S, sizeof(float) * nv, hipMemcpyDeviceToDevice, s));
    const View none{nullptr, 0, 0, 0, 0, 0};
    // the skip tensors e1, e2: the last channels of the concatenations in
    // training, tensors of their own in inference
    const View e1a = view(n->e1a, T, H, W, 16, 0),
               e1 = tr ? view(n->cat1, T, H, W, 48, 32) : view(n->cat1, T, H, W, 16, 0),
               cat1 = view(n->cat1, T, H, W, 48, 0), u1 = view(n->cat1, T, H, W, 48, 0),
               p1 = view(n->p1, Th, Hh, Wh, 16, 0), e2a = view(n->e2a, Th, Hh, Wh, 32, 0),
               e2 = tr ? view(n->cat2, Th, Hh, Wh, 96, 64) : view(n->cat2, Th, Hh, Wh, 32, 0),
               cat2 = view(n->cat2, Th, Hh, Wh, 96, 0),
               u2 = view(n->cat2, Th, Hh, Wh, 96, 0), p2 = view(n->p2, Tq, Hq, Wq, 32, 0),
               ba = view(n->ba, Tq, Hq, Wq, 64, 0), bb = view(n->bb, Tq, Hq, Wq, 64, 0),
               d2a = view(n->d2a, Th, Hh, Wh, 32, 0), d2 = view(n->d2, Th, Hh, Wh, 32, 0),
               d1a = view(n->d1a, T, H, W, 16, 0), d1 = view(n->d1, T, H, W, 16, 0);
    const float* w = n->w;
    auto bias = [&](int l) { return w + layer_offset(l) + layer_weights(l); };
    HIP_TRY(conv_fwd_c1(tr ? n->in32 : S, e1a, n->ffwd[ENC1A], bias(ENC1A), s));
    HIP_TRY(conv_fwd(16, 16, e1a, e1, n->ffwd[ENC1B], bias(ENC1B), none, 0, s));
    hipLaunchKernelGGL(sfseg::unet::pool2_fwd, dim3(grid_for((int64_t)Th * Hh * Wh * 2)), dim3(256), 0,
                       s, e1, p1, 16);
    HIP_TRY(hipGetLastError());
    HIP_TRY(conv_fwd(16, 32, p1, e2a, n->ffwd[ENC2A], bias(ENC2A), none, 0, s));
    HIP_TRY(conv_fwd(32, 32, e2a, e2, n->ffwd[ENC2B], bias(ENC2B), none, 0, s));
    hipLaunchKernelGGL(sfseg::unet::pool2_fwd, dim3(grid_for((int64_t)Tq * Hq * Wq * 4)), dim3(256), 0,
                       s, e2, p2, 32);
    HIP_TRY(hipGetLastError());
    HIP_TRY(conv_fwd(32, 64, p2, ba, n->ffwd[BOTA], bias(BOTA), none, 0, s));
    HIP_TRY(conv_fwd(64, 64, ba, bb, n->ffwd[BOTB], bias(BOTB), none, 0, s));
    if (tr) {
        hipLaunchKernelGGL(sfseg::unet::up2_fwd, dim3(grid_for((int64_t)Th * Hh * Wh * 8)), dim3(256),
                           0, s, bb, u2, 64);
        HIP_TRY(hipGetLastError());
        HIP_TRY(conv_fwd(96, 32, cat2, d2a, n->ffwd[DEC2A], bias(DEC2A), none, 0, s));
    } else {
        // the upsampled half of the concatenation read at the parent voxels
        // while the convolution stages its input
        HIP_TRY(conv_fwd_up(96, 32, e2, bb, 64, d2a, n->ffwd[DEC2A], bias(DEC2A), none, 0, s));
    }
    HIP_TRY(conv_fwd(32, 32, d2a, d2, n->ffwd[DEC2B], bias(DEC2B), none, 0, s));
    if (tr) {
        // the backward pass reads the concatenation, d1 and z
        hipLaunchKernelGGL(sfseg::unet::up2_fwd, dim3(grid_for(nv * 4)), dim3(256), 0, s, d2, u1, 32);
        HIP_TRY(hipGetLastError());
        HIP_TRY(conv_fwd(48, 16, cat1, d1a, n->ffwd[DEC1A], bias(DEC1A), none, 0, s));
        HIP_TRY(conv_fwd(16, 16, d1a, d1, n->ffwd[DEC1B], bias(DEC1B), none, 0, s));
        hipLaunchKernelGGL(sfseg::unet::head_fwd, dim3(grid_for(nv)), dim3(256), 0, s, d1,
                           w + layer_offset(HEAD), n->z, n->xh);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(out, n->xh, sizeof(float) * nv, hipMemcpyDeviceToDevice, s));
    } else {
        // the same at full resolution, and the head in the last
        // convolution's epilogue
        HIP_TRY(conv_fwd_up(48, 16, e1, d2, 32, d1a, n->ffwd[DEC1A], bias(DEC1A), none, 0, s));
        HIP_TRY(conv_fwd_head(d1a, d1a, n->ffwd[DEC1B], bias(DEC1B), w + layer_offset(HEAD), out, s));
    }
    n->T = T;
    n->H = H;
    n->W = W;
    n->have_forward = true;
    return SFSEG_OK;
}

}  // extern "C"

namespace {

// Backward pass from dL/dx^: either the cosine loss against `target` (loss
// written to *loss) or an external gradient `gext`.
int backward_core(sfseg_unet* n, const float* target, const float* gext, double* loss) {
    int rc = SFSEG_OK;
    HIP_TRY(hipSetDevice(n->device));
    hipStream_t s = n->stream;
    const int T = n->T, H = n->H, W = n->W;
    const int64_t nv = (int64_t)T * H * W;
    const int Th = (int)ceil2(T), Hh = (int)ceil2(H), Wh = (int)ceil2(W);
    const int Tq = (int)ceil2(Th), Hq = (int)ceil2(Hh), Wq = (int)ceil2(Wh);
    const View none{nullptr, 0, 0, 0, 0, 0};
    const View e1a = view(n->e1a, T, H, W, 16, 0), e1 = view(n->cat1, T, H, W, 48, 32),
               cat1 = view(n->cat1, T, H, W, 48, 0), p1 = view(n->p1, Th, Hh, Wh, 16, 0),
               e2a = view(n->e2a, Th, Hh, Wh, 32, 0), e2 = view(n->cat2, Th, Hh, Wh, 96, 64),
               cat2 = view(n->cat2, Th, Hh, Wh, 96, 0), p2 = view(n->p2, Tq, Hq, Wq, 32, 0),
               ba = view(n->ba, Tq, Hq, Wq, 64, 0), bb = view(n->bb, Tq, Hq, Wq, 64, 0),
               d2a = view(n->d2a, Th, Hh, Wh, 32, 0), d2 = view(n->d2, Th, Hh, Wh, 32, 0),
               d1a = view(n->d1a, T, H, W, 16, 0), d1 = view(n->d1, T, H, W, 16, 0);
    // gradient views
    const View gd1 = view(n->gA, T, H, W, 16, 0), gd1a = view(n->gB, T, H, W, 16, 0),
               gcat1 = view(n->gC, T, H, W, 48, 0), gu1 = view(n->gC, T, H, W, 48, 0),
               gskip1 = view(n->gC, T, H, W, 48, 32), ge1 = view(n->gA, T, H, W, 16, 0),
               ge1a = view(n->gB, T, H, W, 16, 0), gd2 = view(n->gD, Th, Hh, Wh, 32, 0),
               gd2a = view(n->gE, Th, Hh, Wh, 32, 0), gcat2 = view(n->gF, Th, Hh, Wh, 96, 0),
               gu2 = view(n->gF, Th, Hh, Wh, 96, 0), gskip2 = view(n->gF, Th, Hh, Wh, 96, 64),
               ge2 = view(n->gD, Th, Hh, Wh, 32, 0), ge2a = view(n->gE, Th, Hh, Wh, 32, 0),
               gp1 = view(n->gG, Th, Hh, Wh, 16, 0), gb = view(n->gH, Tq, Hq, Wq, 64, 0),
               gba = view(n->gI, Tq, Hq, Wq, 64, 0), gp2 = view(n->gJ, Tq, Hq, Wq, 32, 0);

    // loss and its scale factors
    double coef0 = 0.0, coef1 = 0.0;
    if (!gext) {
        hipLaunchKernelGGL(sfseg::unet::loss_sums, dim3(kRedBlocks), dim3(256), 0, s, n->xh, target,
                           nv, n->dpart);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(n->h_dpart, n->dpart, sizeof(double) * 3 * kRedBlocks,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double dot = 0.0, xx = 0.0, tt = 0.0;
        for (int b = 0; b < kRedBlocks; ++b) {
            dot += n->h_dpart[3 * b];
            xx += n->h_dpart[3 * b + 1];
            tt += n->h_dpart[3 * b + 2];
        }
        const double nx = sqrt(xx), nt = sqrt(tt);
        if (!(nx > 0.0) || !(nt > 0.0) || !isfinite(dot))
            return fail(SFSEG_ERR_ZERO_NORM, "network output or target has zero or non-finite norm");
        const double cosv = dot / (nx * nt);
        if (loss) *loss = 1.0 - cosv;
        coef0 = 1.0 / (nx * nt);
        coef1 = cosv / (nx * nx);
    }
    const float* w = n->w;
    hipLaunchKernelGGL(sfseg::unet::head_bwd, dim3(kRedBlocks), dim3(256), 0, s, d1,
                       w + layer_offset(HEAD), n->z, n->xh, target, gext, coef0, coef1, gd1,
                       n->dpart);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(sfseg::unet::sum_partials, dim3(1), dim3(64), 0, s, n->dpart, kRedBlocks, 17,
                       n->g + layer_offset(HEAD));
    HIP_TRY(hipGetLastError());

    // decoder level 1
    if ((rc = layer_grads(n, DEC1B, gd1, d1a, nullptr))) return rc;
    HIP_TRY(conv_fwd(16, 16, gd1, gd1a, n->fbwd[DEC1B], nullptr, d1a, 1, s));
    if ((rc = layer_grads(n, DEC1A, gd1a, cat1, nullptr))) return rc;
    HIP_TRY(conv_fwd(16, 48, gd1a, gcat1, n->fbwd[DEC1A], nullptr, none, 1, s));
    hipLaunchKernelGGL(sfseg::unet::up2_bwd, dim3(grid_for((int64_t)Th * Hh * Wh * 32)), dim3(256), 0, s,
                       gu1, d2, gd2, 32);
    HIP_TRY(hipGetLastError());
    // decoder level 2
    if ((rc = layer_grads(n, DEC2B, gd2, d2a, nullptr))) return rc;
    HIP_TRY(conv_fwd(32, 32, gd2, gd2a, n->fbwd[DEC2B], nullptr, d2a, 1, s));
    if ((rc = layer_grads(n, DEC2A, gd2a, cat2, nullptr))) return rc;
    HIP_TRY(conv_fwd(32, 96, gd2a, gcat2, n->fbwd[DEC2A], nullptr, none, 1, s));
    hipLaunchKernelGGL(sfseg::unet::up2_bwd, dim3(grid_for((int64_t)Tq * Hq * Wq * 64)), dim3(256), 0, s,
                       gu2, bb, gb, 64);
    HIP_TRY(hipGetLastError());
    // bottleneck
    if ((rc = layer_grads(n, BOTB, gb, ba, nullptr))) return rc;
    HIP_TRY(conv_fwd(64, 64, gb, gba, n->fbwd[BOTB], nullptr, ba, 1, s));
    if ((rc = layer_grads(n, BOTA, gba, p2, nullptr))) return rc;
    HIP_TRY(conv_fwd(64, 32, gba, gp2, n->fbwd[BOTA], nullptr, none, 1, s));
    hipLaunchKernelGGL(sfseg::unet::pool2_bwd, dim3(grid_for((int64_t)Th * Hh * Wh * 32)), dim3(256), 0,
                       s, gp2, gskip2, e2, ge2, 32);
    HIP_TRY(hipGetLastError());
    // encoder level 2
    if ((rc = layer_grads(n, ENC2B, ge2, e2a, nullptr))) return rc;
    HIP_TRY(conv_fwd(32, 32, ge2, ge2a, n->fbwd[ENC2B], nullptr, e2a, 1, s));
    if ((rc = layer_grads(n, ENC2A, ge2a, p1, nullptr))) return rc;
    HIP_TRY(conv_fwd(32, 16, ge2a, gp1, n->fbwd[ENC2A], nullptr, none, 1, s));
    hipLaunchKernelGGL(sfseg::unet::pool2_bwd, dim3(grid_for(nv * 16)), dim3(256), 0, s, gp1, gskip1,
                       e1, ge1, 16);
    HIP_TRY(hipGetLastError());
    // encoder level 1
    if ((rc = layer_grads(n, ENC1B, ge1, e1a, nullptr))) return rc;
    HIP_TRY(conv_fwd(16, 16, ge1, ge1a, n->fbwd[ENC1B], nullptr, e1a, 1, s));
    if ((rc = layer_grads(n, ENC1A, ge1a, none, n->in32))) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    return SFSEG_OK;
}

int check_backward(const sfseg_unet* n) {
    int rc = check_net(n);
    if (rc) return rc;
    if (!n->training) return fail(SFSEG_ERR_STATE, "network was created without training buffers");
    if (!n->have_forward) return fail(SFSEG_ERR_STATE, "no forward pass to differentiate");
    return SFSEG_OK;
}

}  // namespace

extern "C" {

int sfseg_unet_backward(sfseg_unet* n, const float* target, double* loss) {
    int rc = check_backward(n);
    if (rc) return rc;
    if (!target) return fail(SFSEG_ERR_INVALID_ARG, "target is NULL");
    return backward_core(n, target, nullptr, loss);
}

int sfseg_unet_backward_from(sfseg_unet* n, const float* grad_out) {
    int rc = check_backward(n);
    if (rc) return rc;
    if (!grad_out) return fail(SFSEG_ERR_INVALID_ARG, "grad_out is NULL");
    return backward_core(n, nullptr, grad_out, nullptr);
}

int sfseg_unet_adam_step(sfseg_unet* n, double lr, double beta1, double beta2, double eps,
                         int32_t step) {
    int rc = check_net(n);
    if (rc) return rc;
    if (!n->training) return fail(SFSEG_ERR_STATE, "network was created without training buffers");
    if (step < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
        !(eps > 0.0))
        return fail(SFSEG_ERR_INVALID_ARG, "bad Adam hyper-parameters");
    HIP_TRY(hipSetDevice(n->device));
    const int64_t np = param_total();
    const float c1 = (float)(1.0 - pow(beta1, step)), c2 = (float)(1.0 - pow(beta2, step));
    hipLaunchKernelGGL(sfseg::unet::adam_step, dim3(grid_for(np)), dim3(256), 0, n->stream, n->w, n->g,
                       n->m, n->v, np, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
    HIP_TRY(hipGetLastError());
    rc = refresh_fragments(n);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(n->stream));
    return SFSEG_OK;
}

int sfseg_unet_sync(sfseg_unet* n) {
    int rc = check_net(n);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(n->device));
    HIP_TRY(hipStreamSynchronize(n->stream));
    return SFSEG_OK;
}

}  // extern "C"

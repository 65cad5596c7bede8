// C ABI of the SFSeg power-iteration library (declared in include/sfseg.h).
//
// Host side: argument checks, buffer ownership, launch geometry and the
// iteration loop.  Steps are launched in chunks on the context's stream; each
// chunk is captured once as a HIP graph and replayed.  After each chunk the
// host reads the 80-byte device state once to see whether the iteration has
// stopped (later launches in a chunk exit at once when it has).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "sfseg.h"
#include "sfseg_internal.h"

#include "host_internal.h"

using sfseg::DevState;
using sfseg::StepParams;
using namespace sfseg_host;

namespace sfseg_host {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

size_t dtype_size(int dt) { return dt == SFSEG_F32 ? 4 : 2; }

}  // namespace sfseg_host

extern "C" {

void sfseg_config_default(sfseg_config* cfg) {
    if (!cfg) return;
    memset(cfg, 0, sizeof(*cfg));
    cfg->r_t = 1;
    cfg->r_s = 2;
    cfg->storage = SFSEG_F32;
    cfg->sigma_t = 1.0;
    cfg->sigma_s = 1.0;
    cfg->alpha = 1.0;
    cfg->p = 0.2;
}

int sfseg_config_validate(const sfseg_config* c) {
    if (!c) return fail(SFSEG_ERR_INVALID_ARG, "config is NULL");
    if (c->T < 1 || c->H < 1 || c->W < 1)
        return fail(SFSEG_ERR_INVALID_ARG, "T, H, W must be >= 1 (got %d, %d, %d)", c->T, c->H,
                    c->W);
    if ((int64_t)c->T * c->H * c->W >= ((int64_t)1 << 31))
        return fail(SFSEG_ERR_INVALID_ARG, "T*H*W must be < 2^31");
    if (c->r_t < 0 || c->r_s < 0)
        return fail(SFSEG_ERR_INVALID_ARG, "radii must be >= 0 (r_t=%d, r_s=%d)", c->r_t, c->r_s);
    if (c->r_t > SFSEG_MAX_RT || c->r_s > SFSEG_MAX_RS)
        return fail(SFSEG_ERR_UNSUPPORTED, "radius beyond the compiled maximum (r_t<=%d, r_s<=%d)",
                    SFSEG_MAX_RT, SFSEG_MAX_RS);
    if (!(c->sigma_t > 0.0) || !(c->sigma_s > 0.0) || !isfinite(c->sigma_t) ||
        !isfinite(c->sigma_s))
        return fail(SFSEG_ERR_INVALID_ARG, "sigma_t and sigma_s must be finite and > 0");
    if (!(c->alpha >= 0.0) || !isfinite(c->alpha))
        return fail(SFSEG_ERR_INVALID_ARG, "alpha must be finite and >= 0");
    if (!(c->p >= 0.0) || !isfinite(c->p))
        return fail(SFSEG_ERR_INVALID_ARG, "p must be finite and >= 0");
    if (c->storage != SFSEG_F32 && c->storage != SFSEG_BF16 && c->storage != SFSEG_F16)
        return fail(SFSEG_ERR_INVALID_ARG, "storage must be SFSEG_F32, SFSEG_BF16 or SFSEG_F16");
    return SFSEG_OK;
}

const char* sfseg_status_string(int s) {
    switch (s) {
        case SFSEG_OK: return "ok";
        case SFSEG_ERR_INVALID_ARG: return "invalid argument";
        case SFSEG_ERR_OOM: return "out of memory";
        case SFSEG_ERR_HIP: return "HIP runtime error";
        case SFSEG_ERR_ZERO_NORM: return "zero norm";
        case SFSEG_ERR_NONFINITE: return "non-finite value";
        case SFSEG_ERR_STATE: return "call out of order";
        case SFSEG_ERR_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char* sfseg_last_error(void) { return g_err; }

void sfseg_destroy(sfseg_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->batch) destroy_batch(ctx->batch);
    if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    void* dev[] = {ctx->w, ctx->f, ctx->s0, ctx->buf[0], ctx->buf[1], ctx->apply_in,
                   ctx->apply_out, ctx->st, ctx->st_apply, ctx->d_bad, ctx->partials,
                   ctx->step_part, ctx->items, ctx->spec_buf, ctx->spec_norms, ctx->spec_part,
                   ctx->ritz_part, ctx->ritz_fac};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    if (ctx->h_st) (void)hipHostFree(ctx->h_st);
    if (ctx->h_bad) (void)hipHostFree(ctx->h_bad);
    if (ctx->h_spec) (void)hipHostFree(ctx->h_spec);
    if (ctx->h_ritz) (void)hipHostFree(ctx->h_ritz);
    delete ctx;
}

}  // extern "C"

namespace sfseg_host {

// Gaussian taps of Eq. (1), one axis: exp(-d^2 / (2 sigma^2)), d = 0..r,
// evaluated in float64 and rounded once to float32.
void axis_taps(int r, double sigma, float* out) {
    for (int d = 0; d <= r; ++d) out[d] = (float)exp(-(double)d * d / (2.0 * sigma * sigma));
}

int run_prep(sfseg_ctx* ctx, const float* S, const float* F) {
    HIP_TRY(hipMemsetAsync(ctx->d_bad, 0, sizeof(int32_t), ctx->stream));
    HIP_TRY(sfseg::launch_prep(ctx->cfg.storage, S, F, ctx->cfg.p, ctx->w, ctx->f, ctx->s0, ctx->L,
                               ctx->d_bad, ctx->ew_grid, ctx->stream));
    // further feature channels: F holds them one after another
    const int64_t n = (int64_t)ctx->cfg.T * ctx->cfg.H * ctx->cfg.W;
    for (int c = 1; c < ctx->nf; ++c)
        HIP_TRY(sfseg::launch_to_storage(ctx->cfg.storage, F + c * n,
                                         (char*)ctx->f + c * ctx->L.total * dtype_size(ctx->cfg.storage),
                                         ctx->L, ctx->ew_grid, ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->h_bad, ctx->d_bad, sizeof(int32_t), hipMemcpyDeviceToHost,
                           ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->have_iterate = false;
    if (*ctx->h_bad)
        return fail(SFSEG_ERR_NONFINITE, "S or F holds NaN/Inf, or S < 0 with p > 0");
    return SFSEG_OK;
}

// Padded layout for the step kernel: the picture sits at row PT = r_s and
// column PL = r_s rounded up to a multiple of 4; rows are PL + tiles + PL
// wide, so every tile's region (halo rounded out to 16-byte columns) lies
// inside the frame and starts on a 16-byte boundary.
sfseg::Layout make_layout(const sfseg_config& c) {
    sfseg::Layout L{};
    L.T = c.T;
    L.H = c.H;
    L.W = c.W;
    L.tiles_x = (c.W + sfseg::TILE_X - 1) / sfseg::TILE_X;
    L.tiles_y = (c.H + sfseg::TILE_Y - 1) / sfseg::TILE_Y;
    L.PT = c.r_s;
    L.PL = (c.r_s + 3) / 4 * 4;  // halo rounded up to 16-byte columns
    L.Hp = L.PT + L.tiles_y * sfseg::TILE_Y + c.r_s;
    L.Wp = L.PL + L.tiles_x * sfseg::TILE_X + L.PL;
    L.frame = (int64_t)L.Hp * L.Wp;
    L.total = L.frame * L.T;
    return L;
}

// Work items of the step kernel: every tile over `chunks` equal runs of
// frames, chunk-major, then tile rows, then tile columns; padded with empty
// items to a multiple of 8 blocks (one share per XCD).
// Balanced work list (chunks = 0, vector shapes): each of the 8 XCDs gets a
// contiguous band of tiles and exactly two items per resident block slot of
// its CUs; a band's tiles are cut into runs of frames -- some tiles one run
// more than others -- to make up that count, and the band's items go longest
// first, run by run, so that the blocks the dispatcher hands out last are
// the short ones.  Two items per slot fill the slots in two even waves
// instead of the 1.6 waves of three equal runs per tile, for a few more
// warm-up frames.  Returns an empty list when the clip has too few tiles or
// frames for it (every band needs at least one tile, every run 4 r_t + 4
// frames).
std::vector<int4> balanced_items(const sfseg::Layout& L, int slots, int most_runs) {
    std::vector<int4> items;
    const int tiles = L.tiles_x * L.tiles_y;
    const int per_band = 2 * (slots / 8);
    if (tiles < 8 || per_band < 1) return items;
    for (int band = 0; band < 8; ++band) {
        const int a = tiles * band / 8, b = tiles * (band + 1) / 8;
        const int n = b - a;
        const int lo = per_band / n, extra = per_band - lo * n;  // `extra` tiles get lo + 1
        if (lo < 1 || lo + (extra ? 1 : 0) > most_runs) return std::vector<int4>();
        // longest items first: the tiles with lo runs (the last n - extra of
        // the band), then those with lo + 1
        for (int pass = 0; pass < 2; ++pass) {
            const int runs = pass == 0 ? lo : lo + 1;
            const int t_first = pass == 0 ? a + extra : a, t_last = pass == 0 ? b : a + extra;
            for (int r = 0; r < runs; ++r) {
                const int t0 = (int)((int64_t)L.T * r / runs), t1 = (int)((int64_t)L.T * (r + 1) / runs);
                for (int t = t_first; t < t_last; ++t) {
                    const int tx = t % L.tiles_x, ty = t / L.tiles_x;
                    items.push_back(make_int4(tx * sfseg::TILE_X, ty * sfseg::TILE_Y, t0, t1));
                }
            }
        }
    }
    return items;
}

std::vector<int4> plan_items(const sfseg::Layout& L, int chunks, int shape) {
    // the fused two-step kernel works on smaller tiles (its LDS holds two
    // steps' rings); they cover the same area as the 64 x 16 tiling
    const bool fused = shape == sfseg::SHAPE_FUSED2;
    const int tw = fused ? sfseg::FUSED_TILE_X : sfseg::TILE_X;
    const int th = fused ? sfseg::FUSED_TILE_Y : sfseg::TILE_Y;
    const int nx = L.tiles_x * (sfseg::TILE_X / tw), ny = L.tiles_y * (sfseg::TILE_Y / th);
    std::vector<int4> items;
    for (int ch = 0; ch < chunks; ++ch) {
        const int t0 = (int)((int64_t)L.T * ch / chunks), t1 = (int)((int64_t)L.T * (ch + 1) / chunks);
        if (t1 <= t0) continue;
        for (int ty = 0; ty < ny; ++ty)
            for (int tx = 0; tx < nx; ++tx) items.push_back(make_int4(tx * tw, ty * th, t0, t1));
    }
    while (items.size() % 8) items.push_back(make_int4(0, 0, 0, 0));
    return items;
}

// Install a work plan: block shape and number of frame runs per tile.  The
// work items and the grid follow from it; a captured graph is dropped.
int install_plan(sfseg_ctx* ctx, int shape, int chunks) {
    std::vector<int4> items;
    if (chunks == 0) {
        int occ = 1;
        HIP_TRY(sfseg::step_max_blocks_per_cu(ctx->cfg.storage, sfseg::kernel_shape(shape, ctx->nf),
                                              ctx->cfg.r_s, ctx->cfg.r_t, &occ));
        items = balanced_items(ctx->L, ctx->cus * (occ < 1 ? 1 : occ), max_chunks(ctx->cfg));
        if (items.empty())
            return fail(SFSEG_ERR_INVALID_ARG,
                        "the clip has too few tiles or frames for the balanced plan (chunks = 0)");
    } else {
        items = plan_items(ctx->L, chunks, shape);
    }
    if (items.size() > ctx->items_cap) {
        if (ctx->items) HIP_TRY(hipFree(ctx->items));
        ctx->items = nullptr;
        HIP_TRY(hipMalloc((void**)&ctx->items, sizeof(int4) * items.size()));
        ctx->items_cap = items.size();
    }
    const int grid = (int)items.size();
    const int need = grid > ctx->ew_grid ? grid : ctx->ew_grid;
    if (need > ctx->partial_slots) {
        if (ctx->partials) HIP_TRY(hipFree(ctx->partials));
        ctx->partials = nullptr;
        HIP_TRY(hipMalloc((void**)&ctx->partials, sizeof(double) * 2 * need));
        ctx->partial_slots = need;
    }
    if (grid > ctx->step_part_slots) {
        if (ctx->step_part) HIP_TRY(hipFree(ctx->step_part));
        ctx->step_part = nullptr;
        // two sets (one per iterate buffer) of up to two pairs of sums per block
        HIP_TRY(hipMalloc((void**)&ctx->step_part, sizeof(double) * 8 * grid));
        ctx->step_part_slots = grid;
    }
    HIP_TRY(hipMemcpyAsync(ctx->items, items.data(), sizeof(int4) * items.size(),
                           hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->shape = shape;
    ctx->chunks = chunks;
    ctx->step_grid = grid;
    for (int b = 0; b < 2; ++b) {
        StepParams& p = ctx->params[b];
        p.items = ctx->items;
        p.part_in = ctx->step_part + 4 * (size_t)ctx->step_part_slots * b;
        p.part_out = ctx->step_part + 4 * (size_t)ctx->step_part_slots * (1 - b);
        p.half = 0;
    }
    if (ctx->graph) {
        (void)hipGraphExecDestroy(ctx->graph);
        ctx->graph = nullptr;
    }
    return SFSEG_OK;
}

// Longest useful split of time: every run keeps at least 4 r_t + 4 frames
// (the register ring warms up over 2 r_t of them).
int max_chunks(const sfseg_config& c) {
    const int m = c.T / (4 * c.r_t + 4);
    return m > 1 ? m : 1;
}

// Default plan: the 256-thread shape; one run per tile when the tiles alone
// fill the resident block slots, otherwise enough runs to fill them.
int default_plan(sfseg_ctx* ctx, int* shape, int* chunks) {
    const sfseg_config& c = ctx->cfg;
    *shape = 0;
    int occ = 1;
    HIP_TRY(sfseg::step_max_blocks_per_cu(c.storage, sfseg::kernel_shape(*shape, ctx->nf), c.r_s,
                                          c.r_t, &occ));
    if (occ < 1) occ = 1;
    const int tiles = ctx->L.tiles_x * ctx->L.tiles_y;
    int ch = ctx->cus * occ / tiles;
    if (ch > max_chunks(c)) ch = max_chunks(c);
    *chunks = ch < 1 ? 1 : ch;
    return SFSEG_OK;
}

int setup(sfseg_ctx* ctx, const float* S, const float* F) {
    const sfseg_config& c = ctx->cfg;
    ctx->L = make_layout(c);
    const sfseg::Layout& L = ctx->L;
    if (L.total * (int64_t)dtype_size(c.storage) >= ((int64_t)1 << 31))
        return fail(SFSEG_ERR_INVALID_ARG, "padded volume exceeds 2 GiB per array");
    const size_t bytes = (size_t)L.total * dtype_size(c.storage);
    HIP_TRY(hipGetDevice(&ctx->device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, ctx->device));
    ctx->cus = prop.multiProcessorCount;
    ctx->ew_grid = ctx->cus * 8;

    HIP_TRY(hipMalloc(&ctx->w, bytes));
    HIP_TRY(hipMalloc(&ctx->f, bytes * ctx->nf));
    HIP_TRY(hipMalloc(&ctx->s0, bytes));
    HIP_TRY(hipMalloc(&ctx->buf[0], bytes));
    HIP_TRY(hipMalloc(&ctx->buf[1], bytes));
    HIP_TRY(hipMalloc((void**)&ctx->st, 2 * sizeof(DevState)));
    HIP_TRY(hipMalloc((void**)&ctx->st_apply, 2 * sizeof(DevState)));
    HIP_TRY(hipMalloc((void**)&ctx->d_bad, sizeof(int32_t)));
    HIP_TRY(hipHostMalloc((void**)&ctx->h_st, 3 * sizeof(DevState), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void**)&ctx->h_bad, sizeof(int32_t), hipHostMallocDefault));
    for (auto& e : ctx->ev) HIP_TRY(hipEventCreate(&e));
    // The padding of every volume must hold zeros; nothing ever writes it.
    void* vols[] = {ctx->w, ctx->s0, ctx->buf[0], ctx->buf[1]};
    for (void* v : vols) HIP_TRY(hipMemsetAsync(v, 0, bytes, ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->f, 0, bytes * ctx->nf, ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->st, 0, 2 * sizeof(DevState), ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->st_apply, 0, 2 * sizeof(DevState), ctx->stream));

    for (int b = 0; b < 2; ++b) {
        StepParams& p = ctx->params[b];
        memset(&p, 0, sizeof(p));
        p.x = ctx->buf[b];
        p.y = ctx->buf[1 - b];
        p.w = ctx->w;
        p.f = ctx->f;
        p.st_in = ctx->st + b;
        p.st_out = ctx->st + (1 - b);
        p.T = c.T;
        p.Wp = L.Wp;
        p.PT = L.PT;
        p.PL = L.PL;
        p.frame = L.frame;
        p.fstride = L.total;
        axis_taps(c.r_s, c.sigma_s, p.gs);
        axis_taps(c.r_t, c.sigma_t, p.gt);
        p.alpha = (float)c.alpha;
    }
    int shape = 0, chunks = 1;
    int rc = default_plan(ctx, &shape, &chunks);
    if (rc != SFSEG_OK) return rc;
    rc = install_plan(ctx, shape, chunks);
    if (rc != SFSEG_OK) return rc;
    return run_prep(ctx, S, F);
}

// Gain that keeps the stored iterate values O(1): sqrt(N) / sum of all taps.
// For w <= 1 and |1 - alpha dF^2| <= 1, sum(G) bounds lambda, so stored
// values stay below sqrt(N) * max|x_i| <= sqrt(N).
double storage_gain(const sfseg_config& c, int64_t n) {
    double st = 0.0, ss = 0.0;
    for (int d = -c.r_t; d <= c.r_t; ++d) st += exp(-(double)d * d / (2.0 * c.sigma_t * c.sigma_t));
    for (int d = -c.r_s; d <= c.r_s; ++d) ss += exp(-(double)d * d / (2.0 * c.sigma_s * c.sigma_s));
    return sqrt((double)n) / (st * ss * ss);
}

// Copy the start vector into Y_0 and reset the iteration state: tolerance,
// step budget and storage gain from the host, the rest from init_kernel.
// `h_st` is pinned host memory that stays untouched until the stream has
// passed this point.
int run_init(hipStream_t stream, const sfseg_config& c, const sfseg::Layout& L, int64_t n,
             const void* src, int src_is_storage, void* y0, DevState* st, DevState* h_st,
             double* partials, int grid, int32_t max_iters, double tol) {
    DevState h{};
    h.tol = tol;
    h.max_iters = max_iters;
    h.gain = storage_gain(c, n);
    h.delta = INFINITY;
    *h_st = h;
    HIP_TRY(hipMemcpyAsync(st, h_st, sizeof(DevState), hipMemcpyHostToDevice, stream));
    HIP_TRY(sfseg::launch_init(c.storage, src, src_is_storage, y0, L, st, partials, grid, stream));
    return SFSEG_OK;
}

int launch_steps(sfseg_ctx* ctx, int first_buf, int count, int* last_buf) {
    // one launch per step, or per two steps with the fused kernel (an odd
    // last step in its one-step mode); launches alternate the two buffers
    const int per = sfseg::steps_per_launch(ctx->shape);
    int b = first_buf & 1;
    for (int done = 0; done < count;) {
        sfseg::StepParams p = ctx->params[b];
        p.half = count - done < per ? 1 : 0;
        HIP_TRY(sfseg::launch_step(ctx->cfg.storage, sfseg::kernel_shape(ctx->shape, ctx->nf),
                                   ctx->cfg.r_s, ctx->cfg.r_t, p, ctx->step_grid, ctx->stream));
        done += p.half ? 1 : per;
        b ^= 1;
    }
    if (last_buf) *last_buf = b;
    return SFSEG_OK;
}

int launch_finish(sfseg_ctx* ctx, int slot) {
    HIP_TRY(sfseg::launch_step_finish(ctx->st, slot & 1,
                                      ctx->step_part + 4 * (size_t)ctx->step_part_slots * (slot & 1),
                                      ctx->step_grid, ctx->stream));
    return SFSEG_OK;
}

// Buffer that holds the iterate after k steps from buf[0]: launches
// alternate the buffers, and the fused kernel takes two steps per launch
// (only the last launch of a run can take one).
int buffer_after(const sfseg_ctx* ctx, int k) {
    return sfseg::steps_per_launch(ctx->shape) == 2 ? ((k + 1) / 2) & 1 : k & 1;
}

// kChunk steps from buf[0] (kChunk / 2 is even as well, so with one or two
// steps per launch they end in buf[0]) and the fold of the last one.
static_assert(kChunk % 4 == 0, "a captured chunk must end in buf[0]");
int ensure_graph(sfseg_ctx* ctx) {
    if (ctx->graph) return SFSEG_OK;
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    int last = 0;
    int rc = launch_steps(ctx, 0, kChunk, &last);
    if (rc == SFSEG_OK) rc = launch_finish(ctx, last);
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    if (rc != SFSEG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(SFSEG_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&ctx->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        ctx->graph = nullptr;
        return fail(SFSEG_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return SFSEG_OK;
}

}  // namespace sfseg_host

extern "C" {

int sfseg_create_mc(const sfseg_config* cfg, const float* S, const float* F, int32_t n_features,
                    void* stream, sfseg_ctx** out) {
    if (!out) return fail(SFSEG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int rc = sfseg_config_validate(cfg);
    if (rc != SFSEG_OK) return rc;
    if (!S) return fail(SFSEG_ERR_INVALID_ARG, "S is NULL");
    if (n_features < 1 || n_features > SFSEG_MAX_FEATURES)
        return fail(SFSEG_ERR_INVALID_ARG, "n_features must be 1..%d", SFSEG_MAX_FEATURES);
    if (n_features > 1 && !F)
        return fail(SFSEG_ERR_INVALID_ARG, "F must hold the %d feature channels", n_features);
    if (n_features > 1 && cfg->storage != SFSEG_F32)
        return fail(SFSEG_ERR_UNSUPPORTED, "several feature channels need float32 storage");
    sfseg_ctx* ctx = new (std::nothrow) sfseg_ctx();
    if (!ctx) return fail(SFSEG_ERR_OOM, "host allocation failed");
    ctx->nf = n_features;
    ctx->cfg = *cfg;
    ctx->stream = (hipStream_t)stream;
    ctx->n = (int64_t)cfg->T * cfg->H * cfg->W;
    rc = setup(ctx, S, F);
    if (rc != SFSEG_OK) {
        char keep[sizeof(g_err)];
        memcpy(keep, g_err, sizeof(keep));
        sfseg_destroy(ctx);
        memcpy(g_err, keep, sizeof(keep));
        return rc;
    }
    *out = ctx;
    return SFSEG_OK;
}

int sfseg_create(const sfseg_config* cfg, const float* S, const float* F, void* stream,
                 sfseg_ctx** out) {
    return sfseg_create_mc(cfg, S, F, 1, stream, out);
}

int sfseg_set_features(sfseg_ctx* ctx, const float* S, const float* F) {
    if (!ctx) return fail(SFSEG_ERR_INVALID_ARG, "ctx is NULL");
    if (ctx->batch) return fail(SFSEG_ERR_STATE, "batch context: use the sfseg_batch_* calls");
    if (!S) return fail(SFSEG_ERR_INVALID_ARG, "S is NULL");
    if (ctx->nf > 1 && !F)
        return fail(SFSEG_ERR_INVALID_ARG, "F must hold the %d feature channels", ctx->nf);
    HIP_TRY(hipSetDevice(ctx->device));
    return run_prep(ctx, S, F);
}

int sfseg_power_iterate(sfseg_ctx* ctx, const float* x0, int32_t max_iters, double tol,
                        sfseg_result* res) {
    if (!ctx) return fail(SFSEG_ERR_INVALID_ARG, "ctx is NULL");
    if (ctx->batch) return fail(SFSEG_ERR_STATE, "batch context: use the sfseg_batch_* calls");
    if (max_iters < 0) return fail(SFSEG_ERR_INVALID_ARG, "max_iters must be >= 0");
    if (isnan(tol)) return fail(SFSEG_ERR_INVALID_ARG, "tol is NaN");
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->have_iterate = false;

    HIP_TRY(hipEventRecord(ctx->ev[0], ctx->stream));
    int rc0 = run_init(ctx->stream, ctx->cfg, ctx->L, ctx->n, x0 ? (const void*)x0 : ctx->s0,
                       x0 ? 0 : 1, ctx->buf[0], ctx->st, ctx->h_st, ctx->partials, ctx->ew_grid,
                       max_iters, tol);
    if (rc0 != SFSEG_OK) return rc0;
    HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));

    // Keep up to two chunks in flight: while chunk i runs, chunk i+1 is queued
    // and the host inspects the state copied out after chunk i-1.
    int launched = 0, enq = 0, chk = 0;
    int cur = 0;  // buffer holding the iterate after `launched` steps
    const bool use_graph = ctx->stream != nullptr && ensure_graph(ctx) == SFSEG_OK;
    while (true) {
        while (enq - chk < 2 && launched < max_iters) {
            const int remaining = max_iters - launched;
            if (use_graph && remaining >= kChunk && cur == 0) {
                HIP_TRY(hipGraphLaunch(ctx->graph, ctx->stream));
                launched += kChunk;
            } else {
                const int cnt = remaining < kChunk ? remaining : kChunk;
                int rc = launch_steps(ctx, cur, cnt, &cur);
                if (rc == SFSEG_OK) rc = launch_finish(ctx, cur);
                if (rc != SFSEG_OK) return rc;
                launched += cnt;
            }
            HIP_TRY(hipMemcpyAsync(ctx->h_st + 1 + (enq & 1), ctx->st, sizeof(DevState),
                                   hipMemcpyDeviceToHost, ctx->stream));
            HIP_TRY(hipEventRecord(ctx->ev[3 + (enq & 1)], ctx->stream));
            ++enq;
        }
        if (chk == enq) break;
        HIP_TRY(hipEventSynchronize(ctx->ev[3 + (chk & 1)]));
        const bool done = ctx->h_st[1 + (chk & 1)].done != 0;
        ++chk;
        if (done) break;
    }
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
    ctx->timing.launches = launched;

    if (res) {
        res->iters = s.k;
        res->converged = s.converged;
        res->delta = s.delta;
        res->lambda = s.lambda;
    }
    if (s.status != SFSEG_OK) {
        return fail(s.status, s.status == SFSEG_ERR_ZERO_NORM
                                  ? "zero norm (start vector or iterate %d)"
                                  : "non-finite value (start vector or iterate %d)",
                    s.k);
    }
    ctx->cur = buffer_after(ctx, s.k);
    ctx->have_iterate = true;
    return SFSEG_OK;
}

int sfseg_eigvec(sfseg_ctx* ctx, float* out) {
    if (!ctx || !out) return fail(SFSEG_ERR_INVALID_ARG, "ctx or out is NULL");
    if (ctx->batch) return fail(SFSEG_ERR_STATE, "batch context: use sfseg_batch_eigvec");
    if (!ctx->have_iterate) return fail(SFSEG_ERR_STATE, "no iterate: call sfseg_power_iterate first");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(sfseg::launch_eigvec(ctx->cfg.storage, ctx->buf[ctx->cur], ctx->st, out, ctx->L,
                                 ctx->ew_grid, ctx->stream));
    return SFSEG_OK;
}

int sfseg_apply(sfseg_ctx* ctx, const float* x, float* y) {
    if (!ctx || !x || !y) return fail(SFSEG_ERR_INVALID_ARG, "ctx, x or y is NULL");
    if (ctx->batch) return fail(SFSEG_ERR_STATE, "batch context: sfseg_apply works on one clip");
    if (x == (const float*)y) return fail(SFSEG_ERR_INVALID_ARG, "x and y may not alias");
    HIP_TRY(hipSetDevice(ctx->device));
    if (int rc = sfseg_host::apply_async(ctx, x, y)) return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SFSEG_OK;
}

}  // extern "C"

namespace sfseg_host {

// y = M x on the context's stream, through the staging volumes (allocated on
// the first call); does not wait.
int apply_async(sfseg_ctx* ctx, const float* x, float* y) {
    const size_t bytes = (size_t)ctx->L.total * dtype_size(ctx->cfg.storage);
    if (!ctx->apply_in) {
        HIP_TRY(hipMalloc(&ctx->apply_in, bytes));
        HIP_TRY(hipMemsetAsync(ctx->apply_in, 0, bytes, ctx->stream));
    }
    if (!ctx->apply_out) {
        HIP_TRY(hipMalloc(&ctx->apply_out, bytes));
        HIP_TRY(hipMemsetAsync(ctx->apply_out, 0, bytes, ctx->stream));
    }
    DevState h{};
    h.s = 1.0;
    h.c = 1.0f;
    h.gain = 1.0;
    h.tol = -1.0;
    h.max_iters = 1;
    *ctx->h_st = h;
    HIP_TRY(hipMemcpyAsync(ctx->st_apply, ctx->h_st, sizeof(DevState), hipMemcpyHostToDevice,
                           ctx->stream));  // slot 0: nothing pending
    HIP_TRY(sfseg::launch_to_storage(ctx->cfg.storage, x, ctx->apply_in, ctx->L, ctx->ew_grid,
                                     ctx->stream));
    StepParams p = ctx->params[0];
    p.x = ctx->apply_in;
    p.y = ctx->apply_out;
    p.st_in = ctx->st_apply;
    p.st_out = ctx->st_apply + 1;
    p.half = 1;  // one application (the fused kernel's one-step mode)
    HIP_TRY(sfseg::launch_step(ctx->cfg.storage, sfseg::kernel_shape(ctx->shape, ctx->nf),
                               ctx->cfg.r_s, ctx->cfg.r_t, p,
                               ctx->step_grid, ctx->stream));
    HIP_TRY(sfseg::launch_from_storage(ctx->cfg.storage, ctx->apply_out, y, ctx->L, ctx->ew_grid,
                                       ctx->stream));
    return SFSEG_OK;
}

}  // namespace sfseg_host

extern "C" {

int sfseg_get_plan(const sfseg_ctx* ctx, sfseg_plan* out) {
    if (!ctx || !out) return fail(SFSEG_ERR_INVALID_ARG, "ctx or out is NULL");
    if (ctx->batch) return batch_get_plan(ctx, out);
    out->shape = ctx->shape;
    out->chunks = ctx->chunks;
    out->blocks = ctx->step_grid;
    out->threads = sfseg::step_threads(ctx->shape);
    return SFSEG_OK;
}

int sfseg_set_plan(sfseg_ctx* ctx, int32_t shape, int32_t chunks) {
    if (!ctx) return fail(SFSEG_ERR_INVALID_ARG, "ctx is NULL");
    if (ctx->batch) return batch_set_plan(ctx, shape, chunks);
    if (shape < 0 || shape >= sfseg::STEP_SHAPES)
        return fail(SFSEG_ERR_INVALID_ARG, "shape must be 0..%d", sfseg::STEP_SHAPES - 1);
    if (!sfseg::shape_supported(shape, ctx->cfg.storage, ctx->nf, ctx->cfg.r_s, ctx->cfg.r_t,
                                false))
        return fail(SFSEG_ERR_UNSUPPORTED,
                    "shape %d needs float32 storage, one feature channel and radii within "
                    "its limits (r_t <= %d; fused: r_s <= %d, r_t <= %d)",
                    shape, sfseg::MFMA_MAX_RT, sfseg::FUSED_MAX_RS, sfseg::FUSED_MAX_RT);
    if (chunks == 0 && shape > 1)
        return fail(SFSEG_ERR_UNSUPPORTED, "the balanced plan (chunks = 0) is for shapes 0 and 1");
    if (chunks < 0 || chunks > max_chunks(ctx->cfg))
        return fail(SFSEG_ERR_INVALID_ARG, "chunks must be 1..%d for this clip", max_chunks(ctx->cfg));
    HIP_TRY(hipSetDevice(ctx->device));
    return install_plan(ctx, shape, chunks);
}

int sfseg_last_timing(const sfseg_ctx* ctx, sfseg_timing* out) {
    if (!ctx || !out) return fail(SFSEG_ERR_INVALID_ARG, "ctx or out is NULL");
    *out = ctx->timing;
    return SFSEG_OK;
}

}  // extern "C"

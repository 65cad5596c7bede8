// Batched power iteration: many clips of uneven size iterated together by one
// persistent launch per step (declared in include/sfseg.h).
//
// Every clip keeps its own padded volumes and iteration state; the batched
// step kernel walks a shared work list of (clip, tile, frame run) items and
// advances each clip independently, so a clip that has converged is skipped
// by the following launches.  All clips share the graph parameters (radii,
// widths, alpha, p, storage) -- they are one workload cut into clips.
//
// sfseg_autotune, for single-clip and batch contexts alike, times a few
// steps of each candidate work plan and keeps the fastest.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "host_internal.h"

using sfseg::BatchClip;
using sfseg::BatchParams;
using sfseg::DevState;
using namespace sfseg_host;

namespace sfseg_host {

struct ClipBuffers {
    sfseg_config cfg{};
    sfseg::Layout L{};
    int64_t n = 0;
    void* w = nullptr;
    void* f = nullptr;
    void* s0 = nullptr;
    void* buf[2] = {nullptr, nullptr};
    DevState* st = nullptr;
};

struct BatchState {
    std::vector<ClipBuffers> clips;
    BatchClip* d_clips = nullptr;
    int4* d_items = nullptr;
    size_t items_cap = 0;
    double* d_partials = nullptr;
    size_t partials_cap = 0;  // doubles
    uint32_t* d_queue = nullptr;  // 9 counters
    DevState* h_st = nullptr;     // pinned: 3 slots per clip ([0] final, [1..2] per chunk)
    std::vector<BatchClip> h_clips;
    BatchParams params[2]{};  // parity 0 and 1
    int n_items = 0;
    int grid = 0;
    hipGraphExec_t graph = nullptr;  // kChunk launches, parity 0, 1, 0, ...
};

void destroy_batch(BatchState* b) {
    if (!b) return;
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (auto& c : b->clips) {
        void* p[] = {c.w, c.f, c.s0, c.buf[0], c.buf[1], c.st};
        for (void* q : p)
            if (q) (void)hipFree(q);
    }
    void* p[] = {b->d_clips, b->d_items, b->d_partials, b->d_queue};
    for (void* q : p)
        if (q) (void)hipFree(q);
    if (b->h_st) (void)hipHostFree(b->h_st);
    delete b;
}

namespace {

// Work list of the whole batch: clip by clip, each clip's frames cut into
// `chunks` runs (at most what the clip allows), then tile rows and columns.
// The list is split into 8 contiguous runs of about equal work (frames per
// item, warm-up included), one per XCD queue.
int build_items(sfseg_ctx* ctx, int chunks) {
    BatchState& b = *ctx->batch;
    std::vector<int4> items;
    std::vector<double> work;
    for (size_t c = 0; c < b.clips.size(); ++c) {
        const ClipBuffers& cl = b.clips[c];
        const int ch = std::min(chunks, max_chunks(cl.cfg));
        const int first = (int)items.size();
        for (int k = 0; k < ch; ++k) {
            const int t0 = (int)((int64_t)cl.L.T * k / ch), t1 = (int)((int64_t)cl.L.T * (k + 1) / ch);
            for (int ty = 0; ty < cl.L.tiles_y; ++ty)
                for (int tx = 0; tx < cl.L.tiles_x; ++tx) {
                    items.push_back(make_int4((int)c, (tx * sfseg::TILE_X) | ((ty * sfseg::TILE_Y) << 16),
                                              t0, t1));
                    work.push_back((double)(t1 - t0 + 2 * cl.cfg.r_t));
                }
        }
        b.h_clips[c].first_item = first;
        b.h_clips[c].n_items = (int)items.size() - first;
    }
    const int n = (int)items.size();
    if (items.size() > b.items_cap) {
        if (b.d_items) HIP_TRY(hipFree(b.d_items));
        b.d_items = nullptr;
        HIP_TRY(hipMalloc((void**)&b.d_items, sizeof(int4) * items.size()));
        b.items_cap = items.size();
    }
    const size_t need = 2 * (size_t)std::max(n, ctx->ew_grid);
    if (need > b.partials_cap) {
        if (b.d_partials) HIP_TRY(hipFree(b.d_partials));
        b.d_partials = nullptr;
        HIP_TRY(hipMalloc((void**)&b.d_partials, sizeof(double) * need));
        b.partials_cap = need;
    }
    HIP_TRY(hipMemcpyAsync(b.d_items, items.data(), sizeof(int4) * items.size(),
                           hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(b.d_clips, b.h_clips.data(), sizeof(BatchClip) * b.h_clips.size(),
                           hipMemcpyHostToDevice, ctx->stream));
    // split into 8 runs of about equal work
    double total = 0.0;
    for (double w : work) total += w;
    int32_t qfirst[8], qcount[8];
    int start = 0;
    double acc = 0.0;
    for (int x = 0; x < 8; ++x) {
        int end = start;
        const double goal = total * (x + 1) / 8.0;
        while (end < n && (x == 7 || acc + work[end] * 0.5 <= goal)) acc += work[end++];
        qfirst[x] = start;
        qcount[x] = end - start;
        start = end;
    }
    for (auto& p : b.params) {
        p.items = b.d_items;
        p.partials = b.d_partials;
        memcpy(p.qfirst, qfirst, sizeof(qfirst));
        memcpy(p.qcount, qcount, sizeof(qcount));
    }
    b.n_items = n;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SFSEG_OK;
}

int install_batch_plan(sfseg_ctx* ctx, int shape, int chunks) {
    BatchState& b = *ctx->batch;
    const sfseg_config& c = ctx->cfg;
    int occ = 1;
    HIP_TRY(sfseg::batch_max_blocks_per_cu(c.storage, shape, c.r_s, c.r_t, &occ));
    if (occ < 1) occ = 1;
    ctx->shape = shape;
    ctx->chunks = chunks;
    int rc = build_items(ctx, chunks);
    if (rc != SFSEG_OK) return rc;
    // persistent grid: every resident slot, a multiple of 8 (one share per XCD)
    b.grid = std::max(8, (ctx->cus * occ) / 8 * 8);
    ctx->step_grid = b.grid;
    if (b.graph) {
        (void)hipGraphExecDestroy(b.graph);
        b.graph = nullptr;
    }
    return SFSEG_OK;
}

int launch_batch_steps(sfseg_ctx* ctx, int first_parity, int count) {
    BatchState& b = *ctx->batch;
    for (int i = 0; i < count; ++i) {
        HIP_TRY(sfseg::launch_batch_step(ctx->cfg.storage, ctx->shape, ctx->cfg.r_s, ctx->cfg.r_t,
                                         b.params[(first_parity + i) & 1], b.grid, ctx->stream));
        HIP_TRY(sfseg::launch_batch_finish(b.d_clips, (int)b.h_clips.size(), b.d_partials,
                                           b.d_queue, ctx->stream));
    }
    return SFSEG_OK;
}

int ensure_batch_graph(sfseg_ctx* ctx) {
    BatchState& b = *ctx->batch;
    if (b.graph) return SFSEG_OK;
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    int rc = launch_batch_steps(ctx, 0, kChunk);
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    if (rc != SFSEG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(SFSEG_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b.graph = nullptr;
        return fail(SFSEG_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return SFSEG_OK;
}

int check_batch(const sfseg_ctx* ctx) {
    if (!ctx) return fail(SFSEG_ERR_INVALID_ARG, "ctx is NULL");
    if (!ctx->batch) return fail(SFSEG_ERR_STATE, "not a batch context (made by sfseg_create)");
    return SFSEG_OK;
}

}  // namespace

int batch_get_plan(const sfseg_ctx* ctx, sfseg_plan* out) {
    out->shape = ctx->shape;
    out->chunks = ctx->chunks;
    out->blocks = ctx->batch->grid;
    out->threads = sfseg::step_threads(ctx->shape);
    return SFSEG_OK;
}

int batch_set_plan(sfseg_ctx* ctx, int32_t shape, int32_t chunks) {
    if (shape < 0 || shape >= sfseg::STEP_SHAPES)
        return fail(SFSEG_ERR_INVALID_ARG, "shape must be 0..%d", sfseg::STEP_SHAPES - 1);
    if (!sfseg::shape_supported(shape, ctx->cfg.storage, ctx->nf, ctx->cfg.r_s, ctx->cfg.r_t, true))
        return fail(SFSEG_ERR_UNSUPPORTED, "shape %d is not available for batches", shape);
    int most = 1;
    for (auto& c : ctx->batch->clips) most = std::max(most, max_chunks(c.cfg));
    if (chunks < 1 || chunks > most)
        return fail(SFSEG_ERR_INVALID_ARG, "chunks must be 1..%d for this batch", most);
    HIP_TRY(hipSetDevice(ctx->device));
    return install_batch_plan(ctx, shape, chunks);
}

}  // namespace sfseg_host

extern "C" {

int sfseg_batch_create(const sfseg_config* cfgs, int32_t n, const float* const* S,
                       const float* const* F, void* stream, sfseg_ctx** out) {
    if (!out) return fail(SFSEG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cfgs || !S || n < 1) return fail(SFSEG_ERR_INVALID_ARG, "cfgs, S or n invalid");
    for (int i = 0; i < n; ++i) {
        int rc = sfseg_config_validate(&cfgs[i]);
        if (rc != SFSEG_OK) return rc;
        if (!S[i]) return fail(SFSEG_ERR_INVALID_ARG, "S[%d] is NULL", i);
        const sfseg_config& a = cfgs[0];
        const sfseg_config& c = cfgs[i];
        if (c.r_t != a.r_t || c.r_s != a.r_s || c.sigma_t != a.sigma_t || c.sigma_s != a.sigma_s ||
            c.alpha != a.alpha || c.p != a.p || c.storage != a.storage)
            return fail(SFSEG_ERR_INVALID_ARG,
                        "clip %d: every clip of a batch must share r_t, r_s, sigmas, alpha, p and "
                        "storage", i);
    }
    sfseg_ctx* ctx = new (std::nothrow) sfseg_ctx();
    if (!ctx) return fail(SFSEG_ERR_OOM, "host allocation failed");
    ctx->batch = new (std::nothrow) BatchState();
    if (!ctx->batch) {
        delete ctx;
        return fail(SFSEG_ERR_OOM, "host allocation failed");
    }
    ctx->cfg = cfgs[0];
    ctx->stream = (hipStream_t)stream;
    auto body = [&]() -> int {
        BatchState& b = *ctx->batch;
        HIP_TRY(hipGetDevice(&ctx->device));
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, ctx->device));
        ctx->cus = prop.multiProcessorCount;
        ctx->ew_grid = ctx->cus * 8;
        HIP_TRY(hipMalloc((void**)&ctx->d_bad, sizeof(int32_t)));
        HIP_TRY(hipHostMalloc((void**)&ctx->h_bad, sizeof(int32_t), hipHostMallocDefault));
        for (auto& e : ctx->ev) HIP_TRY(hipEventCreate(&e));
        HIP_TRY(hipHostMalloc((void**)&b.h_st, 3 * sizeof(DevState) * n, hipHostMallocDefault));
        HIP_TRY(hipMalloc((void**)&b.d_clips, sizeof(BatchClip) * n));
        HIP_TRY(hipMalloc((void**)&b.d_queue, sizeof(uint32_t) * 9));
        HIP_TRY(hipMemsetAsync(b.d_queue, 0, sizeof(uint32_t) * 9, ctx->stream));
        HIP_TRY(hipMemsetAsync(ctx->d_bad, 0, sizeof(int32_t), ctx->stream));
        b.clips.resize(n);
        b.h_clips.resize(n);
        for (int i = 0; i < n; ++i) {
            ClipBuffers& cl = b.clips[i];
            cl.cfg = cfgs[i];
            cl.L = make_layout(cfgs[i]);
            cl.n = (int64_t)cfgs[i].T * cfgs[i].H * cfgs[i].W;
            if (cl.L.total * (int64_t)dtype_size(cl.cfg.storage) >= ((int64_t)1 << 31))
                return fail(SFSEG_ERR_INVALID_ARG, "clip %d: padded volume exceeds 2 GiB", i);
            const size_t bytes = (size_t)cl.L.total * dtype_size(cl.cfg.storage);
            void** vols[] = {&cl.w, &cl.f, &cl.s0, &cl.buf[0], &cl.buf[1]};
            for (void** v : vols) {
                HIP_TRY(hipMalloc(v, bytes));
                HIP_TRY(hipMemsetAsync(*v, 0, bytes, ctx->stream));
            }
            HIP_TRY(hipMalloc((void**)&cl.st, sizeof(DevState)));
            HIP_TRY(hipMemsetAsync(cl.st, 0, sizeof(DevState), ctx->stream));
            HIP_TRY(sfseg::launch_prep(cl.cfg.storage, S[i], F ? F[i] : nullptr, cl.cfg.p, cl.w, cl.f,
                                       cl.s0, cl.L, ctx->d_bad, ctx->ew_grid, ctx->stream));
            BatchClip& h = b.h_clips[i];
            h.buf[0] = cl.buf[0];
            h.buf[1] = cl.buf[1];
            h.w = cl.w;
            h.f = cl.f;
            h.st = cl.st;
            h.frame = cl.L.frame;
            h.T = cl.L.T;
            h.Wp = cl.L.Wp;
            h.PT = cl.L.PT;
            h.PL = cl.L.PL;
        }
        for (int par = 0; par < 2; ++par) {
            BatchParams& p = b.params[par];
            memset(&p, 0, sizeof(p));
            p.clips = b.d_clips;
            p.queue = b.d_queue;
            p.parity = par;
            axis_taps(ctx->cfg.r_s, ctx->cfg.sigma_s, p.gs);
            axis_taps(ctx->cfg.r_t, ctx->cfg.sigma_t, p.gt);
            p.alpha = (float)ctx->cfg.alpha;
        }
        int rc = install_batch_plan(ctx, 0, 1);
        if (rc != SFSEG_OK) return rc;
        HIP_TRY(hipMemcpyAsync(ctx->h_bad, ctx->d_bad, sizeof(int32_t), hipMemcpyDeviceToHost,
                               ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        if (*ctx->h_bad)
            return fail(SFSEG_ERR_NONFINITE, "a clip's S or F holds NaN/Inf, or S < 0 with p > 0");
        return SFSEG_OK;
    };
    int rc = body();
    if (rc != SFSEG_OK) {
        char keep[512];
        strncpy(keep, sfseg_last_error(), sizeof(keep) - 1);
        keep[sizeof(keep) - 1] = 0;
        sfseg_destroy(ctx);
        fail(rc, "%s", keep);
        return rc;
    }
    *out = ctx;
    return SFSEG_OK;
}

int sfseg_batch_size(const sfseg_ctx* ctx, int32_t* n) {
    int rc = check_batch(ctx);
    if (rc != SFSEG_OK) return rc;
    if (!n) return fail(SFSEG_ERR_INVALID_ARG, "n is NULL");
    *n = (int32_t)ctx->batch->clips.size();
    return SFSEG_OK;
}

int sfseg_batch_iterate(sfseg_ctx* ctx, const float* const* x0, int32_t max_iters, double tol,
                        sfseg_result* res) {
    int rc = check_batch(ctx);
    if (rc != SFSEG_OK) return rc;
    if (max_iters < 0) return fail(SFSEG_ERR_INVALID_ARG, "max_iters must be >= 0");
    if (isnan(tol)) return fail(SFSEG_ERR_INVALID_ARG, "tol is NaN");
    HIP_TRY(hipSetDevice(ctx->device));
    BatchState& b = *ctx->batch;
    const int n = (int)b.clips.size();
    ctx->have_iterate = false;

    HIP_TRY(hipEventRecord(ctx->ev[0], ctx->stream));
    for (int i = 0; i < n; ++i) {
        ClipBuffers& cl = b.clips[i];
        const float* src = x0 ? x0[i] : nullptr;
        rc = run_init(ctx->stream, cl.cfg, cl.L, cl.n, src ? (const void*)src : cl.s0, src ? 0 : 1,
                      cl.buf[0], cl.st, b.h_st + 3 * i, b.d_partials, ctx->ew_grid, max_iters, tol);
        if (rc != SFSEG_OK) return rc;
    }
    HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));

    // Same pipelining as the single-clip loop: up to two chunks in flight;
    // the batch is done when every clip's state says so.
    int launched = 0, enq = 0, chk = 0;
    const bool use_graph = ctx->stream != nullptr && ensure_batch_graph(ctx) == SFSEG_OK;
    while (true) {
        while (enq - chk < 2 && launched < max_iters) {
            const int remaining = max_iters - launched;
            if (use_graph && remaining >= kChunk && (launched & 1) == 0) {
                HIP_TRY(hipGraphLaunch(b.graph, ctx->stream));
                launched += kChunk;
            } else {
                const int cnt = remaining < kChunk ? remaining : kChunk;
                rc = launch_batch_steps(ctx, launched & 1, cnt);
                if (rc != SFSEG_OK) return rc;
                launched += cnt;
            }
            for (int i = 0; i < n; ++i)
                HIP_TRY(hipMemcpyAsync(b.h_st + 3 * i + 1 + (enq & 1), b.clips[i].st,
                                       sizeof(DevState), hipMemcpyDeviceToHost, ctx->stream));
            HIP_TRY(hipEventRecord(ctx->ev[3 + (enq & 1)], ctx->stream));
            ++enq;
        }
        if (chk == enq) break;
        HIP_TRY(hipEventSynchronize(ctx->ev[3 + (chk & 1)]));
        bool all_done = true;
        for (int i = 0; i < n; ++i) all_done = all_done && b.h_st[3 * i + 1 + (chk & 1)].done;
        ++chk;
        if (all_done) break;
    }
    HIP_TRY(hipEventRecord(ctx->ev[2], ctx->stream));
    for (int i = 0; i < n; ++i)
        HIP_TRY(hipMemcpyAsync(b.h_st + 3 * i, b.clips[i].st, sizeof(DevState),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));

    float t_init = 0.f, t_all = 0.f;
    HIP_TRY(hipEventElapsedTime(&t_init, ctx->ev[0], ctx->ev[1]));
    HIP_TRY(hipEventElapsedTime(&t_all, ctx->ev[0], ctx->ev[2]));
    ctx->timing.total_ms = t_all;
    ctx->timing.init_ms = t_init;
    ctx->timing.loop_ms = t_all - t_init;
    ctx->timing.launches = launched;
    int most = 0, status = SFSEG_OK, bad = -1;
    for (int i = 0; i < n; ++i) {
        const DevState& s = b.h_st[3 * i];
        most = std::max(most, s.k);
        if (res) {
            res[i].iters = s.k;
            res[i].converged = s.converged;
            res[i].delta = s.delta;
            res[i].lambda = s.lambda;
        }
        if (s.status != SFSEG_OK && status == SFSEG_OK) {
            status = s.status;
            bad = i;
        }
    }
    ctx->timing.iters = most;
    if (status != SFSEG_OK)
        return fail(status, "clip %d: %s", bad, sfseg_status_string(status));
    ctx->have_iterate = true;
    return SFSEG_OK;
}

int sfseg_batch_eigvec(sfseg_ctx* ctx, float* const* out) {
    int rc = check_batch(ctx);
    if (rc != SFSEG_OK) return rc;
    if (!out) return fail(SFSEG_ERR_INVALID_ARG, "out is NULL");
    if (!ctx->have_iterate)
        return fail(SFSEG_ERR_STATE, "no iterate: call sfseg_batch_iterate first");
    HIP_TRY(hipSetDevice(ctx->device));
    BatchState& b = *ctx->batch;
    for (size_t i = 0; i < b.clips.size(); ++i) {
        if (!out[i]) return fail(SFSEG_ERR_INVALID_ARG, "out[%d] is NULL", (int)i);
        ClipBuffers& cl = b.clips[i];
        const int k = b.h_st[3 * i].k;
        HIP_TRY(sfseg::launch_eigvec(cl.cfg.storage, cl.buf[k & 1], cl.st, out[i], cl.L,
                                     ctx->ew_grid, ctx->stream));
    }
    return SFSEG_OK;
}

int sfseg_autotune(sfseg_ctx* ctx, int32_t steps, sfseg_plan* best) {
    if (!ctx) return fail(SFSEG_ERR_INVALID_ARG, "ctx is NULL");
    if (steps < 1) return fail(SFSEG_ERR_INVALID_ARG, "steps must be >= 1");
    HIP_TRY(hipSetDevice(ctx->device));
    int most = 1;
    if (ctx->batch) {
        for (auto& c : ctx->batch->clips) most = std::max(most, max_chunks(c.cfg));
    } else {
        most = max_chunks(ctx->cfg);
    }
    double best_ms = 1e300;
    int best_shape = ctx->shape, best_chunks = ctx->chunks;
    // frame runs per tile; 0 = the balanced work list (single clips, shapes 0, 1)
    const int chunk_opts[] = {1, 2, 3, 4, 0};
    for (int shape = 0; shape < sfseg::STEP_SHAPES; ++shape) {
        if (!sfseg::shape_supported(shape, ctx->cfg.storage, ctx->nf, ctx->cfg.r_s, ctx->cfg.r_t,
                                    ctx->batch != nullptr))
            continue;
        for (int ch : chunk_opts) {
            if (ch > most || (ch == 0 && (ctx->batch || shape > 1))) continue;
            int rc = sfseg_set_plan(ctx, shape, ch);
            if (rc != SFSEG_OK && ch == 0) continue;  // the clip is too small for it
            if (rc != SFSEG_OK) return rc;
            double ms = 1e300;
            for (int rep = 0; rep < 2; ++rep) {  // first run warms caches and captures the graph
                rc = ctx->batch ? sfseg_batch_iterate(ctx, nullptr, steps, 0.0, nullptr)
                                : sfseg_power_iterate(ctx, nullptr, steps, 0.0, nullptr);
                if (rc != SFSEG_OK) return rc;
                ms = std::min(ms, ctx->timing.loop_ms);
            }
            if (ms < best_ms) {
                best_ms = ms;
                best_shape = shape;
                best_chunks = ch;
            }
        }
    }
    int rc = sfseg_set_plan(ctx, best_shape, best_chunks);
    if (rc != SFSEG_OK) return rc;
    ctx->have_iterate = false;
    if (best) return sfseg_get_plan(ctx, best);
    return SFSEG_OK;
}

}  // extern "C"

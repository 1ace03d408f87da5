// api.hip -- C ABI entry points of libgsn (declared in include/gsn.h).
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <set>
#include <utility>
#include <vector>

#include "gsn_internal.h"

// Set on the host thread that is capturing a context's stream into a graph: buffers may not grow
// then (an allocation is not part of the graph, and the graph keeps the addresses it captured).
static thread_local bool t_capturing = false;

hipError_t buf_reserve(DevBuf& b, size_t bytes) {
    if (bytes <= b.bytes && b.p) return hipSuccess;
    if (t_capturing) return hipErrorStreamCaptureUnsupported;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
        b.p = nullptr;
        b.bytes = 0;
    }
    // round up so repeated small growth does not reallocate every call
    size_t want = bytes + bytes / 8 + 256;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        return e;
    }
    b.bytes = want;
    return hipSuccess;
}

void buf_free(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

StageTimer::StageTimer(gsn_ctx* c, int stage) : ctx(c) {
    if (!ctx || !ctx->prof || ctx->capturing) return;
    ProfRec r;
    r.stage = stage;
    for (hipEvent_t* e : {&r.start, &r.stop}) {
        if (!ctx->pool.empty()) {
            *e = ctx->pool.back();
            ctx->pool.pop_back();
        } else if (hipEventCreate(e) != hipSuccess) {
            return;
        }
    }
    if (hipEventRecord(r.start, ctx->stream) != hipSuccess) return;
    ctx->recs.push_back(r);
    idx = (int)ctx->recs.size() - 1;
}

StageTimer::~StageTimer() {
    if (idx >= 0) (void)hipEventRecord(ctx->recs[idx].stop, ctx->stream);
}

namespace {

gsn_status fail(gsn_ctx* ctx, gsn_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
gsn_status fail(gsn_ctx* ctx, gsn_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) {
        ctx->err = buf;
        if (ctx->capturing) ctx->capture_failed = true;  // the graph would miss this call's work
    }
    return st;
}

#define HIP_TRY(ctx, expr)                                                                                  \
    do {                                                                                                    \
        hipError_t _e = (expr);                                                                             \
        if (_e != hipSuccess)                                                                               \
            return fail(ctx, _e == hipErrorOutOfMemory ? GSN_E_NOMEM : GSN_E_HIP, "%s: %s (%s:%d)", #expr, \
                        hipGetErrorString(_e), __FILE__, __LINE__);                                         \
    } while (0)

DevCam make_devcam(const gsn_camera& c) {
    DevCam d;
    for (int i = 0; i < 9; ++i) d.R[i] = c.R[i];
    for (int i = 0; i < 3; ++i) d.t[i] = c.t[i];
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    for (int i = 0; i < 3; ++i) {
        const double o = -((double)c.R[i] * c.t[0] + (double)c.R[3 + i] * c.t[1] + (double)c.R[6 + i] * c.t[2]);
        d.o[i] = (float)o;
    }
    d.W = c.width;
    d.H = c.height;
    d.tiles_x = (c.width + GSN_TILE - 1) / GSN_TILE;
    d.tiles_y = (c.height + GSN_TILE - 1) / GSN_TILE;
    d.znear = c.znear;
    return d;
}

gsn_status check_gaussians(gsn_ctx* ctx, const gsn_gaussians* g) {
    if (!g) return fail(ctx, GSN_E_INVALID, "gaussians is NULL");
    if (g->n < 0) return fail(ctx, GSN_E_SHAPE, "n = %d < 0", g->n);
    if (g->sh_degree < 0 || g->sh_degree > 3) return fail(ctx, GSN_E_INVALID, "sh_degree %d not in 0..3", g->sh_degree);
    if (g->n > 0 && (!g->d_pos || !g->d_rot || !g->d_scale || !g->d_opac || !g->d_sh))
        return fail(ctx, GSN_E_INVALID, "a gaussian attribute array is NULL");
    if ((int64_t)g->n >= (1ll << 31) / 64) return fail(ctx, GSN_E_CAPACITY, "n = %d too large", g->n);
    return GSN_OK;
}

gsn_status check_camera(gsn_ctx* ctx, const gsn_camera* c) {
    if (!c) return fail(ctx, GSN_E_INVALID, "camera is NULL");
    if (c->width <= 0 || c->height <= 0) return fail(ctx, GSN_E_SHAPE, "image %dx%d", c->width, c->height);
    if ((c->width + GSN_TILE - 1) / GSN_TILE > 65535 || (c->height + GSN_TILE - 1) / GSN_TILE > 65535)
        return fail(ctx, GSN_E_CAPACITY, "image too large");
    if ((int64_t)c->width * c->height > (1ll << 28)) return fail(ctx, GSN_E_CAPACITY, "image too large");
    if (!(c->fx > 0.f) || !(c->fy > 0.f) || !(c->znear > 0.f))
        return fail(ctx, GSN_E_INVALID, "focal lengths and znear must be positive");
    return GSN_OK;
}

}  // namespace

extern "C" {

// The streams and events of gsn_accumulate_views (those created so far).
static void destroy_side(gsn_ctx* c) {
    for (int i = 0; i < gsn_ctx::kSide; ++i) {
        if (c->side[i]) {
            (void)hipStreamSynchronize(c->side[i]);
            (void)hipStreamDestroy(c->side[i]);
        }
        if (c->ev_join[i]) (void)hipEventDestroy(c->ev_join[i]);
    }
    for (int i = 0; i < gsn_ctx::kMaxViews; ++i)
        if (c->ev_chain[i]) (void)hipEventDestroy(c->ev_chain[i]);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
}

gsn_status gsn_create(gsn_ctx** out, int32_t device, void* hip_stream) {
    if (!out) return GSN_E_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return GSN_E_INVALID;
    float* scratch = nullptr;
    if (solve_scratch_address(device, &scratch) != hipSuccess || !scratch) return GSN_E_HIP;
    gsn_ctx* c = new (std::nothrow) gsn_ctx;
    if (!c) return GSN_E_NOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->noalloc_gram = scratch;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess) e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc((void**)&c->d_stats, GSN_STAT_N * sizeof(unsigned long long));
    // default-priority, non-blocking streams for gsn_accumulate_views, and their events
    for (int i = 0; i < gsn_ctx::kSide && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join[i], hipEventDisableTiming);
    }
    for (int i = 0; i < gsn_ctx::kMaxViews && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&c->ev_chain[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) {
        launch_fill_u32(reinterpret_cast<uint32_t*>(c->d_stats), 0u, 2 * GSN_STAT_N, c->stream);
        e = hipStreamSynchronize(c->stream);
    }
    (void)hipSetDevice(cur);
    if (e != hipSuccess) {
        if (c->d_stats) (void)hipFree(c->d_stats);
        destroy_side(c);
        delete c;
        return e == hipErrorOutOfMemory ? GSN_E_NOMEM : GSN_E_HIP;
    }
    *out = c;
    return GSN_OK;
}

gsn_status gsn_destroy(gsn_ctx* ctx) {
    if (!ctx) return GSN_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (const ProfRec& r : ctx->recs) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->d_counts) (void)hipFree(ctx->d_counts);
    if (ctx->d_stats) (void)hipFree(ctx->d_stats);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    destroy_side(ctx);
    buf_free(ctx->mlp_part);
    buf_free(ctx->mlp_stat);
    buf_free(ctx->label_part);
    buf_free(ctx->solve_table);
    buf_free(ctx->gram);
    delete ctx;
    return GSN_OK;
}

gsn_status gsn_profile_enable(gsn_ctx* ctx, int32_t on) {
    if (!ctx) return GSN_E_INVALID;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (const ProfRec& r : ctx->recs) {
        ctx->pool.push_back(r.start);
        ctx->pool.push_back(r.stop);
    }
    ctx->recs.clear();
    if (on && !ctx->d_counts)
        HIP_TRY(ctx, hipMalloc((void**)&ctx->d_counts, GSN_PROF_WORDS * sizeof(unsigned long long)));
    if (ctx->d_counts) launch_fill_u32(reinterpret_cast<uint32_t*>(ctx->d_counts), 0u, 2 * GSN_PROF_WORDS, ctx->stream);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->prof = on != 0;
    ctx->prof_steps = on == 2;
    return GSN_OK;
}

gsn_status gsn_profile_read(gsn_ctx* ctx, double* h_ms, int64_t* h_launches, int64_t* h_counts) {
    if (!ctx) return GSN_E_INVALID;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    double ms[GSN_STAGE_COUNT] = {0};
    int64_t nl[GSN_STAGE_COUNT] = {0};
    for (const ProfRec& r : ctx->recs) {
        float t = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&t, r.start, r.stop));
        ms[r.stage] += t;
        nl[r.stage] += 1;
    }
    for (int i = 0; i < GSN_STAGE_COUNT; ++i) {
        if (h_ms) h_ms[i] = ms[i];
        if (h_launches) h_launches[i] = nl[i];
    }
    if (h_counts) {
        std::vector<unsigned long long> c(GSN_PROF_WORDS, 0ull);
        if (ctx->d_counts)
            HIP_TRY(ctx, hipMemcpy(c.data(), ctx->d_counts, c.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
        for (int r = 0; r < GSN_SOLVE_SPREAD; ++r)
            for (int e = 0; e < GSN_SOLVE_EVENTS; ++e)
                c[GSN_COUNT_SOLVE_ESCALATED + e] += c[GSN_COUNT_N + (size_t)r * GSN_SOLVE_EVENTS + e];
        for (int i = 0; i < GSN_COUNT_N; ++i) h_counts[i] = (int64_t)c[i];
    }
    return GSN_OK;
}

gsn_status gsn_sync_status(gsn_ctx* ctx, int64_t* h_stats) {
    if (!ctx) return GSN_E_INVALID;
    if (ctx->capturing) return fail(ctx, GSN_E_INVALID, "gsn_sync_status while capturing a graph");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    unsigned long long c[GSN_STAT_N] = {0};
    HIP_TRY(ctx, hipMemcpy(c, ctx->d_stats, sizeof c, hipMemcpyDeviceToHost));
    launch_fill_u32(reinterpret_cast<uint32_t*>(ctx->d_stats), 0u, 2 * GSN_STAT_N, ctx->stream);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (h_stats)
        for (int i = 0; i < GSN_STAT_N; ++i) h_stats[i] = (int64_t)c[i];
    if (c[GSN_STAT_PAIR_OVERFLOW])
        return fail(ctx, GSN_E_CAPACITY,
                    "%llu render(s) exceeded the reserved pair capacity (largest need %llu pairs) and drew nothing; "
                    "%llu kernel(s) culled and %llu skipped for non-finite values",
                    c[GSN_STAT_PAIR_OVERFLOW], c[GSN_STAT_PAIRS_NEEDED], c[GSN_STAT_CULLED_NONFINITE],
                    c[GSN_STAT_SKIPPED_NONFINITE]);
    if (c[GSN_STAT_CULLED_NONFINITE] || c[GSN_STAT_SKIPPED_NONFINITE])
        return fail(ctx, GSN_E_NUMERIC, "%llu kernel(s) culled by renders and %llu skipped by solves for NaN or Inf",
                    c[GSN_STAT_CULLED_NONFINITE], c[GSN_STAT_SKIPPED_NONFINITE]);
    ctx->err.clear();
    return GSN_OK;
}

const char* gsn_last_error(const gsn_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gsn_status gsn_set_stream(gsn_ctx* ctx, void* hip_stream) {
    if (!ctx) return GSN_E_INVALID;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return GSN_OK;
}

gsn_status gsn_frame_create(gsn_ctx* ctx, gsn_frame** out) {
    if (!ctx || !out) return GSN_E_INVALID;
    gsn_frame* f = new (std::nothrow) gsn_frame;
    if (!f) return fail(ctx, GSN_E_NOMEM, "frame allocation failed");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipHostMalloc((void**)&f->h_total, sizeof(uint32_t), hipHostMallocDefault));
    *out = f;
    return GSN_OK;
}

gsn_status gsn_frame_destroy(gsn_ctx* ctx, gsn_frame* f) {
    if (!ctx || !f) return GSN_E_INVALID;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    DevBuf* all[] = {&f->rec, &f->rect, &f->depth_key, &f->ntiles, &f->ids_a, &f->ids_b, &f->keys_a, &f->keys_b,
                     &f->offsets, &f->pair_off, &f->nsup, &f->moffs, &f->pk_a, &f->pv_a, &f->pk_b, &f->pv_b, &f->sranges,
                     &f->seg_base, &f->seg_counts, &f->seg_offs, &f->partial, &f->flags, &f->kflag,
                     &f->ranges, &f->img, &f->img64, &f->Tfin, &f->ncontrib, &f->dL, &f->hd, &f->coef, &f->zsum,
                     &f->zsum_f, &f->sumrows, &f->contrib, &f->zstats,
                     &f->loss_part, &f->hist, &f->scan_tmp, &f->total, &f->masks, &f->tile_order, &f->tile_len, &f->bwd_order};
    for (DevBuf* b : all) buf_free(*b);
    if (f->h_total) (void)hipHostFree(f->h_total);
    delete f;
    return GSN_OK;
}

// Reserves the buffers a render of n kernels on a W x H view and its gsn_accumulate_hessian need,
// with pair buffers for `pairs` pairs (0: the pair buffers are left as they are).
static hipError_t frame_buffers(gsn_frame* f, int n, int W, int H, size_t pairs) {
    const size_t nn = (size_t)std::max(n, 1);
    const size_t npx = (size_t)W * H;
    const size_t tiles = (size_t)((W + GSN_TILE - 1) / GSN_TILE) * ((H + GSN_TILE - 1) / GSN_TILE);
    DevBuf* per_kernel4[] = {&f->depth_key, &f->ntiles, &f->ids_a, &f->ids_b, &f->keys_a, &f->keys_b, &f->pair_off,
                             &f->nsup, &f->moffs};
    hipError_t e = buf_reserve(f->rec, nn * 4 * sizeof(float4));
    if (e == hipSuccess) e = buf_reserve(f->rect, nn * sizeof(uint2));
    for (DevBuf* b : per_kernel4)
        if (e == hipSuccess) e = buf_reserve(*b, nn * 4);
    if (e == hipSuccess) e = buf_reserve(f->offsets, (nn + 1) * 4);
    if (e == hipSuccess) e = buf_reserve(f->kflag, (nn + 3) / 4 * 4);
    if (e == hipSuccess) e = buf_reserve(f->zsum_f, nn * GSN_NZ * 4);
    if (e == hipSuccess) e = buf_reserve(f->zsum, nn * 10 * 8);
    if (e == hipSuccess) e = buf_reserve(f->sumrows, nn * (kSumOverlap + 1) * 4);
    if (e == hipSuccess) e = buf_reserve(f->contrib, (nn + 3) / 4 * 4);
    if (e == hipSuccess) e = buf_reserve(f->ranges, tiles * sizeof(uint2));
    DevBuf* per_tile4[] = {&f->tile_order, &f->tile_len, &f->bwd_order};
    for (DevBuf* b : per_tile4)
        if (e == hipSuccess) e = buf_reserve(*b, tiles * 4);
    const int tx = (W + GSN_TILE - 1) / GSN_TILE, ty = (H + GSN_TILE - 1) / GSN_TILE;
    const size_t n_super = super_tiles(tx, ty);
    if (e == hipSuccess) e = buf_reserve(f->sranges, n_super * sizeof(uint2));
    if (e == hipSuccess) e = buf_reserve(f->seg_base, (n_super + 1) * 4);
    if (e == hipSuccess) e = buf_reserve(f->img, 3 * npx * 4);
    if (e == hipSuccess) e = buf_reserve(f->img64, 3 * npx * 8);
    if (e == hipSuccess) e = buf_reserve(f->Tfin, npx * 4);
    if (e == hipSuccess) e = buf_reserve(f->ncontrib, npx * 4);
    if (e == hipSuccess) e = buf_reserve(f->masks, tiles * GSN_MASK_BATCHES * 4 * GSN_BLOCK * sizeof(uint64_t));
    if (e == hipSuccess) e = buf_reserve(f->dL, 3 * npx * 4);
    if (e == hipSuccess) e = buf_reserve(f->hd, 3 * npx * 4);
    if (e == hipSuccess) e = buf_reserve(f->coef, 24 * npx * 4);
    if (e == hipSuccess) e = buf_reserve(f->loss_part, (size_t)2 * 3 * tiles * sizeof(double));
    if (e == hipSuccess) e = buf_reserve(f->total, 32);
    const size_t pp = std::max<size_t>(pairs, 1);
    // the histogram size is not monotone in the key count (the tile grows past 4M keys): cover
    // every count up to nn
    const size_t hist = std::max({radix_hist_bytes((uint32_t)nn), radix_hist_bytes((uint32_t)std::min<size_t>(nn, 1u << 22)),
                                  radix_hist_bytes((uint32_t)pp), radix_hist_bytes((uint32_t)std::min<size_t>(pp, 1u << 22))});
    if (e == hipSuccess) e = buf_reserve(f->hist, hist);
    if (e == hipSuccess) e = buf_reserve(f->scan_tmp, scan_tmp_bytes((uint32_t)std::max(nn, tiles)));
    if (pairs == 0 || e != hipSuccess) return e;
    DevBuf* per_pair4[] = {&f->pk_a, &f->pv_a, &f->pk_b, &f->pv_b};
    for (DevBuf* b : per_pair4)
        if (e == hipSuccess) e = buf_reserve(*b, pp * 4);
    const size_t words = segment_words(pp, tx, ty);
    if (e == hipSuccess) e = buf_reserve(f->seg_counts, words * 4);
    if (e == hipSuccess) e = buf_reserve(f->seg_offs, words * 4);
    if (e == hipSuccess) e = buf_reserve(f->scan_tmp, scan_tmp_bytes((uint32_t)std::max({nn, tiles, words})));
    if (e == hipSuccess) e = buf_reserve(f->partial, pp * GSN_NZ * 4);
    if (e == hipSuccess) e = buf_reserve(f->flags, (pp + 3) / 4 * 4);
    return e;
}

gsn_status gsn_frame_reserve(gsn_ctx* ctx, gsn_frame* f, int32_t n, int32_t width, int32_t height,
                             int64_t max_pairs) {
    if (!ctx || !f) return fail(ctx, GSN_E_INVALID, "null context or frame");
    if (n < 0 || width <= 0 || height <= 0 || max_pairs < 0)
        return fail(ctx, GSN_E_SHAPE, "n = %d, image %dx%d, max_pairs = %lld", n, width, height, (long long)max_pairs);
    if (max_pairs >= (1ll << 31)) return fail(ctx, GSN_E_CAPACITY, "max_pairs = %lld >= 2^31", (long long)max_pairs);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (max_pairs == 0) {
        f->cap_pairs = 0;
        f->cap_n = f->cap_W = f->cap_H = 0;
        return GSN_OK;
    }
    HIP_TRY(ctx, frame_buffers(f, n, width, height, (size_t)max_pairs));
    f->cap_pairs = max_pairs;
    f->cap_n = n;
    f->cap_W = width;
    f->cap_H = height;
    return GSN_OK;
}

gsn_status gsn_render(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_camera* cam, const gsn_render_opts* opts,
                      gsn_frame* f, float* d_rgb_out, float* d_T_out) {
    if (!ctx || !f || !opts) return fail(ctx, GSN_E_INVALID, "null context, frame or options");
    gsn_status st = check_gaussians(ctx, g);
    if (st != GSN_OK) return st;
    if ((st = check_camera(ctx, cam)) != GSN_OK) return st;
    if (opts->tile != GSN_TILE) return fail(ctx, GSN_E_INVALID, "tile must be %d", GSN_TILE);
    if (!(opts->alpha_max > 0.f && opts->alpha_max < 1.f) || !(opts->alpha_min >= 0.f) || !(opts->T_min >= 0.f) ||
        !(opts->kappa >= 0.f) || !(opts->radius_sigma > 0.f) || (opts->precision != 0 && opts->precision != 1))
        return fail(ctx, GSN_E_INVALID, "render option out of range");
    const bool reserved = f->cap_pairs > 0;
    if (reserved && (g->n > f->cap_n || (int64_t)cam->width * cam->height > (int64_t)f->cap_W * f->cap_H ||
                     (int64_t)((cam->width + 15) / 16) * ((cam->height + 15) / 16) >
                         (int64_t)((f->cap_W + 15) / 16) * ((f->cap_H + 15) / 16)))
        return fail(ctx, GSN_E_CAPACITY, "frame reserved for %d kernels at %dx%d: got %d kernels at %dx%d", f->cap_n,
                    f->cap_W, f->cap_H, g->n, cam->width, cam->height);
    if (!reserved && ctx->capturing)
        return fail(ctx, GSN_E_INVALID, "a render under graph capture needs a reserved frame (gsn_frame_reserve)");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int n = g->n;
    f->rendered = false;
    f->fp32 = opts->precision == 1;
    f->n = n;
    f->K = (g->sh_degree + 1) * (g->sh_degree + 1);
    f->cam = make_devcam(*cam);
    f->W = cam->width;
    f->H = cam->height;
    f->tiles_x = f->cam.tiles_x;
    f->tiles_y = f->cam.tiles_y;
    f->ro.alpha_min = opts->alpha_min;
    f->ro.alpha_max = opts->alpha_max;
    f->ro.T_min = opts->T_min;
    f->ro.kappa = opts->kappa;
    f->ro.radius_sigma = opts->radius_sigma;
    for (int i = 0; i < 3; ++i) f->ro.bg[i] = opts->bg[i];
    const size_t nn = (size_t)std::max(n, 1);
    const size_t npx = (size_t)f->W * f->H, tiles = (size_t)f->tiles_x * f->tiles_y;
    // per-kernel and per-pixel buffers (and, in reserved mode, everything): no buffer is reallocated
    // while work that uses it may still be queued
    if (!reserved) HIP_TRY(ctx, frame_buffers(f, n, f->W, f->H, 0));
    uint32_t* d_total = bp<uint32_t>(f->total);  // [0] scanned pair total, [1] live pair count
    {
        // 1. projection and binning decisions
        StageTimer st_(ctx, GSN_STAGE_PROJECT);
        launch_preprocess(*g, f->cam, f->ro, bp<float4>(f->rec), bp<uint2>(f->rect), bp<uint32_t>(f->keys_a),
                          bp<uint32_t>(f->ids_a), bp<uint32_t>(f->ntiles), ctx->d_stats + GSN_STAT_CULLED_NONFINITE,
                          s);
        HIP_TRY(ctx, hipGetLastError());
    }
    {
        // 2. depth order of the kernels: stable radix sort of (depth bits, id)
        StageTimer st_(ctx, GSN_STAGE_SORT);
        HIP_TRY(ctx, radix_sort_pairs(bp<uint32_t>(f->keys_a), bp<uint32_t>(f->ids_a), bp<uint32_t>(f->keys_b),
                                      bp<uint32_t>(f->ids_b), (uint32_t)n, nullptr, 0, 32, f->hist, s));
        // 3. pair offsets in depth order
        launch_gather_u32(bp<uint32_t>(f->ntiles), bp<uint32_t>(f->ids_a), bp<uint32_t>(f->keys_b), (uint32_t)n, s);
        if (n > 0) {
            HIP_TRY(ctx, exclusive_scan_u32(bp<uint32_t>(f->keys_b), bp<uint32_t>(f->offsets), (uint32_t)n, d_total,
                                            f->scan_tmp, s));
        } else {
            launch_fill_u32(d_total, 0u, 1, s);
        }
    }
    uint32_t cap;
    if (reserved) {
        cap = (uint32_t)f->cap_pairs;
        f->pairs = -1;
    } else {
        HIP_TRY(ctx, hipMemcpyAsync(f->h_total, d_total, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        cap = *f->h_total;
        f->pairs = cap;
        // the stream is idle here: growing the pair buffers cannot race with queued work
        HIP_TRY(ctx, frame_buffers(f, n, f->W, f->H, std::max<size_t>(cap, 1)));
    }
    const uint32_t* d_pairs = d_total + 1;
    {
        // 4. pairs in depth order, then a stable partition by tile id
        StageTimer st_(ctx, GSN_STAGE_SORT);
        launch_pair_capacity(d_total, cap, ctx->d_stats, prof_counts(ctx), s);
        // per-pair written-flags of the backward pass, cleared once per render (which slots it writes
        // depends only on this render, not on the loss)
        launch_fill_u32_dev(bp<uint32_t>(f->flags), 0u, d_pairs, 4, ((size_t)cap + 3) / 4, s);
        launch_fill_u32(bp<uint32_t>(f->kflag), 0u, (nn + 3) / 4, s);
        launch_pair_off(bp<uint32_t>(f->ids_a), bp<uint32_t>(f->offsets), (uint32_t)n, bp<uint32_t>(f->pair_off),
                        bp<float4>(f->rec), s);
        const TileListBufs tb{bp<uint32_t>(f->nsup),       bp<uint32_t>(f->moffs),    bp<uint32_t>(f->pk_a),
                              bp<uint32_t>(f->pv_a),       bp<uint32_t>(f->pk_b),     bp<uint32_t>(f->pv_b),
                              bp<uint2>(f->sranges),       bp<uint32_t>(f->seg_base), bp<uint32_t>(f->seg_counts),
                              bp<uint32_t>(f->seg_offs),   bp<uint2>(f->ranges)};
        HIP_TRY(ctx, build_tile_lists(bp<uint32_t>(f->ids_a), bp<uint2>(f->rect), (uint32_t)n, d_total, cap, f->tiles_x,
                                      f->tiles_y, tb, f->hist, f->scan_tmp, &f->list_ids, s));
        launch_tile_order(bp<uint2>(f->ranges), nullptr, (int)tiles, bp<uint32_t>(f->tile_order), s);
    }
    {
        // 5. front-to-back compositing
        StageTimer st_(ctx, GSN_STAGE_RASTER_FWD);
        launch_raster_fwd(bp<uint2>(f->ranges), bp<uint32_t>(f->tile_order), f->list_ids,
                          bp<float4>(f->rec), (uint32_t)n, f->cam, f->ro, f->fp32, bp<float>(f->img), bp<double>(f->img64),
                          bp<float>(f->Tfin), bp<uint32_t>(f->ncontrib), bp<uint64_t>(f->masks),
                          bp<uint32_t>(f->tile_len), prof_counts(ctx), ctx->prof_steps, s);
        // the backward pass takes the tiles with the longest composited prefixes first
        launch_tile_order(nullptr, bp<uint32_t>(f->tile_len), (int)tiles, bp<uint32_t>(f->bwd_order), s);
        HIP_TRY(ctx, hipGetLastError());
    }
    if (d_rgb_out) launch_copy_u32(reinterpret_cast<uint32_t*>(d_rgb_out), bp<uint32_t>(f->img), 3 * npx, s);
    if (d_T_out) launch_copy_u32(reinterpret_cast<uint32_t*>(d_T_out), bp<uint32_t>(f->Tfin), npx, s);
    HIP_TRY(ctx, hipGetLastError());
    f->rendered = true;
    return GSN_OK;
}

// gsn_accumulate_hessian on the context's current stream.  When not null, wait_reduce is waited for
// before the view's per-kernel sums (a secondary slot reads the primary coverage row) and done_reduce
// is recorded after them; with sum_now the view's shares of the rows summed over the views are added
// to the blocks at once (else the caller adds them, gsn_accumulate_views after all its views).
static gsn_status accumulate_impl(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_frame* fc, const float* d_target,
                                  const gsn_loss_opts* opts, int32_t view_slot, gsn_blocks* b, double* d_loss_out,
                                  hipEvent_t wait_reduce, hipEvent_t done_reduce, bool sum_now) {
    if (!ctx || !fc || !opts || !b || !d_target) return fail(ctx, GSN_E_INVALID, "null argument");
    gsn_frame* f = const_cast<gsn_frame*>(fc);
    gsn_status st = check_gaussians(ctx, g);
    if (st != GSN_OK) return st;
    if (!f->rendered) return fail(ctx, GSN_E_INVALID, "frame was never rendered");
    if (g->n != f->n || b->n != g->n) return fail(ctx, GSN_E_SHAPE, "n mismatch (g %d, frame %d, blocks %d)", g->n, f->n, b->n);
    if ((g->sh_degree + 1) * (g->sh_degree + 1) != f->K) return fail(ctx, GSN_E_SHAPE, "sh_degree differs from the frame's");
    if (view_slot < 0 || view_slot >= b->n_views) return fail(ctx, GSN_E_SHAPE, "view_slot %d outside 0..%d", view_slot, b->n_views - 1);
    if (!b->d_data && b->n > 0) return fail(ctx, GSN_E_INVALID, "blocks data is NULL");
    if (!(opts->lambda_ssim >= 0.f)) return fail(ctx, GSN_E_INVALID, "lambda_ssim must be >= 0");
    if (opts->precision != 0 && opts->precision != 1) return fail(ctx, GSN_E_INVALID, "precision must be 0 or 1");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const size_t npx = (size_t)f->W * f->H;
    HIP_TRY(ctx, buf_reserve(f->dL, 3 * npx * 4));
    HIP_TRY(ctx, buf_reserve(f->hd, 3 * npx * 4));
    HIP_TRY(ctx, buf_reserve(f->coef, 24 * npx * 4));
    const int nparts = ((f->W + 15) / 16) * ((f->H + 15) / 16) * 3;
    HIP_TRY(ctx, buf_reserve(f->loss_part, (size_t)2 * nparts * sizeof(double)));
    {
        StageTimer st_(ctx, GSN_STAGE_LOSS);
        int np_out = 0;
        launch_loss_maps(bp<float>(f->img), d_target, f->W, f->H, opts->lambda_ssim, opts->precision == 1,
                         bp<float>(f->coef),
                         bp<float>(f->dL), bp<float>(f->hd), bp<double>(f->loss_part), &np_out, s);
        if (d_loss_out) launch_loss_reduce(bp<double>(f->loss_part), np_out, f->W, f->H, d_loss_out, s);
        HIP_TRY(ctx, hipGetLastError());
    }
    HIP_TRY(ctx, buf_reserve(f->zsum_f, (size_t)std::max(f->n, 1) * GSN_NZ * 4));
    HIP_TRY(ctx, buf_reserve(f->zsum, (size_t)std::max(f->n, 1) * 10 * 8));
    HIP_TRY(ctx, buf_reserve(f->sumrows, (size_t)std::max(f->n, 1) * (kSumOverlap + 1) * 4));
    HIP_TRY(ctx, buf_reserve(f->contrib, ((size_t)std::max(f->n, 1) + 3) / 4 * 4));
    float* zs = nullptr;
    if (opts->keep_zstats) {
        HIP_TRY(ctx, buf_reserve(f->zstats, (size_t)std::max(f->n, 1) * GSN_NZ * 4));
        zs = bp<float>(f->zstats);
    }
    {
        StageTimer st_(ctx, GSN_STAGE_RASTER_BWD);
        if (f->pairs != 0)  // reserved frames (pairs = -1) always launch: empty lists end at once
            launch_raster_bwd(*f, bp<float>(f->dL), bp<float>(f->hd), opts->gauss_newton != 0, prof_counts(ctx),
                              ctx->prof && ctx->prof_steps, s);
    }
    {
        StageTimer st_(ctx, GSN_STAGE_CHAIN);
        if (wait_reduce) HIP_TRY(ctx, hipStreamWaitEvent(s, wait_reduce, 0));
        launch_reduce_pairs(*f, *g, view_slot, opts->precision == 1, *b, s);
        if (done_reduce) HIP_TRY(ctx, hipEventRecord(done_reduce, s));
        launch_chain(*f, *g, opts->weight, view_slot, opts->gauss_newton != 0, opts->precision == 1, *b, zs, s);
        if (sum_now) {
            SumViews sv{};
            sv.count = 1;
            sv.rows[0] = bp<float>(f->sumrows);
            sv.contrib[0] = bp<uint8_t>(f->contrib);
            launch_sum_views(*b, sv, s);
        }
    }
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_accumulate_hessian(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_frame* fc, const float* d_target,
                                  const gsn_loss_opts* opts, int32_t view_slot, gsn_blocks* b, double* d_loss_out) {
    return accumulate_impl(ctx, g, fc, d_target, opts, view_slot, b, d_loss_out, nullptr, nullptr, true);
}

gsn_status gsn_add_view_shares(gsn_ctx* ctx, gsn_blocks* b, int32_t n_views, gsn_frame* const* frames) {
    if (!ctx || !b || !frames) return fail(ctx, GSN_E_INVALID, "null argument");
    if (n_views < 0 || n_views > gsn_ctx::kMaxViews) return fail(ctx, GSN_E_SHAPE, "n_views %d not in 0..9", n_views);
    SumViews sv{};
    sv.count = n_views;
    for (int i = 0; i < n_views; ++i) {
        const gsn_frame* f = frames[i];
        if (!f || !f->rendered || f->n != b->n || f->sumrows.bytes < (size_t)b->n * (kSumOverlap + 1) * 4 ||
            f->contrib.bytes < (size_t)b->n)
            return fail(ctx, GSN_E_INVALID, "frame %d holds no accumulated view of these blocks", i);
        sv.rows[i] = bp<float>(f->sumrows);
        sv.contrib[i] = bp<uint8_t>(f->contrib);
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    StageTimer st_(ctx, GSN_STAGE_CHAIN);
    launch_sum_views(*b, sv, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_accumulate_views(gsn_ctx* ctx, const gsn_gaussians* g, int32_t n_views, int32_t first_slot,
                                const gsn_camera* cams, gsn_frame* const* frames, const float* const* d_targets,
                                const gsn_render_opts* ro, const gsn_loss_opts* lo, gsn_blocks* b,
                                double* d_loss_out, int32_t add_shares) {
    if (!ctx || !cams || !frames || !d_targets || !ro || !lo || !b) return fail(ctx, GSN_E_INVALID, "null argument");
    if (n_views < 1 || first_slot < 0 || first_slot + n_views > b->n_views || n_views > gsn_ctx::kMaxViews)
        return fail(ctx, GSN_E_SHAPE, "views %d..%d outside the blocks' slots 0..%d", first_slot,
                    first_slot + n_views - 1, b->n_views - 1);
    for (int i = 0; i < n_views; ++i) {
        if (!frames[i] || !d_targets[i]) return fail(ctx, GSN_E_INVALID, "view %d: null frame or target", i);
        for (int j = 0; j < i; ++j)
            if (frames[j] == frames[i]) return fail(ctx, GSN_E_INVALID, "views %d and %d share a frame", j, i);
        gsn_status r = check_camera(ctx, &cams[i]);
        if (r != GSN_OK) return r;
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    double* loss = d_loss_out;
    if (ctx->prof || n_views == 1) {  // one stream: the stage timers bracket each stage alone
        for (int i = 0; i < n_views; ++i) {
            gsn_status r = gsn_render(ctx, g, &cams[i], ro, frames[i], nullptr, nullptr);
            if (r == GSN_OK)
                r = accumulate_impl(ctx, g, frames[i], d_targets[i], lo, first_slot + i, b, loss ? loss + 2 * i : nullptr,
                                    nullptr, nullptr, add_shares != 0);
            if (r != GSN_OK) return r;
        }
        return GSN_OK;
    }
    hipStream_t home = ctx->stream;
    // view i goes to stream i % 4: the context's stream, then the side streams
    auto stream_of = [&](int i) { return i % (gsn_ctx::kSide + 1) == 0 ? home : ctx->side[i % (gsn_ctx::kSide + 1) - 1]; };
    const int used = std::min(n_views - 1, gsn_ctx::kSide);
    HIP_TRY(ctx, hipEventRecord(ctx->ev_fork, home));
    for (int k = 0; k < used; ++k) HIP_TRY(ctx, hipStreamWaitEvent(ctx->side[k], ctx->ev_fork, 0));
    gsn_status r = GSN_OK;
    // every view's render is issued before any accumulation, so that every stream has work early
    for (int i = 0; i < n_views && r == GSN_OK; ++i) {
        ctx->stream = stream_of(i);
        r = gsn_render(ctx, g, &cams[i], ro, frames[i], nullptr, nullptr);
    }
    for (int i = 0; i < n_views && r == GSN_OK; ++i) {
        ctx->stream = stream_of(i);
        // a secondary view's sums wait for the primary's coverage row when the primary is among the views
        hipEvent_t wait_reduce = (first_slot == 0 && i > 0) ? ctx->ev_chain[0] : nullptr;
        hipEvent_t done_reduce = (first_slot == 0 && i == 0) ? ctx->ev_chain[0] : nullptr;
        r = accumulate_impl(ctx, g, frames[i], d_targets[i], lo, first_slot + i, b, loss ? loss + 2 * i : nullptr,
                            wait_reduce, done_reduce, false);
    }
    // join every stream that took work, also after a failure, so that later calls stay ordered
    ctx->stream = home;
    for (int k = 0; k < used; ++k) {
        const hipError_t e1 = hipEventRecord(ctx->ev_join[k], ctx->side[k]);
        const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(home, ctx->ev_join[k], 0) : e1;
        if (e2 != hipSuccess && r == GSN_OK) r = fail(ctx, GSN_E_HIP, "joining the view streams: %s", hipGetErrorString(e2));
    }
    if (r == GSN_OK && add_shares) {
        // the views' shares of the summed rows, added in view order: the additions of the same calls
        // made one after another
        SumViews sv{};
        sv.count = n_views;
        for (int i = 0; i < n_views; ++i) {
            sv.rows[i] = bp<float>(frames[i]->sumrows);
            sv.contrib[i] = bp<uint8_t>(frames[i]->contrib);
        }
        StageTimer st_(ctx, GSN_STAGE_CHAIN);
        launch_sum_views(*b, sv, home);
        HIP_TRY(ctx, hipGetLastError());
    }
    return r;
}

// Argument checks shared by both solve entry points.
static gsn_status check_solve_args(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_camera* primary,
                                   const gsn_blocks* b, const gsn_solve_opts* o, const gsn_steps* st) {
    if (!ctx || !b || !o || !st) return fail(ctx, GSN_E_INVALID, "null argument");
    gsn_status r = check_gaussians(ctx, g);
    if (r != GSN_OK) return r;
    if ((r = check_camera(ctx, primary)) != GSN_OK) return r;
    if (b->n != g->n || st->n != g->n) return fail(ctx, GSN_E_SHAPE, "n mismatch");
    if (st->sh_degree != g->sh_degree) return fail(ctx, GSN_E_SHAPE, "steps sh_degree differs");
    if (b->n_views < 1 || b->n_views > 9) return fail(ctx, GSN_E_CAPACITY, "n_views %d not in 1..9", b->n_views);
    if (g->n > 0 && (!b->d_data || !st->d_data || !st->d_flags)) return fail(ctx, GSN_E_INVALID, "null device array");
    if (o->npix_primary <= 0 || o->max_escalations < 0 || o->max_escalations > 30)
        return fail(ctx, GSN_E_INVALID, "solve option out of range");
    if (o->precision != 0 && o->precision != 1) return fail(ctx, GSN_E_INVALID, "precision must be 0 or 1");
    if (o->precision == 1 && b->n_views > 4) return fail(ctx, GSN_E_SHAPE, "the mixed form takes at most 4 views");
    if (o->view_limit < 0) return fail(ctx, GSN_E_INVALID, "view_limit must be >= 0");
    return GSN_OK;
}

// The solve launches of the three solve entry points: gram is the mixed form's Gram scratch (the
// context's buffer, or the no-allocation array), ap the update fused into the solve (mask 0: none).
static void launch_solve_any(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_camera* primary, const gsn_blocks* b,
                             const gsn_solve_opts* o, gsn_steps* st, float* gram, const ApplyTo& ap) {
    unsigned long long* nonfinite = ctx->d_stats + GSN_STAT_SKIPPED_NONFINITE;
    if (o->precision == 1) {
        const int K = (g->sh_degree + 1) * (g->sh_degree + 1);
        launch_sh_gram(b->d_data, g->n, K, solve_view_slots(b->n_views, *o), gram, ctx->stream);
        launch_solve_mixed(*g, make_devcam(*primary), o->kappa, *b, *o, gram, *st, nonfinite, prof_counts(ctx), ap,
                           ctx->stream);
    } else {
        launch_solve(*g, make_devcam(*primary), o->kappa, *b, *o, *st, nonfinite, prof_counts(ctx), ap, ctx->stream);
    }
}

gsn_status gsn_local_newton_solve(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_camera* primary,
                                  const gsn_blocks* b, const gsn_solve_opts* o, gsn_steps* st) {
    gsn_status r = check_solve_args(ctx, g, primary, b, o, st);
    if (r != GSN_OK) return r;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (o->precision == 1) HIP_TRY(ctx, buf_reserve(ctx->gram, (size_t)std::max(g->n, 1) * 10 * 4));
    StageTimer st_(ctx, GSN_STAGE_SOLVE);
    launch_solve_any(ctx, g, primary, b, o, st, bp<float>(ctx->gram), ApplyTo{});
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_solve_apply(gsn_ctx* ctx, gsn_gaussians* g, const gsn_camera* primary, const gsn_blocks* b,
                           const gsn_solve_opts* o, gsn_steps* st, uint32_t group_mask) {
    gsn_status r = check_solve_args(ctx, g, primary, b, o, st);
    if (r != GSN_OK) return r;
    if (group_mask > 31u) return fail(ctx, GSN_E_INVALID, "group_mask 0x%x has bits beyond the five groups", group_mask);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (o->precision == 1) HIP_TRY(ctx, buf_reserve(ctx->gram, (size_t)std::max(g->n, 1) * 10 * 4));
    StageTimer st_(ctx, GSN_STAGE_SOLVE);
    ApplyTo ap;
    ap.pos = g->d_pos;
    ap.rot = g->d_rot;
    ap.scale = g->d_scale;
    ap.opac = g->d_opac;
    ap.sh = g->d_sh;
    ap.mask = group_mask;
    launch_solve_any(ctx, g, primary, b, o, st, bp<float>(ctx->gram), ap);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_local_newton_solve_noalloc(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_camera* primary,
                                          const gsn_blocks* b, const gsn_solve_opts* o, gsn_steps* st) {
    gsn_status r = check_solve_args(ctx, g, primary, b, o, st);
    if (r != GSN_OK) return r;
    if (g->n > GSN_NOALLOC_MAX_N)
        return fail(ctx, GSN_E_CAPACITY, "n = %d exceeds the no-allocation limit of %d kernels", g->n,
                    GSN_NOALLOC_MAX_N);
    if (!ctx->noalloc_gram) return fail(ctx, GSN_E_INVALID, "no scratch address for this device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // no stage timing here: timing may create events; no buffer is reserved or grown
    launch_solve_any(ctx, g, primary, b, o, st, ctx->noalloc_gram, ApplyTo{});
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_sh_gram(gsn_ctx* ctx, const gsn_blocks* b, int32_t sh_degree, float* d_out) {
    if (!ctx || !b) return fail(ctx, GSN_E_INVALID, "null argument");
    if (sh_degree < 0 || sh_degree > 3) return fail(ctx, GSN_E_SHAPE, "sh_degree must be 0..3");
    if (b->n_views < 1 || b->n_views > 4) return fail(ctx, GSN_E_SHAPE, "n_views must be 1..4");
    if (b->n > 0 && (!b->d_data || !d_out)) return fail(ctx, GSN_E_INVALID, "null device array");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    launch_sh_gram(b->d_data, b->n, (sh_degree + 1) * (sh_degree + 1), b->n_views, d_out, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

// Validates the items of a batched solve and builds the host scene table.
static gsn_status build_solve_table(gsn_ctx* ctx, const gsn_solve_item* items, int32_t count,
                                    std::vector<SolveScene>& table, long long& total, int& max_views) {
    if (!items || count < 1 || count > GSN_SOLVE_MAX_SCENES)
        return fail(ctx, GSN_E_INVALID, "count %d not in 1..%d", count, GSN_SOLVE_MAX_SCENES);
    table.clear();
    total = 0;
    max_views = 1;
    for (int i = 0; i < count; ++i) {
        const gsn_solve_item& it = items[i];
        if (!it.g || !it.primary || !it.blocks || !it.opts || !it.steps)
            return fail(ctx, GSN_E_INVALID, "item %d: null pointer", i);
        gsn_status r = check_gaussians(ctx, it.g);
        if (r != GSN_OK) return r;
        if ((r = check_camera(ctx, it.primary)) != GSN_OK) return r;
        const gsn_blocks& b = *it.blocks;
        const gsn_steps& st = *it.steps;
        const gsn_solve_opts& o = *it.opts;
        if (b.n != it.g->n || st.n != it.g->n) return fail(ctx, GSN_E_SHAPE, "item %d: n mismatch", i);
        if (st.sh_degree != it.g->sh_degree) return fail(ctx, GSN_E_SHAPE, "item %d: steps sh_degree differs", i);
        if (b.n_views < 1 || b.n_views > 9) return fail(ctx, GSN_E_CAPACITY, "item %d: n_views not in 1..9", i);
        if (it.g->n > 0 && (!b.d_data || !st.d_data || !st.d_flags))
            return fail(ctx, GSN_E_INVALID, "item %d: null device array", i);
        if (o.npix_primary <= 0 || o.max_escalations < 0 || o.max_escalations > 30)
            return fail(ctx, GSN_E_INVALID, "item %d: solve option out of range", i);
        if (o.precision != 0) return fail(ctx, GSN_E_INVALID, "item %d: the batched solve runs the plain form", i);
        SolveScene sc;
        sc.pos = it.g->d_pos;
        sc.rot = it.g->d_rot;
        sc.scale = it.g->d_scale;
        sc.opac = it.g->d_opac;
        sc.n = it.g->n;
        sc.K = (it.g->sh_degree + 1) * (it.g->sh_degree + 1);
        sc.V = b.n_views;
        sc.cam = make_devcam(*it.primary);
        sc.kappa = o.kappa;
        sc.blk = b.d_data;
        sc.o = o;
        sc.st = st.d_data;
        sc.fl = st.d_flags;
        sc.first = total;
        total += it.g->n;
        max_views = std::max(max_views, b.n_views);
        table.push_back(sc);
    }
    return GSN_OK;
}

static void default_solve_shape(gsn_ctx* ctx, int& block, int& grid) {
    if (ctx->solve_block > 0) {
        block = ctx->solve_block;
        grid = ctx->solve_grid;
        return;
    }
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    block = 128;
    grid = 4 * cus;
}

gsn_status gsn_solve_batched(gsn_ctx* ctx, const gsn_solve_item* items, int32_t count) {
    if (!ctx) return GSN_E_INVALID;
    std::vector<SolveScene> table;
    long long total = 0;
    int max_views = 1;
    gsn_status r = build_solve_table(ctx, items, count, table, total, max_views);
    if (r != GSN_OK) return r;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // the stream may still read an earlier table: wait before overwriting it
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, buf_reserve(ctx->solve_table, table.size() * sizeof(SolveScene)));
    HIP_TRY(ctx, hipMemcpy(ctx->solve_table.p, table.data(), table.size() * sizeof(SolveScene),
                           hipMemcpyHostToDevice));
    int block, grid;
    default_solve_shape(ctx, block, grid);
    StageTimer st_(ctx, GSN_STAGE_SOLVE);
    launch_solve_batched(bp<SolveScene>(ctx->solve_table), count, total, max_views, block, grid,
                         ctx->d_stats + GSN_STAT_SKIPPED_NONFINITE, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_solve_tune(gsn_ctx* ctx, const gsn_solve_item* items, int32_t count, int32_t* h_block,
                          int32_t* h_grid) {
    if (!ctx) return GSN_E_INVALID;
    std::vector<SolveScene> table;
    long long total = 0;
    int max_views = 1;
    gsn_status r = build_solve_table(ctx, items, count, table, total, max_views);
    if (r != GSN_OK) return r;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, buf_reserve(ctx->solve_table, table.size() * sizeof(SolveScene)));
    HIP_TRY(ctx, hipMemcpy(ctx->solve_table.p, table.data(), table.size() * sizeof(SolveScene),
                           hipMemcpyHostToDevice));
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    float best = 1e30f;
    int best_block = 128, best_grid = 4 * cus;
    // persistent grids of 1..16 workgroups per compute unit, and the full grid (one thread per kernel)
    const int blocks[3] = {64, 128, 256}, per_cu[6] = {1, 2, 4, 8, 16, 0};
    for (int bi = 0; bi < 3; ++bi)
        for (int pi = 0; pi < 6; ++pi) {
            const long long full = (total + blocks[bi] - 1) / blocks[bi];
            const int grid = per_cu[pi] ? per_cu[pi] * cus : (int)std::min<long long>(full, 1ll << 30);
            float ms_min = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {  // the first run warms the caches
                (void)hipEventRecord(e0, ctx->stream);
                launch_solve_batched(bp<SolveScene>(ctx->solve_table), count, total, max_views, blocks[bi], grid,
                                     ctx->d_stats + GSN_STAT_SKIPPED_NONFINITE, ctx->stream);
                (void)hipEventRecord(e1, ctx->stream);
                hipError_t e = hipEventSynchronize(e1);
                if (e != hipSuccess) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return fail(ctx, GSN_E_HIP, "tuning launch: %s", hipGetErrorString(e));
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) ms_min = std::min(ms_min, ms);
            }
            if (ms_min < best) {
                best = ms_min;
                best_block = blocks[bi];
                best_grid = grid;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_TRY(ctx, hipGetLastError());
    ctx->solve_block = best_block;
    ctx->solve_grid = best_grid;
    if (h_block) *h_block = best_block;
    if (h_grid) *h_grid = best_grid;
    return GSN_OK;
}

gsn_status gsn_solve_graph_create(gsn_ctx* ctx, const gsn_solve_item* items, int32_t count, gsn_graph** out) {
    if (!ctx || !out) return fail(ctx, GSN_E_INVALID, "null argument");
    *out = nullptr;
    std::vector<SolveScene> table;
    long long total = 0;
    int max_views = 1;
    gsn_status r = build_solve_table(ctx, items, count, table, total, max_views);
    if (r != GSN_OK) return r;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    gsn_graph* gr = new gsn_graph();
    hipStream_t cs = nullptr;
    auto cleanup = [&]() {
        if (cs) (void)hipStreamDestroy(cs);
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
        buf_free(gr->table);
        delete gr;
    };
    hipError_t e = buf_reserve(gr->table, table.size() * sizeof(SolveScene));
    if (e == hipSuccess)
        e = hipMemcpy(gr->table.p, table.data(), table.size() * sizeof(SolveScene), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        int block, grid;
        default_solve_shape(ctx, block, grid);
        launch_solve_batched(bp<SolveScene>(gr->table), count, total, max_views, block, grid,
                             ctx->d_stats + GSN_STAT_SKIPPED_NONFINITE, cs);
        hipError_t el = hipGetLastError();
        e = hipStreamEndCapture(cs, &gr->graph);
        if (e == hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        cleanup();
        return fail(ctx, GSN_E_HIP, "graph capture: %s", hipGetErrorString(e));
    }
    (void)hipStreamDestroy(cs);
    *out = gr;
    return GSN_OK;
}

gsn_status gsn_graph_launch(gsn_ctx* ctx, gsn_graph* gr) {
    if (!ctx || !gr || !gr->exec) return fail(ctx, GSN_E_INVALID, "null graph");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (ctx->capturing) return fail(ctx, GSN_E_INVALID, "graph launch while capturing");
    if (gr->stage >= 0) {
        StageTimer st_(ctx, gr->stage);
        HIP_TRY(ctx, hipGraphLaunch(gr->exec, ctx->stream));
    } else {
        // a captured sequence of calls spans every stage: it is not timed by stage
        HIP_TRY(ctx, hipGraphLaunch(gr->exec, ctx->stream));
    }
    return GSN_OK;
}

gsn_status gsn_capture_begin(gsn_ctx* ctx) {
    if (!ctx) return GSN_E_INVALID;
    if (ctx->capturing) return fail(ctx, GSN_E_INVALID, "the context is already capturing");
    if (t_capturing) return fail(ctx, GSN_E_INVALID, "another context is capturing on this thread");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (!ctx->cap_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    // what the caller queued so far finishes first; the graph's work is ordered by its launch
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    ctx->user_stream = ctx->stream;
    ctx->stream = ctx->cap_stream;
    ctx->capturing = true;
    ctx->capture_failed = false;
    t_capturing = true;
    return GSN_OK;
}

gsn_status gsn_capture_end(gsn_ctx* ctx, gsn_graph** out) {
    if (!ctx || !out) return fail(ctx, GSN_E_INVALID, "null argument");
    *out = nullptr;
    if (!ctx->capturing) return fail(ctx, GSN_E_INVALID, "the context is not capturing");
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
    ctx->stream = ctx->user_stream;
    ctx->user_stream = nullptr;
    ctx->capturing = false;
    t_capturing = false;
    const bool failed = ctx->capture_failed;
    ctx->capture_failed = false;
    if (e != hipSuccess || failed || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(ctx, GSN_E_HIP, "graph capture: %s", hipGetErrorString(e));
        return fail(ctx, GSN_E_INVALID, "a call failed while capturing: no graph");
    }
    gsn_graph* gr = new (std::nothrow) gsn_graph();
    if (!gr) {
        (void)hipGraphDestroy(graph);
        return fail(ctx, GSN_E_NOMEM, "graph allocation failed");
    }
    gr->graph = graph;
    gr->stage = -1;
    const hipError_t ei = hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete gr;
        return fail(ctx, GSN_E_HIP, "graph instantiation: %s", hipGetErrorString(ei));
    }
    *out = gr;
    return GSN_OK;
}

gsn_status gsn_graph_destroy(gsn_ctx* ctx, gsn_graph* gr) {
    if (!gr) return GSN_OK;
    if (ctx) {
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
    }
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    buf_free(gr->table);
    delete gr;
    return GSN_OK;
}

gsn_status gsn_apply_step(gsn_ctx* ctx, gsn_gaussians* g, const gsn_steps* st, const gsn_solve_opts* o,
                          const float* d_scale, uint32_t group_mask) {
    if (!ctx || !st || !o) return fail(ctx, GSN_E_INVALID, "null argument");
    gsn_status r = check_gaussians(ctx, g);
    if (r != GSN_OK) return r;
    if (st->n != g->n || st->sh_degree != g->sh_degree) return fail(ctx, GSN_E_SHAPE, "steps do not match gaussians");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    StageTimer st_(ctx, GSN_STAGE_APPLY);
    launch_apply(*g, *st, *o, d_scale, group_mask, prof_counts(ctx), ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_first_order_step(gsn_ctx* ctx, gsn_gaussians* g, const gsn_blocks* b, const gsn_solve_opts* o,
                                const gsn_first_order_opts* fo, float* d_state, uint32_t group_mask) {
    if (!ctx || !b || !o || !fo) return fail(ctx, GSN_E_INVALID, "null argument");
    gsn_status r = check_gaussians(ctx, g);
    if (r != GSN_OK) return r;
    if (b->n != g->n) return fail(ctx, GSN_E_SHAPE, "n mismatch");
    if (b->n_views < 1 || b->n_views > 9) return fail(ctx, GSN_E_CAPACITY, "n_views %d not in 1..9", b->n_views);
    if (g->n > 0 && !b->d_data) return fail(ctx, GSN_E_INVALID, "blocks data is NULL");
    for (int i = 0; i < 5; ++i)
        if (!(fo->lr[i] >= 0.f)) return fail(ctx, GSN_E_INVALID, "learning rates must be >= 0");
    double c1 = 1.0, c2 = 1.0;
    if (fo->adam) {
        if (g->n > 0 && !d_state) return fail(ctx, GSN_E_INVALID, "Adam needs a moment buffer");
        if (fo->step < 1) return fail(ctx, GSN_E_INVALID, "Adam step count must be >= 1");
        if (!(fo->beta1 >= 0.f && fo->beta1 < 1.f && fo->beta2 >= 0.f && fo->beta2 < 1.f && fo->eps >= 0.f))
            return fail(ctx, GSN_E_INVALID, "Adam moments out of range");
        c1 = 1.0 / (1.0 - std::pow((double)fo->beta1, fo->step));
        c2 = 1.0 / (1.0 - std::pow((double)fo->beta2, fo->step));
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    StageTimer st_(ctx, GSN_STAGE_APPLY);
    launch_first_order(*g, *b, *fo, (float)c1, (float)c2, o->scale_floor, o->opac_eps, fo->adam ? d_state : nullptr,
                       group_mask, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_step_features(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_camera* primary,
                             const gsn_blocks* b, const gsn_solve_opts* o, const float* d_resid, float* d_feat,
                             uint8_t* d_ok) {
    if (!ctx || !b || !o) return fail(ctx, GSN_E_INVALID, "null argument");
    gsn_status r = check_gaussians(ctx, g);
    if (r != GSN_OK) return r;
    if ((r = check_camera(ctx, primary)) != GSN_OK) return r;
    if (b->n != g->n) return fail(ctx, GSN_E_SHAPE, "n mismatch");
    if (g->n > 0 && (!b->d_data || !d_feat || !d_ok)) return fail(ctx, GSN_E_INVALID, "null device array");
    if (o->npix_primary <= 0) return fail(ctx, GSN_E_INVALID, "npix_primary must be positive");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    launch_features(*g, make_devcam(*primary), o->kappa, *b, *o, d_resid, d_feat, d_ok, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_neighbour_residual(gsn_ctx* ctx, const gsn_blocks* b, float* d_resid) {
    if (!ctx || !b) return fail(ctx, GSN_E_INVALID, "null argument");
    if (b->n_views < 2) return fail(ctx, GSN_E_SHAPE, "the blocks hold no secondary view");
    if (b->n > 0 && (!b->d_data || !d_resid)) return fail(ctx, GSN_E_INVALID, "null device array");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    launch_neighbour_residual(*b, d_resid, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_step_labels(gsn_ctx* ctx, const gsn_steps* prim, const gsn_steps* aug, const uint8_t* d_ok,
                           const float* d_alpha, float* d_label, float* d_mask, double* d_err) {
    if (!ctx || !prim || !aug) return fail(ctx, GSN_E_INVALID, "null argument");
    if (prim->n != aug->n || prim->sh_degree != aug->sh_degree) return fail(ctx, GSN_E_SHAPE, "steps differ in shape");
    if (prim->n < 0 || prim->sh_degree < 0 || prim->sh_degree > 3) return fail(ctx, GSN_E_SHAPE, "bad steps shape");
    if (prim->n > 0 && (!prim->d_data || !prim->d_flags || !aug->d_data || !d_label || !d_mask))
        return fail(ctx, GSN_E_INVALID, "null device array");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int K = (prim->sh_degree + 1) * (prim->sh_degree + 1);
    if (d_alpha && d_err) HIP_TRY(ctx, buf_reserve(ctx->label_part, label_part_words(prim->n) * 8));
    launch_labels(prim->n, K, prim->d_data, prim->d_flags, aug->d_data, d_ok, d_alpha, d_label, d_mask,
                  bp<double>(ctx->label_part), d_err, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_mlp_reset(gsn_ctx* ctx, gsn_mlp* mlp) {
    if (!ctx || !mlp || !mlp->d_params || !mlp->d_m || !mlp->d_v || !mlp->d_half)
        return fail(ctx, GSN_E_INVALID, "null argument");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    mlp->step = 0;
    launch_mlp_reset(*mlp, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_mlp_infer(gsn_ctx* ctx, const gsn_mlp* mlp, int32_t n, const float* d_feat, const uint8_t* d_ok,
                         float* d_alpha, uint32_t* d_out_of_range) {
    if (!ctx || !mlp || !mlp->d_half) return fail(ctx, GSN_E_INVALID, "null argument");
    if (n < 0) return fail(ctx, GSN_E_INVALID, "n < 0");
    if (n > 0 && (!d_feat || !d_ok || !d_alpha)) return fail(ctx, GSN_E_INVALID, "null device array");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    launch_mlp_infer(mlp->d_half, n, d_feat, d_ok, d_alpha, d_out_of_range, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_mlp_train_step(gsn_ctx* ctx, gsn_mlp* mlp, int32_t n, const float* d_feat, const float* d_label,
                              const float* d_mask, const gsn_adam_opts* a, double* d_loss, float* d_grad) {
    if (!ctx || !mlp || !a || !mlp->d_params || !mlp->d_m || !mlp->d_v || !mlp->d_half)
        return fail(ctx, GSN_E_INVALID, "null argument");
    if (n < 0) return fail(ctx, GSN_E_INVALID, "n < 0");
    if (n > 0 && (!d_feat || !d_label || !d_mask)) return fail(ctx, GSN_E_INVALID, "null device array");
    if (!(a->lr > 0.f) || !(a->beta1 >= 0.f && a->beta1 < 1.f) || !(a->beta2 >= 0.f && a->beta2 < 1.f) ||
        !(a->eps > 0.f))
        return fail(ctx, GSN_E_INVALID, "Adam option out of range");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int nb = std::max(mlp_grad_blocks(n), 1);
    HIP_TRY(ctx, buf_reserve(ctx->mlp_part, (size_t)nb * GSN_MLP_PARAMS * 4));
    HIP_TRY(ctx, buf_reserve(ctx->mlp_stat, mlp_stat_words(n) * 8));
    mlp->step += 1;
    launch_mlp_train(*mlp, n, d_feat, d_label, d_mask, bp<float>(ctx->mlp_part), bp<double>(ctx->mlp_stat), *a,
                     d_grad, d_loss, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

int64_t gsn_blocks_floats(int32_t n, int32_t n_views) {
    if (n < 0 || n_views < 1) return 0;
    return (int64_t)(GSN_BLK_BASE + GSN_BLK_VIEW * n_views + 1) * n;
}

gsn_status gsn_blocks_zero(gsn_ctx* ctx, gsn_blocks* b) {
    if (!ctx || !b) return GSN_E_INVALID;
    if (b->n == 0) return GSN_OK;
    if (!b->d_data) return fail(ctx, GSN_E_INVALID, "blocks data is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    launch_fill_f32(b->d_data, 0.f, (size_t)gsn_blocks_floats(b->n, b->n_views), ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

int64_t gsn_steps_floats(int32_t n, int32_t sh_degree) {
    if (n < 0 || sh_degree < 0 || sh_degree > 3) return 0;
    return (int64_t)(GSN_STEP_BASE + 3 * (sh_degree + 1) * (sh_degree + 1)) * n;
}

gsn_status gsn_downsample2x(gsn_ctx* ctx, const float* d_src, int32_t width, int32_t height, float* d_dst) {
    if (!ctx || !d_src || !d_dst) return fail(ctx, GSN_E_INVALID, "null argument");
    if (width < 2 || height < 2) return fail(ctx, GSN_E_SHAPE, "image %dx%d too small", width, height);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    launch_downsample2x(d_src, width, height, d_dst, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_camera_half(const gsn_camera* cam, gsn_camera* out) {
    if (!cam || !out) return GSN_E_INVALID;
    if (cam->width < 2 || cam->height < 2) return GSN_E_SHAPE;
    gsn_camera h = *cam;
    h.fx = (float)(0.5 * (double)cam->fx);
    h.fy = (float)(0.5 * (double)cam->fy);
    h.cx = (float)(0.5 * ((double)cam->cx + 0.5) - 0.5);
    h.cy = (float)(0.5 * ((double)cam->cy + 0.5) - 0.5);
    h.width = cam->width / 2;
    h.height = cam->height / 2;
    *out = h;
    return GSN_OK;
}

gsn_status gsn_scene_center(gsn_ctx* ctx, const gsn_gaussians* g, double* d_out) {
    if (!ctx || !d_out) return fail(ctx, GSN_E_INVALID, "null argument");
    gsn_status r = check_gaussians(ctx, g);
    if (r != GSN_OK) return r;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    launch_scene_center(g->d_pos, g->n, d_out, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_camera_knn(const double* c, int32_t ncam, const double* sc, int32_t k, int32_t* out) {
    if (!c || !sc || !out || k < 1 || k >= ncam) return GSN_E_INVALID;
    std::vector<double> u(3 * (size_t)ncam);
    for (int i = 0; i < ncam; ++i) {
        double d[3], nn = 0;
        for (int a = 0; a < 3; ++a) {
            d[a] = c[3 * i + a] - sc[a];
            nn += d[a] * d[a];
        }
        nn = std::sqrt(nn);
        for (int a = 0; a < 3; ++a) u[3 * i + a] = d[a] / nn;
    }
    std::vector<std::pair<double, int>> dist;
    for (int i = 0; i < ncam; ++i) {
        dist.clear();
        for (int j = 0; j < ncam; ++j) {
            if (j == i) continue;
            const double dot = u[3 * i] * u[3 * j] + u[3 * i + 1] * u[3 * j + 1] + u[3 * i + 2] * u[3 * j + 2];
            dist.emplace_back(std::acos(std::max(-1.0, std::min(1.0, dot))), j);
        }
        std::partial_sort(dist.begin(), dist.begin() + k, dist.end());
        for (int a = 0; a < k; ++a) out[(size_t)i * k + a] = dist[a].second;
    }
    return GSN_OK;
}

// The pair count of the frame's last render (read from the device for reserved frames).
static gsn_status frame_pairs(gsn_ctx* ctx, const gsn_frame* f, int64_t* out) {
    *out = f->pairs;
    if (f->pairs >= 0) return GSN_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    uint32_t live = 0;
    HIP_TRY(ctx, hipMemcpyAsync(f->h_total, bp<uint32_t>(f->total) + 1, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    live = *f->h_total;
    *out = live;
    return GSN_OK;
}

gsn_status gsn_frame_info(gsn_ctx* ctx, const gsn_frame* f, int64_t* pairs, int32_t* tx, int32_t* ty) {
    if (!ctx || !f) return GSN_E_INVALID;
    if (pairs) {
        gsn_status r = frame_pairs(ctx, f, pairs);
        if (r != GSN_OK) return r;
    }
    if (tx) *tx = f->tiles_x;
    if (ty) *ty = f->tiles_y;
    return GSN_OK;
}

gsn_status gsn_frame_lists(gsn_ctx* ctx, const gsn_frame* f, uint32_t* d_ranges, uint32_t* d_ids,
                           uint32_t* d_depth_bits, int32_t* d_rect, uint32_t* d_ncontrib) {
    if (!ctx || !f) return GSN_E_INVALID;
    if (!f->rendered) return fail(ctx, GSN_E_INVALID, "frame was never rendered");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const size_t tiles = (size_t)f->tiles_x * f->tiles_y, npx = (size_t)f->W * f->H;
    if (d_ranges) HIP_TRY(ctx, hipMemcpyAsync(d_ranges, f->ranges.p, tiles * 8, hipMemcpyDeviceToDevice, s));
    int64_t pairs = 0;
    if (d_ids) {
        gsn_status r = frame_pairs(ctx, f, &pairs);
        if (r != GSN_OK) return r;
    }
    if (d_ids && pairs) HIP_TRY(ctx, hipMemcpyAsync(d_ids, f->list_ids, (size_t)pairs * 4, hipMemcpyDeviceToDevice, s));
    if (d_ncontrib) HIP_TRY(ctx, hipMemcpyAsync(d_ncontrib, f->ncontrib.p, npx * 4, hipMemcpyDeviceToDevice, s));
    if ((d_depth_bits || d_rect) && f->n > 0) {
        // depth keys were sorted in place; recompute the per-kernel view from the rect/keys copies
        std::vector<uint2> rect(f->n);
        HIP_TRY(ctx, hipMemcpyAsync(rect.data(), f->rect.p, (size_t)f->n * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        if (d_rect) {
            std::vector<int32_t> r4((size_t)4 * f->n);
            for (int k = 0; k < f->n; ++k) {
                r4[k] = rect[k].x & 0xffff;
                r4[f->n + k] = rect[k].x >> 16;
                r4[2 * (size_t)f->n + k] = rect[k].y & 0xffff;
                r4[3 * (size_t)f->n + k] = rect[k].y >> 16;
            }
            HIP_TRY(ctx, hipMemcpy(d_rect, r4.data(), r4.size() * 4, hipMemcpyHostToDevice));
        }
        if (d_depth_bits) {
            // the sorted keys are in keys_a in depth order with ids in ids_a: scatter them back by id
            std::vector<uint32_t> keys(f->n), ids(f->n), out(f->n);
            HIP_TRY(ctx, hipMemcpy(keys.data(), f->keys_a.p, (size_t)f->n * 4, hipMemcpyDeviceToHost));
            HIP_TRY(ctx, hipMemcpy(ids.data(), f->ids_a.p, (size_t)f->n * 4, hipMemcpyDeviceToHost));
            for (int r = 0; r < f->n; ++r) out[ids[r]] = keys[r];
            HIP_TRY(ctx, hipMemcpy(d_depth_bits, out.data(), (size_t)f->n * 4, hipMemcpyHostToDevice));
        }
    }
    return GSN_OK;
}

gsn_status gsn_frame_zstats(gsn_ctx* ctx, const gsn_frame* f, float* d_out) {
    if (!ctx || !f || !d_out) return GSN_E_INVALID;
    if (!f->zstats.p) return fail(ctx, GSN_E_INVALID, "no statistics kept: run gsn_accumulate_hessian with keep_zstats");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipMemcpyAsync(d_out, f->zstats.p, (size_t)f->n * GSN_NZ * 4, hipMemcpyDeviceToDevice, ctx->stream));
    return GSN_OK;
}

gsn_status gsn_frame_records(gsn_ctx* ctx, const gsn_frame* f, float* d_out) {
    if (!ctx || !f || !d_out) return GSN_E_INVALID;
    if (!f->rendered) return fail(ctx, GSN_E_INVALID, "frame was never rendered");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    launch_records_out(bp<float4>(f->rec), f->n, reinterpret_cast<float4*>(d_out), ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return GSN_OK;
}

gsn_status gsn_frame_loss_maps(gsn_ctx* ctx, const gsn_frame* f, float* d_dL, float* d_h) {
    if (!ctx || !f) return GSN_E_INVALID;
    if (!f->dL.p) return fail(ctx, GSN_E_INVALID, "no loss maps: run gsn_accumulate_hessian first");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const size_t bytes = (size_t)3 * f->W * f->H * 4;
    if (d_dL) HIP_TRY(ctx, hipMemcpyAsync(d_dL, f->dL.p, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    if (d_h) HIP_TRY(ctx, hipMemcpyAsync(d_h, f->hd.p, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    return GSN_OK;
}

}  // extern "C"

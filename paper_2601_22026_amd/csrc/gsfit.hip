// gsfit.hip - host runtime and C ABI (include/gsfit.h) of the gfx950 fit path.
//
// A context pins a device and a stream.  A plan fixes the view sizes, SH
// degree, tile size, LDS batch and key capacity, carves the caller-owned
// workspace into the buffers of the pipeline and enqueues the kernels:
//
//   forward   project (+ per-record tile counts) -> record-order scan (gradient
//             slots, key total) -> depth sort of the records with keys -> their keys
//             emitted in depth order -> stable sort by tile -> tile ranges and
//             compositing order -> composite
//   loss      masked L1 -> dL/dRGBA
//   backward  zero screen-space gradient -> composite adjoint -> projection adjoint
//   adam      step counter + update
//
// All views of a plan share one launch per stage: their tiles form one global
// tile space (per-view offsets) and their records one record space r = v*n + i.
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <cmath>
#include <vector>

#include "gs_internal.h"

using namespace gsf;

struct gsf_ctx {
    int device = 0;
    int cus = 256;                             // compute units of the device
    hipStream_t stream = nullptr;
    std::string err;
    unsigned long long *warp_scratch = nullptr;   // device address of the no-allocation z-buffer
    hipError_t warp_scratch_err = hipSuccess;
};

namespace {

struct Buffers {
    // per record (view v, Gaussian i)
    float4 *rec = nullptr;                       // 64 B: splat and support ellipse (SplatPtrs)
    uint32_t *depth_key = nullptr;               // float32 depth bits; 0xFFFFFFFF = culled
    uint2 *rect = nullptr;                       // touched tile rectangle
    uint32_t *count = nullptr;                   // listed tiles
    uint2 *rspan = nullptr;                      // packed row spans of short boxes (else row-table size)
    uint32_t *koff = nullptr;                    // position of the record's first key (record order)
    uint32_t *block_sums = nullptr;              // scan of the per-record tile counts
    uint32_t *block_act = nullptr;               // scan of the records that list a tile
    uint32_t *emit_sums = nullptr;               // scan of the counts in depth order
    unsigned long long *seg_tot = nullptr;       // segment totals of those scans
    uint32_t *seg_act = nullptr;
    uint4 *arec = nullptr;                       // per record with keys: the emission's data (32 B)
    // per global tile
    uint2 *ranges = nullptr;
    uint32_t *order = nullptr;                   // compositing order of the tiles
    uint2 *fovea_rows = nullptr;                 // fovea culling: per view and tile row, the disk's columns
    uint32_t *order_counts = nullptr;            // per-workgroup class counts of that order
    // per key (key capacity): two (key, value) buffer pairs.  The active
    // records' (depth, record) pairs are sorted in them first (ending in the
    // depth pair), their keys emitted in depth order into the emission pair,
    // and the keys sorted by tile between the two; `vals` is then the sorted
    // record-id list the compositing reads.
    uint32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr, *v1 = nullptr;
    uint32_t *dsorted = nullptr;                 // depth-ordered active records (the depth sort's values)
    uint32_t *depth_mm = nullptr;                // per depth-sort workgroup: smallest, largest key
    uint32_t *depth_ctl = nullptr;               // depth sort: key base, 24 bits suffice
    uint32_t *ek = nullptr, *ev = nullptr;       // emission pair
    uint32_t *tk = nullptr, *tv = nullptr;       // the other pair
    uint32_t *keys = nullptr, *vals = nullptr;   // sorted pair (one of the above)
    uint32_t *hist = nullptr, *digit_tot = nullptr;   // radix-sort histograms
    uint2 *rowtab = nullptr;                     // per key position: row tables of boxes not packed
    // per key, at its position in the record-order scan: the adjoint's
    // screen-space gradient, one 64-byte chunk (fields 0-3, 4-7, 8)
    float4 *pg = nullptr;
    // per pixel
    float *tfinal = nullptr;
    uint32_t *ncontrib = nullptr;
    float4 *ckpt = nullptr, *fstate = nullptr;   // checkpointed mode only
    float *tstore = nullptr;                     // stored mode only
    float *g2d = nullptr;
    uint32_t *m_dev = nullptr, *a_dev = nullptr, *flags = nullptr, *mask_count = nullptr;
    unsigned long long *m_total = nullptr;
    unsigned long long *counters = nullptr;
    float *loss_partial = nullptr;
    float *bg = nullptr;                         // per-view random background of the step [V][3]
    ViewDesc *views = nullptr;
    uint8_t *vis = nullptr;                      // per-Gaussian visibility of the masked Adam [n_max]
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Depth keys are float32 bits of positive depths: the sign bit is zero.

}  // namespace

struct gsf_plan {
    gsf_ctx *ctx = nullptr;
    int64_t n_max = 0;
    int deg = 0, V = 0, tile = 16, batch = 128, t_mode = 0, host_sized = 0;
    int64_t cap = 0;
    std::vector<ViewDesc> views;
    int64_t total_tiles = 0, total_pix = 0, nrec_max = 0;
    int tile_bits = 0, radix_grid = 1, bwd_grid = 1;
    uint32_t m_host = 0;                      // key count of the last host-sized forward
    size_t ws_bytes = 0;
    void *ws = nullptr;
    Buffers b;
    bool have_forward = false;
    bool fwd_culled = false;                  // the last forward composited only fovea tiles
    const float *fwd_cull_gaze = nullptr;     // its fovea culling (device [V][2]) and radius
    float fwd_cull_radius = 0.f;
    int64_t fwd_n = 0;
    // the last forward's launch tiles, which ranges and order index: the plan's
    // global tiles, or (fwd_tm.gaze) the compact fovea-box tiles of its keys
    TileMap fwd_tm{};
    int64_t fwd_tiles = 0;
    unsigned long long *pinned = nullptr;     // host-pinned readback of the key count
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // per-stage timing (eager only)
    bool timing = false;
    struct Pending {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double stage_ms[GSF_STAGE_COUNT] = {};
    int64_t stage_calls[GSF_STAGE_COUNT] = {};
};

namespace {

gsf_status fail(gsf_ctx *ctx, gsf_status st, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return st;
}

#define GSF_HIP(ctx, expr)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), GSF_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define GSF_LAUNCHED(ctx)                                                                    \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), GSF_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

int planes_of(int deg) { return 11 + 3 * (deg + 1) * (deg + 1); }

// Tile rows of the tallest view: the rows of the fovea-culling row table per view.
int fovea_rows_per_view(const gsf_plan *p) {
    int ty = 1;
    for (const ViewDesc &vd : p->views) ty = std::max(ty, (int)vd.tiles_y);
    return ty;
}

// Carve the workspace (base == nullptr: only measure).  Returns the byte count.
size_t carve(gsf_plan *p, char *base, Buffers *out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *ptr = base ? base + off : nullptr;
        off += align256(bytes);
        return ptr;
    };
    const size_t R = (size_t)p->nrec_max;
    Buffers b;
    b.rec = (float4 *)take(R * kRecF4 * sizeof(float4));   // 256-aligned: records on 64-byte chunks
    b.depth_key = (uint32_t *)take(R * 4);
    b.rect = (uint2 *)take(R * sizeof(uint2));
    b.count = (uint32_t *)take(R * 4);
    b.rspan = (uint2 *)take(R * sizeof(uint2));
    b.koff = (uint32_t *)take(R * 4);
    const size_t T = (size_t)p->total_tiles;
    b.block_sums = (uint32_t *)take((size_t)scan_blocks(p->nrec_max) * 4);
    b.block_act = (uint32_t *)take((size_t)scan_blocks(p->nrec_max) * 4);
    b.emit_sums = (uint32_t *)take((size_t)scan_blocks(p->nrec_max) * 4);
    b.seg_tot = (unsigned long long *)take((size_t)seg_count(p->nrec_max) * 8);
    b.seg_act = (uint32_t *)take((size_t)seg_count(p->nrec_max) * 4);
    b.arec = (uint4 *)take((size_t)std::min<int64_t>(p->nrec_max, p->cap) * 32);
    b.ranges = (uint2 *)take(T * sizeof(uint2));
    b.order = (uint32_t *)take(T * 4);
    b.fovea_rows = (uint2 *)take((size_t)p->V * fovea_rows_per_view(p) * sizeof(uint2));
    b.order_counts = (uint32_t *)take((size_t)33 * order_groups(p->total_tiles) * 4);
    b.k0 = (uint32_t *)take((size_t)p->cap * 4);
    b.v0 = (uint32_t *)take((size_t)p->cap * 4);
    b.k1 = (uint32_t *)take((size_t)p->cap * 4);
    b.v1 = (uint32_t *)take((size_t)p->cap * 4);
    // the depth sort passes between (k0, v0) and (k1, v1) and ends in dsorted;
    // the keys are emitted into (ek, ev) and the tile sort's passes write
    // (tk, tv) then (ek, ev), alternately
    b.dsorted = (uint32_t *)take((size_t)std::min<int64_t>(p->nrec_max, p->cap) * 4);
    b.depth_mm = (uint32_t *)take((size_t)2 * p->radix_grid * 4);
    b.depth_ctl = (uint32_t *)take(2 * 4);
    b.ek = b.k1;
    b.ev = b.v1;
    b.tk = b.k0;
    b.tv = b.v0;
    const bool tiles_odd = radix_passes(p->tile_bits) % 2 == 1;   // tile sort: (tk, tv) first
    b.keys = tiles_odd ? b.tk : b.ek;
    b.vals = tiles_odd ? b.tv : b.ev;
    b.hist = (uint32_t *)take((size_t)kRadixBins * p->radix_grid * 4);
    b.digit_tot = (uint32_t *)take(kRadixBins * 4);
    b.rowtab = (uint2 *)take((size_t)p->cap * sizeof(uint2));
    b.pg = (float4 *)take((size_t)p->cap * kKeyGradF4 * sizeof(float4));
    b.tfinal = (float *)take((size_t)p->total_pix * 4);
    b.ncontrib = (uint32_t *)take((size_t)p->total_pix * 4);
    if (p->t_mode == 1) {
        b.ckpt = (float4 *)take(((size_t)p->cap / p->batch + 1) * p->tile * p->tile * sizeof(float4));
        b.fstate = (float4 *)take((size_t)p->total_pix * sizeof(float4));
    }
    if (p->t_mode == 2) b.tstore = (float *)take((size_t)p->cap * p->tile * p->tile * sizeof(float));
    b.g2d = (float *)take(9 * R * 4);
    b.m_dev = (uint32_t *)take(4);
    b.a_dev = (uint32_t *)take(4);
    b.flags = (uint32_t *)take(4);
    b.mask_count = (uint32_t *)take(4);
    b.m_total = (unsigned long long *)take(8);
    b.counters = (unsigned long long *)take(3 * 8);
    b.loss_partial = (float *)take((size_t)loss_partials(p->total_pix) * 4);
    b.bg = (float *)take(p->views.size() * 3 * sizeof(float));
    b.views = (ViewDesc *)take(p->views.size() * sizeof(ViewDesc));
    b.vis = (uint8_t *)take((size_t)p->n_max);
    if (out) *out = b;
    return off;
}

gsf_status check_ready(gsf_plan *p) {
    if (!p) return GSF_E_INVALID;
    if (!p->ws) return fail(p->ctx, GSF_E_STATE, "no workspace bound to the plan");
    return GSF_OK;
}

SplatPtrs splats(gsf_plan *p) { return SplatPtrs{p->b.rec}; }

RenderArgs render_args(gsf_plan *p, const gsf_camera *cams, int64_t n) {
    RenderArgs a;
    a.tile = p->tile;
    a.batch = p->batch;
    a.total_tiles = (int)(p->fwd_tiles > 0 ? p->fwd_tiles : p->total_tiles);
    a.tm = p->fwd_tm;
    a.nviews = p->V;
    a.nrec = (int)(n * p->V);
    a.t_mode = p->t_mode;
    a.order = p->b.order;
    a.bwd_grid = p->bwd_grid;
    a.ranges = p->b.ranges;
    a.vals = p->b.vals;
    a.sp = splats(p);
    a.views = p->b.views;
    a.cams = cams;
    a.tfinal = p->b.tfinal;
    a.ncontrib = p->b.ncontrib;
    a.ckpt = p->b.ckpt;
    a.fstate = p->b.fstate;
    a.tstore = p->b.tstore;
    a.m_dev = p->host_sized ? nullptr : p->b.m_dev;
    a.m_host = p->m_host;
    a.cus = p->ctx->cus;
    a.kp.koff = p->b.koff;
    a.kp.count = p->b.count;
    a.kp.rect = p->b.rect;
    a.kp.rspan = p->b.rspan;
    a.kp.rowtab = p->b.rowtab;
    a.kp.pg = p->b.pg;
    a.kp.m_total = p->b.m_total;
    a.kp.capacity = p->cap;
    return a;
}

hipEvent_t take_event(gsf_plan *p) {
    if (!p->pool.empty()) {
        hipEvent_t e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

gsf_status flush_timing(gsf_plan *p) {
    for (auto &q : p->pending) {
        float ms = 0.f;
        GSF_HIP(p->ctx, hipEventSynchronize(q.b));
        GSF_HIP(p->ctx, hipEventElapsedTime(&ms, q.a, q.b));
        p->stage_ms[q.stage] += ms;
        p->stage_calls[q.stage] += 1;
        p->pool.push_back(q.a);
        p->pool.push_back(q.b);
    }
    p->pending.clear();
    return GSF_OK;
}

// Brackets one stage with events when timing is on.
struct StageTimer {
    gsf_plan *p;
    int stage;
    hipEvent_t a = nullptr;
    StageTimer(gsf_plan *plan, int st) : p(plan), stage(st) {
        if (p->timing && (a = take_event(p))) hipEventRecord(a, p->ctx->stream);
    }
    ~StageTimer() {
        if (!a) return;
        hipEvent_t b = take_event(p);
        if (!b) return;
        hipEventRecord(b, p->ctx->stream);
        p->pending.push_back({stage, a, b});
    }
};

// Side of the per-view pixel window that holds every tile meeting the fovea
// (0 when the window would not be smaller than the views).
int max_height(const gsf_plan *p) {
    int h = 0;
    for (const ViewDesc &vd : p->views) h = std::max(h, (int)vd.height);
    return h;
}

int fovea_box(const gsf_plan *p, float radius_frac) {
    int wmax = 1;
    for (const ViewDesc &vd : p->views) wmax = std::max(wmax, (int)vd.width);
    const double r = (double)radius_frac * wmax;
    const int64_t tiles = (int64_t)std::ceil((2.0 * r + 4.0) / p->tile) + 1;
    const int64_t side = tiles * p->tile;
    return side > 0 && (int64_t)p->V * side * side <= p->total_pix ? (int)side : 0;
}

// cull_gaze (nullable): fovea culling with radius fraction cull_radius.
gsf_status enqueue_forward(gsf_plan *p, const float *params, int64_t n, const gsf_camera *cams,
                           float *out_rgba, bool *overflow, const float *cull_gaze = nullptr,
                           float cull_radius = 0.f, const float *bg = nullptr) {
    gsf_ctx *ctx = p->ctx;
    hipStream_t s = ctx->stream;
    Buffers &b = p->b;
    const int nrec = (int)(n * p->V);
    *overflow = false;
    if (p->timing && p->pending.size() > 512) {
        gsf_status fs = flush_timing(p);
        if (fs != GSF_OK) return fs;
    }
    {   // splats, support boxes and their tile counts, depth keys
        StageTimer t(p, GSF_STAGE_PROJECT);
        const FoveaRows fr{cull_gaze ? b.fovea_rows : nullptr, fovea_rows_per_view(p)};
        if (cull_gaze) launch_fovea_rows(s, cull_gaze, cull_radius, b.views, p->V, p->tile, fr);
        launch_project_fwd(s, params, (int)n, p->V, p->deg, cams, b.views, p->tile, splats(p),
                           b.depth_key, b.rect, b.count, b.rspan, cull_gaze, cull_radius, fr,
                           b.block_sums, b.block_act);
    }
    GSF_LAUNCHED(ctx);
    {   // record-order scan: gradient slots, row tables, key total + capacity check on
        // the device; the records with keys compacted with their depths
        StageTimer t(p, GSF_STAGE_DUPLICATE);
        launch_scan_records(s, b.count, b.rect, b.rspan, splats(p), b.depth_key, b.koff,
                            b.rowtab, nrec, (int)n, p->tile, b.views,
                            FoveaRows{cull_gaze ? b.fovea_rows : nullptr, fovea_rows_per_view(p)},
                            b.block_sums, b.block_act,
                            b.seg_tot, b.seg_act, b.m_dev, b.m_total, b.a_dev, b.flags, p->cap,
                            b.k0, b.v0, b.arec, b.ranges, (int)p->total_tiles);
    }
    GSF_LAUNCHED(ctx);
    if (p->host_sized) {   // plain path: one host synchronisation per forward
        GSF_HIP(ctx, hipMemcpyAsync(p->pinned, b.m_total, 8, hipMemcpyDeviceToHost, s));
        GSF_HIP(ctx, hipStreamSynchronize(s));
        const unsigned long long total = *p->pinned;
        *overflow = total > (unsigned long long)p->cap;
        p->m_host = *overflow ? 0u : (uint32_t)total;
    }
    const uint32_t *m_dev = p->host_sized ? nullptr : b.m_dev;
    // fovea culling: keys in the compact space of the views' fovea boxes (fewer
    // bits to sort) when that space is smaller than the plan's tiles
    TileMap tm;
    int sort_bits = p->tile_bits;
    if (cull_gaze) {
        const int box = fovea_box(p, cull_radius) / p->tile;
        const int64_t space = (int64_t)p->V * box * box;
        if (box > 0 && space < p->total_tiles) {
            tm = TileMap{cull_gaze, cull_radius, box, p->tile};
            sort_bits = 0;
            while ((int64_t(1) << sort_bits) < space) sort_bits++;
        }
    }
    // ranges, the compositing order and the compositing launches then cover
    // only those tiles
    const int64_t ltiles = tm.gaze ? (int64_t)p->V * tm.box * tm.box : p->total_tiles;
    p->fwd_tm = tm;
    p->fwd_tiles = ltiles;
    {   // depth order of the records with keys (stable: equal depths keep the
        // record order), then their keys emitted in that order
        StageTimer t(p, GSF_STAGE_DEPTH_SORT);
        launch_depth_sort(s, b.k0, b.v0, b.k1, b.v1, b.a_dev, p->radix_grid, b.hist, b.digit_tot,
                          b.depth_mm, b.depth_ctl, b.dsorted);
        launch_emit(s, b.dsorted, b.a_dev, b.arec, b.rowtab, nrec, (int)n, b.views, p->V,
                    b.emit_sums, b.seg_tot, b.m_total, p->cap, tm, b.ek, b.ev);
    }
    GSF_LAUNCHED(ctx);
    {   // stable by tile: each tile's keys stay in (depth, record) order
        StageTimer t(p, GSF_STAGE_TILE_SORT);
        const int grid = p->host_sized ? radix_grid_for(p->m_host) : p->radix_grid;
        const int where = launch_radix_sort(s, b.ek, b.ev, b.tk, b.tv, b.ek, b.ev, m_dev, p->m_host,
                                            sort_bits, grid, b.hist, b.digit_tot);
        p->b.keys = where == 1 ? b.tk : b.ek;   // the sorted pair (passes depend on the key space)
        p->b.vals = where == 1 ? b.tv : b.ev;
    }
    GSF_LAUNCHED(ctx);
    {
        StageTimer t(p, GSF_STAGE_RANGES);
        launch_tile_bounds(s, b.keys, m_dev, p->m_host, p->cap, (int)ltiles, b.views, p->V,
                           TileMap{}, b.ranges);
        launch_tile_order(s, b.ranges, (int)ltiles, b.order, b.order_counts);
    }
    GSF_LAUNCHED(ctx);
    {
        StageTimer t(p, GSF_STAGE_RENDER);
        RenderArgs ra = render_args(p, cams, n);
        ra.cull_gaze = cull_gaze;
        ra.cull_radius = cull_radius;
        ra.bg = bg;
        launch_render_fwd(s, ra, out_rgba);
    }
    GSF_LAUNCHED(ctx);
    p->have_forward = true;
    p->fwd_culled = cull_gaze != nullptr;
    p->fwd_cull_gaze = cull_gaze;
    p->fwd_cull_radius = cull_radius;
    p->fwd_n = n;
    return GSF_OK;
}

// cull: visit only the pixels of the tiles that meet each view's fovea (gaze
// required) - a window of box x box pixels per view, when that is smaller.
// tgt_planes 4: RGBA targets composited over bg (nullable) with an alpha term
// when alpha_term.
gsf_status enqueue_loss(gsf_plan *p, const float *rgba, const float *target, const float *gaze,
                        float radius_frac, float *loss, float *dl, int32_t *step_inc,
                        bool cull = false, int tgt_planes = 3, bool alpha_term = false,
                        const float *bg = nullptr, uint32_t norm_count = 0u,
                        bool accumulate = false) {
    const int box = cull && gaze ? fovea_box(p, radius_frac) : 0;
    StageTimer t(p, GSF_STAGE_LOSS);
    launch_loss_l1(p->ctx->stream, rgba, target, gaze, radius_frac, p->b.views, p->V,
                   p->total_pix, dl, p->b.loss_partial, p->b.mask_count, loss, p->b.flags,
                   step_inc, box, p->tile, tgt_planes, alpha_term, bg, norm_count, accumulate,
                   max_height(p));
    GSF_LAUNCHED(p->ctx);
    return GSF_OK;
}

gsf_status enqueue_backward(gsf_plan *p, const float *params, int64_t n, const gsf_camera *cams,
                            const float *dl, float *grads, const float *bg = nullptr,
                            bool accumulate = false) {
    hipStream_t s = p->ctx->stream;
    RenderArgs ra = render_args(p, cams, n);
    ra.bg = bg;
    {   // per-key screen-space gradients
        StageTimer t(p, GSF_STAGE_RENDER_BWD);
        launch_render_bwd(s, ra, dl);
    }
    GSF_LAUNCHED(p->ctx);
    if (!project_bwd_sums_keys(p->deg)) {   // their per-record sums (every entry of g2d written)
        StageTimer t(p, GSF_STAGE_GRAD_SUM);
        launch_grad_sum(s, ra.kp, (int)(n * p->V), p->b.g2d);
    }
    GSF_LAUNCHED(p->ctx);
    {   // the chain rule to the parameters (summing the per-key terms itself for SH 0-1)
        StageTimer t(p, GSF_STAGE_PROJECT_BWD);
        launch_project_bwd(s, params, (int)n, p->V, p->deg, cams, ra.kp, p->b.g2d, grads, accumulate);
    }
    GSF_LAUNCHED(p->ctx);
    return GSF_OK;
}

bool aligned16(const void *ptr) { return ((uintptr_t)ptr & 15u) == 0; }

gsf_status make_segments(gsf_ctx *ctx, int64_t n_elems, const int64_t *seg_off, const float *seg_lr,
                         int32_t n_seg, SegTable *seg) {
    if (!seg_off || !seg_lr || n_seg < 1 || n_seg > kMaxSeg)
        return fail(ctx, GSF_E_INVALID, "gsf_adam: need 1..16 segments with host offsets and rates");
    if (seg_off[0] != 0 || seg_off[n_seg] != n_elems)
        return fail(ctx, GSF_E_INVALID, "gsf_adam: segments must start at 0 and end at n_elems");
    std::memset(seg, 0, sizeof *seg);
    for (int s = 0; s < n_seg; s++) {
        if (seg_off[s + 1] < seg_off[s])
            return fail(ctx, GSF_E_INVALID, "gsf_adam: segment offsets must be non-decreasing");
        seg->off[s] = seg_off[s];
        seg->lr[s] = seg_lr[s];
    }
    seg->off[n_seg] = seg_off[n_seg];
    seg->n = n_seg;
    return GSF_OK;
}

gsf_status check_step(gsf_plan *p, const gsf_step_args *a) {
    if (!a || !a->params || !a->cams || !a->target_rgb || !a->loss || !a->rgba || !a->dl_drgba ||
        !a->grads || !a->adam_m || !a->adam_v || !a->step_dev || !a->seg_lr)
        return fail(p->ctx, GSF_E_INVALID, "gsf_step: null argument");
    if (a->n < 1 || a->n > p->n_max) return fail(p->ctx, GSF_E_INVALID, "gsf_step: n out of range");
    if (!aligned16(a->params) || !aligned16(a->grads) || !aligned16(a->adam_m) || !aligned16(a->adam_v))
        return fail(p->ctx, GSF_E_INVALID, "gsf_step: parameter buffers must be 16-byte aligned");
    if (a->fovea_cull != 0 && a->fovea_cull != 1)
        return fail(p->ctx, GSF_E_INVALID, "gsf_step: fovea_cull must be 0 or 1");
    if (a->fovea_cull && !a->gaze_px)
        return fail(p->ctx, GSF_E_INVALID, "gsf_step: fovea_cull needs gaze_px");
    if (a->fovea_cull && !(a->mask_radius_frac >= 0.f && a->mask_radius_frac <= 4.f))
        return fail(p->ctx, GSF_E_INVALID, "gsf_step: mask_radius_frac must lie in [0, 4]");
    if ((a->alpha_loss != 0 && a->alpha_loss != 1) || (a->random_bg != 0 && a->random_bg != 1))
        return fail(p->ctx, GSF_E_INVALID, "gsf_step: alpha_loss and random_bg must be 0 or 1");
    if (a->random_bg && !a->alpha_loss)
        return fail(p->ctx, GSF_E_INVALID, "gsf_step: random_bg needs alpha_loss (RGBA targets)");
    if (a->masked_adam != 0 && a->masked_adam != 1)
        return fail(p->ctx, GSF_E_INVALID, "gsf_step: masked_adam must be 0 or 1");
    return GSF_OK;
}

// with_adam = false: forward, loss and backward only (the autotuner's timing,
// which leaves parameters and moments alone).
gsf_status enqueue_step(gsf_plan *p, const gsf_step_args *a, bool with_adam = true) {
    bool overflow = false;
    const bool cull = a->fovea_cull != 0;
    const float *bg = nullptr;
    if (a->random_bg) {   // this step's backgrounds, from the step counter on the device
        launch_draw_bg(p->ctx->stream, a->bg_seed, a->step_dev, p->V, p->b.bg);
        GSF_LAUNCHED(p->ctx);
        bg = p->b.bg;
    }
    gsf_status st = enqueue_forward(p, a->params, a->n, a->cams, a->rgba, &overflow,
                                    cull ? a->gaze_px : nullptr, a->mask_radius_frac, bg);
    if (st != GSF_OK) return st;
    // the loss reduction also advances the Adam step counter of this step
    st = enqueue_loss(p, a->rgba, a->target_rgb, a->gaze_px, a->mask_radius_frac, a->loss,
                      a->dl_drgba, a->step_dev, cull, a->alpha_loss ? 4 : 3, a->alpha_loss != 0, bg);
    if (st != GSF_OK) return st;
    st = enqueue_backward(p, a->params, a->n, a->cams, a->dl_drgba, a->grads, bg);
    if (st != GSF_OK) return st;
    if (!with_adam) return overflow ? fail(p->ctx, GSF_E_CAPACITY, "key capacity exceeded") : GSF_OK;
    const int C = planes_of(p->deg);
    std::vector<int64_t> off(C + 1);
    for (int c = 0; c <= C; c++) off[c] = (int64_t)c * a->n;
    // merge equal neighbouring planes into segments (at most 16)
    std::vector<int64_t> so{0};
    std::vector<float> sl{a->seg_lr[0]};
    for (int c = 1; c < C; c++) {
        if (a->seg_lr[c] != sl.back()) {
            so.push_back(off[c]);
            sl.push_back(a->seg_lr[c]);
        }
    }
    so.push_back(off[C]);
    SegTable seg;
    st = make_segments(p->ctx, off[C], so.data(), sl.data(), (int32_t)sl.size(), &seg);
    if (st != GSF_OK) return st;
    if (a->masked_adam) {   // only the Gaussians that touched a tile in some view
        StageTimer t(p, GSF_STAGE_ADAM);
        PlaneLr lr{};
        for (int c = 0; c < C; c++) lr.lr[c] = a->seg_lr[c];
        launch_visible(p->ctx->stream, p->b.count, (int)a->n, p->V, p->b.vis);
        launch_adam_masked(p->ctx->stream, a->params, a->grads, a->adam_m, a->adam_v, a->n, C, lr,
                           p->b.vis, a->beta1, a->beta2, a->eps, a->step_dev, false, p->b.flags);
    } else {
        StageTimer t(p, GSF_STAGE_ADAM);
        launch_adam(p->ctx->stream, a->params, a->grads, a->adam_m, a->adam_v, off[C], seg,
                    a->beta1, a->beta2, a->eps, a->step_dev, false, p->b.flags);
    }
    GSF_LAUNCHED(p->ctx);
    return overflow ? fail(p->ctx, GSF_E_CAPACITY, "key capacity exceeded") : GSF_OK;
}

}  // namespace

extern "C" {

gsf_status gsf_ctx_create(int device, void *hip_stream, gsf_ctx **out) {
    if (!out) return GSF_E_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return GSF_E_HIP;
    if (hipSetDevice(device) != hipSuccess) return GSF_E_HIP;
    gsf_ctx *c = new (std::nothrow) gsf_ctx;
    if (!c) return GSF_E_INVALID;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cus = cus;
    // the no-allocation warp's z-buffer: its address on this device, found once
    c->warp_scratch_err = warp_scratch_address(device, &c->warp_scratch);
    *out = c;
    return GSF_OK;
}

gsf_status gsf_ctx_destroy(gsf_ctx *ctx) {
    delete ctx;
    return GSF_OK;
}

gsf_status gsf_ctx_set_stream(gsf_ctx *ctx, void *hip_stream) {
    if (!ctx) return GSF_E_INVALID;
    ctx->stream = (hipStream_t)hip_stream;
    return GSF_OK;
}

const char *gsf_last_error(const gsf_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gsf_status gsf_plan_create(gsf_ctx *ctx, const gsf_plan_desc *d, gsf_plan **out) {
    if (!ctx || !d || !out) return fail(ctx, GSF_E_INVALID, "gsf_plan_create: null argument");
    *out = nullptr;
    if (d->n_max < 1) return fail(ctx, GSF_E_INVALID, "n_max must be >= 1");
    if (d->sh_degree < 0 || d->sh_degree > 3) return fail(ctx, GSF_E_INVALID, "sh_degree must be 0..3");
    if (d->n_views < 1 || d->n_views > kMaxViews) return fail(ctx, GSF_E_INVALID, "n_views must be 1..64");
    if (!d->widths || !d->heights) return fail(ctx, GSF_E_INVALID, "widths/heights are null");
    if (d->tile != 8 && d->tile != 16 && d->tile != 32) return fail(ctx, GSF_E_INVALID, "tile must be 8, 16 or 32");
    if (d->lds_batch != 64 && d->lds_batch != 128 && d->lds_batch != 256)
        return fail(ctx, GSF_E_INVALID, "lds_batch must be 64, 128 or 256");
    if (d->t_mode < 0 || d->t_mode > 2) return fail(ctx, GSF_E_INVALID, "t_mode must be 0, 1 or 2");
    if (d->host_sized != 0 && d->host_sized != 1) return fail(ctx, GSF_E_INVALID, "host_sized must be 0 or 1");
    if (d->key_capacity < 0 || d->key_capacity > 0xF0000000ll)
        return fail(ctx, GSF_E_INVALID, "key_capacity out of range");
    const int64_t nrec = d->n_max * d->n_views;
    if (nrec > 0x7FFFFFFFll) return fail(ctx, GSF_E_INVALID, "n_max * n_views must fit in 31 bits");
    gsf_plan *p = new (std::nothrow) gsf_plan;
    if (!p) return fail(ctx, GSF_E_INVALID, "out of host memory");
    p->ctx = ctx;
    p->n_max = d->n_max;
    p->deg = d->sh_degree;
    p->V = d->n_views;
    p->tile = d->tile;
    p->batch = d->lds_batch;
    p->t_mode = d->t_mode;
    p->host_sized = d->host_sized;
    p->nrec_max = nrec;
    int64_t toff = 0, poff = 0;
    for (int v = 0; v < p->V; v++) {
        const int W = d->widths[v], H = d->heights[v];
        if (W < 1 || H < 1 || W > 8192 || H > 8192) {
            delete p;
            return fail(ctx, GSF_E_INVALID, "view sizes must be 1..8192");
        }
        ViewDesc vd{};
        vd.tile_off = (int32_t)toff;
        vd.tiles_x = (W + p->tile - 1) / p->tile;
        vd.tiles_y = (H + p->tile - 1) / p->tile;
        vd.pix_off = (int32_t)poff;
        vd.width = W;
        vd.height = H;
        p->views.push_back(vd);
        toff += (int64_t)vd.tiles_x * vd.tiles_y;
        poff += (int64_t)W * H;
    }
    if (poff > 0x7FFFFFFFll) {
        delete p;
        return fail(ctx, GSF_E_INVALID, "total pixels must fit in 31 bits");
    }
    p->total_tiles = toff;
    p->total_pix = poff;
    p->cap = d->key_capacity > 0 ? d->key_capacity : 32 * nrec + (1 << 20);
    if (p->cap > 0xF0000000ll) p->cap = 0xF0000000ll;
    p->tile_bits = 0;                         // bits of the largest global tile id
    while ((int64_t(1) << p->tile_bits) < p->total_tiles) p->tile_bits++;
    p->radix_grid = radix_grid_for(p->cap);
    // checkpointed adjoint: one workgroup per possible (tile, batch) unit id
    p->bwd_grid = (int)std::max<int64_t>(1, std::min<int64_t>(p->cap / p->batch + p->total_tiles,
                                                               0x7FFFFFFFll));
    p->ws_bytes = carve(p, nullptr, nullptr);
    if (hipHostMalloc((void **)&p->pinned, sizeof(unsigned long long)) != hipSuccess) {
        delete p;
        return fail(ctx, GSF_E_HIP, "hipHostMalloc failed");
    }
    *out = p;
    return GSF_OK;
}

gsf_status gsf_plan_workspace_bytes(const gsf_plan *p, size_t *bytes) {
    if (!p || !bytes) return GSF_E_INVALID;
    *bytes = p->ws_bytes;
    return GSF_OK;
}

gsf_status gsf_plan_info(const gsf_plan *p, int64_t *total_tiles, int64_t *total_pixels) {
    if (!p) return GSF_E_INVALID;
    if (total_tiles) *total_tiles = p->total_tiles;
    if (total_pixels) *total_pixels = p->total_pix;
    return GSF_OK;
}

gsf_status gsf_plan_bind_workspace(gsf_plan *p, void *dev, size_t bytes) {
    if (!p || !dev) return fail(p ? p->ctx : nullptr, GSF_E_INVALID, "gsf_plan_bind_workspace: null");
    if (bytes < p->ws_bytes) return fail(p->ctx, GSF_E_INVALID, "workspace too small");
    if (((uintptr_t)dev & 255u) != 0) return fail(p->ctx, GSF_E_INVALID, "workspace must be 256-byte aligned");
    p->ws = dev;
    carve(p, (char *)dev, &p->b);
    p->have_forward = false;
    GSF_HIP(p->ctx, hipMemcpyAsync(p->b.views, p->views.data(), p->views.size() * sizeof(ViewDesc),
                                   hipMemcpyHostToDevice, p->ctx->stream));
    launch_fill_u32(p->ctx->stream, p->b.flags, 1, 0u);
    launch_fill_u32(p->ctx->stream, p->b.m_dev, 1, 0u);
    GSF_LAUNCHED(p->ctx);
    GSF_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
    return GSF_OK;
}

gsf_status gsf_plan_destroy(gsf_plan *p) {
    if (!p) return GSF_OK;
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->pinned) hipHostFree(p->pinned);
    for (auto &q : p->pending) {
        hipEventDestroy(q.a);
        hipEventDestroy(q.b);
    }
    for (auto e : p->pool) hipEventDestroy(e);
    delete p;
    return GSF_OK;
}

gsf_status gsf_forward(gsf_plan *p, const float *params, int64_t n, const gsf_camera *cams,
                       const float *cull_gaze_px, float cull_radius_frac, float *out_rgba) {
    gsf_status st = check_ready(p);
    if (st != GSF_OK) return st;
    if (!params || !cams || !out_rgba) return fail(p->ctx, GSF_E_INVALID, "gsf_forward: null argument");
    if (n < 1 || n > p->n_max) return fail(p->ctx, GSF_E_INVALID, "gsf_forward: n out of range");
    if (cull_gaze_px && !(cull_radius_frac >= 0.f && cull_radius_frac <= 4.f))
        return fail(p->ctx, GSF_E_INVALID, "gsf_forward: cull_radius_frac must lie in [0, 4]");
    bool overflow = false;
    st = enqueue_forward(p, params, n, cams, out_rgba, &overflow, cull_gaze_px, cull_radius_frac);
    if (st != GSF_OK) return st;
    return overflow ? fail(p->ctx, GSF_E_CAPACITY, "key capacity exceeded") : GSF_OK;
}

gsf_status gsf_loss_l1(gsf_plan *p, const float *rgba, const float *target_rgb, const float *gaze_px,
                       float mask_radius_frac, int64_t norm_count, int32_t accumulate, float *loss,
                       float *dl_drgba) {
    gsf_status st = check_ready(p);
    if (st != GSF_OK) return st;
    if (!rgba || !target_rgb || !loss || !dl_drgba) return fail(p->ctx, GSF_E_INVALID, "gsf_loss_l1: null argument");
    if (gaze_px && !(mask_radius_frac >= 0.f)) return fail(p->ctx, GSF_E_INVALID, "gsf_loss_l1: bad radius");
    if (norm_count < 0 || norm_count > 0xFFFFFFFFll)
        return fail(p->ctx, GSF_E_INVALID, "gsf_loss_l1: norm_count must lie in [0, 2^32 - 1]");
    if (accumulate != 0 && accumulate != 1)
        return fail(p->ctx, GSF_E_INVALID, "gsf_loss_l1: accumulate must be 0 or 1");
    // after a fovea-culled forward only the fovea tiles hold this step's image
    const bool cull = gaze_px && p->have_forward && p->fwd_culled;
    return enqueue_loss(p, rgba, target_rgb, gaze_px, mask_radius_frac, loss, dl_drgba, nullptr,
                        cull, 3, false, nullptr, (uint32_t)norm_count, accumulate != 0);
}

gsf_status gsf_loss_count(gsf_plan *p, const float *gaze_px, float mask_radius_frac,
                          int64_t *count) {
    gsf_status st = check_ready(p);
    if (st != GSF_OK) return st;
    if (!count) return fail(p->ctx, GSF_E_INVALID, "gsf_loss_count: null count");
    if (!gaze_px) {
        *count = 3 * p->total_pix;
        return GSF_OK;
    }
    if (!(mask_radius_frac >= 0.f)) return fail(p->ctx, GSF_E_INVALID, "gsf_loss_count: bad radius");
    launch_loss_count(p->ctx->stream, gaze_px, mask_radius_frac, p->b.views, p->V, max_height(p),
                      fovea_box(p, mask_radius_frac), p->tile, 3u, p->b.mask_count);
    GSF_LAUNCHED(p->ctx);
    uint32_t c = 0;
    GSF_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
    GSF_HIP(p->ctx, hipMemcpy(&c, p->b.mask_count, 4, hipMemcpyDeviceToHost));
    *count = c;
    return GSF_OK;
}

gsf_status gsf_loss_l1_rgba(gsf_plan *p, const float *rgba, const float *target_rgba,
                            const float *bg, int32_t alpha, const float *gaze_px,
                            float mask_radius_frac, float *loss, float *dl_drgba) {
    gsf_status st = check_ready(p);
    if (st != GSF_OK) return st;
    if (!rgba || !target_rgba || !loss || !dl_drgba)
        return fail(p->ctx, GSF_E_INVALID, "gsf_loss_l1_rgba: null argument");
    if (alpha != 0 && alpha != 1) return fail(p->ctx, GSF_E_INVALID, "gsf_loss_l1_rgba: alpha must be 0 or 1");
    if (gaze_px && !(mask_radius_frac >= 0.f))
        return fail(p->ctx, GSF_E_INVALID, "gsf_loss_l1_rgba: bad radius");
    return enqueue_loss(p, rgba, target_rgba, gaze_px, mask_radius_frac, loss, dl_drgba, nullptr,
                        false, 4, alpha != 0, bg);
}

gsf_status gsf_backward(gsf_plan *p, const float *params, int64_t n, const gsf_camera *cams,
                        const float *dl_drgba, int32_t accumulate, float *grads) {
    gsf_status st = check_ready(p);
    if (st != GSF_OK) return st;
    if (!params || !cams || !dl_drgba || !grads) return fail(p->ctx, GSF_E_INVALID, "gsf_backward: null argument");
    if (accumulate != 0 && accumulate != 1)
        return fail(p->ctx, GSF_E_INVALID, "gsf_backward: accumulate must be 0 or 1");
    if (!p->have_forward) return fail(p->ctx, GSF_E_STATE, "gsf_backward before gsf_forward");
    if (n != p->fwd_n) return fail(p->ctx, GSF_E_INVALID, "gsf_backward: n differs from the forward");
    return enqueue_backward(p, params, n, cams, dl_drgba, grads, nullptr, accumulate != 0);
}

gsf_status gsf_seed_scratch_bytes(int32_t n, size_t *bytes) {
    if (!bytes || n < 1 || n > 2048) return GSF_E_INVALID;
    *bytes = seed_scratch_bytes((int64_t)n * n * n);
    return GSF_OK;
}

gsf_status gsf_seed_volume(gsf_ctx *ctx, const uint16_t *vol, int32_t n, double threshold,
                           double range, const double *lo, const double *hi, double opacity,
                           int64_t cap, uint64_t seed, float *params, int64_t *count,
                           void *scratch, size_t scratch_bytes) {
    if (!ctx) return GSF_E_INVALID;
    if (!vol || !lo || !hi || !params || !count || !scratch)
        return fail(ctx, GSF_E_INVALID, "gsf_seed_volume: null argument");
    if (n < 1 || n > 2048) return fail(ctx, GSF_E_INVALID, "gsf_seed_volume: n must lie in [1, 2048]");
    if (cap < 1) return fail(ctx, GSF_E_INVALID, "gsf_seed_volume: cap must be positive");
    if (!(range > 0.0)) return fail(ctx, GSF_E_INVALID, "gsf_seed_volume: range must be positive");
    if (!(opacity > 0.0 && opacity < 1.0)) return fail(ctx, GSF_E_INVALID, "gsf_seed_volume: opacity must lie in (0, 1)");
    if (scratch_bytes < seed_scratch_bytes((int64_t)n * n * n))
        return fail(ctx, GSF_E_INVALID, "gsf_seed_volume: scratch too small");
    GSF_HIP(ctx, run_seed(ctx->stream, vol, n, threshold, range, lo, hi, opacity, cap, seed, params,
                          count, scratch));
    return GSF_OK;
}

gsf_status gsf_raymarch(gsf_ctx *ctx, const uint16_t *vol, int32_t n, const gsf_camera *cams,
                        int32_t n_views, const int32_t *widths, const int32_t *heights, float step,
                        float extinction, float t_stop, float threshold, float range,
                        const float *lo, const float *hi, float *out_rgba) {
    if (!ctx) return GSF_E_INVALID;
    if (!vol || !cams || !widths || !heights || !lo || !hi || !out_rgba)
        return fail(ctx, GSF_E_INVALID, "gsf_raymarch: null argument");
    if (n < 1 || n > 2048 || n_views < 1 || n_views > kMaxViews)
        return fail(ctx, GSF_E_INVALID, "gsf_raymarch: n or n_views out of range");
    for (int v = 0; v < n_views; v++)
        if (widths[v] < 1 || heights[v] < 1 || widths[v] > 8192 || heights[v] > 8192)
            return fail(ctx, GSF_E_INVALID, "gsf_raymarch: image size out of range");
    if (!(step > 0.f) || !(range > 0.f) || !(t_stop >= 0.f) || !(extinction >= 0.f))
        return fail(ctx, GSF_E_INVALID, "gsf_raymarch: step, range, extinction or t_stop invalid");
    GSF_HIP(ctx, run_raymarch(ctx->stream, vol, n, cams, n_views, widths, heights, step, extinction,
                              t_stop, threshold, range, lo, hi, out_rgba));
    return GSF_OK;
}

gsf_status gsf_adam(gsf_ctx *ctx, float *prm, const float *g, float *m, float *v, int64_t n_elems,
                    const int64_t *seg_off, const float *seg_lr, int32_t n_seg, float beta1,
                    float beta2, float eps, int32_t *step_dev) {
    if (!ctx) return GSF_E_INVALID;
    if (!prm || !g || !m || !v || !step_dev || n_elems < 1)
        return fail(ctx, GSF_E_INVALID, "gsf_adam: null argument or empty");
    if (!aligned16(prm) || !aligned16(g) || !aligned16(m) || !aligned16(v))
        return fail(ctx, GSF_E_INVALID, "gsf_adam: buffers must be 16-byte aligned");
    SegTable seg;
    gsf_status st = make_segments(ctx, n_elems, seg_off, seg_lr, n_seg, &seg);
    if (st != GSF_OK) return st;
    launch_adam(ctx->stream, prm, g, m, v, n_elems, seg, beta1, beta2, eps, step_dev, true);
    GSF_LAUNCHED(ctx);
    return GSF_OK;
}

gsf_status gsf_adam_masked(gsf_ctx *ctx, float *prm, const float *g, float *m, float *v,
                           int64_t n, int32_t planes, const float *plane_lr,
                           const uint8_t *visible, float beta1, float beta2, float eps,
                           int32_t *step_dev) {
    if (!ctx) return GSF_E_INVALID;
    if (!prm || !g || !m || !v || !plane_lr || !visible || !step_dev)
        return fail(ctx, GSF_E_INVALID, "gsf_adam_masked: null argument");
    if (n < 1 || planes < 1 || planes > kMaxPlanes || n > (int64_t)1 << 40)
        return fail(ctx, GSF_E_INVALID, "gsf_adam_masked: n or planes out of range");
    PlaneLr lr{};
    for (int c = 0; c < planes; c++) {
        if (!std::isfinite(plane_lr[c]))
            return fail(ctx, GSF_E_INVALID, "gsf_adam_masked: non-finite learning rate");
        lr.lr[c] = plane_lr[c];
    }
    launch_adam_masked(ctx->stream, prm, g, m, v, n, planes, lr, visible, beta1, beta2, eps,
                       step_dev, true);
    GSF_LAUNCHED(ctx);
    return GSF_OK;
}

gsf_status gsf_adam_reset(gsf_ctx *ctx, float *m, float *v, int64_t n_elems, int32_t *step_dev) {
    if (!ctx) return GSF_E_INVALID;
    if (!m || !v || !step_dev || n_elems < 1)
        return fail(ctx, GSF_E_INVALID, "gsf_adam_reset: null argument or empty");
    if (!aligned16(m) || !aligned16(v))
        return fail(ctx, GSF_E_INVALID, "gsf_adam_reset: buffers must be 16-byte aligned");
    launch_adam_reset(ctx->stream, m, v, n_elems, step_dev);
    GSF_LAUNCHED(ctx);
    return GSF_OK;
}

gsf_status gsf_first_hit_scratch_bytes(int64_t n_rays, size_t *bytes) {
    if (!bytes || n_rays < 1 || n_rays > 0x7FFFFFFFll) return GSF_E_INVALID;
    *bytes = first_hit_scratch_bytes(n_rays);
    return GSF_OK;
}

gsf_status gsf_seed_first_hits(gsf_ctx *ctx, const uint16_t *vol, int32_t n, const gsf_camera *cams,
                               int32_t n_views, const int32_t *widths, const int32_t *heights,
                               float step, float extinction, float threshold, float range,
                               const float *lo, const float *hi, float hit_alpha,
                               int32_t color_steps, double opacity, int64_t cap, uint64_t seed,
                               float *params, int32_t *ray_ids, int64_t *count, void *scratch,
                               size_t scratch_bytes) {
    if (!ctx) return GSF_E_INVALID;
    if (!vol || !cams || !widths || !heights || !lo || !hi || !params || !count || !scratch)
        return fail(ctx, GSF_E_INVALID, "gsf_seed_first_hits: null argument");
    if (n < 1 || n > 2048 || n_views < 1 || n_views > kMaxViews || cap < 1)
        return fail(ctx, GSF_E_INVALID, "gsf_seed_first_hits: n, n_views or cap out of range");
    int64_t nrays = 0;
    for (int v = 0; v < n_views; v++) {
        if (widths[v] < 1 || heights[v] < 1 || widths[v] > 8192 || heights[v] > 8192)
            return fail(ctx, GSF_E_INVALID, "gsf_seed_first_hits: image size out of range");
        nrays += (int64_t)widths[v] * heights[v];
    }
    if (nrays > 0x7FFFFFFFll)
        return fail(ctx, GSF_E_INVALID, "gsf_seed_first_hits: more than 2^31 - 1 rays");
    if (!(step > 0.f) || !(range > 0.f) || !(extinction >= 0.f) || !(hit_alpha > 0.f) ||
        !(hit_alpha < 1.f) || color_steps < 1 || !(opacity > 0.0) || !(opacity < 1.0))
        return fail(ctx, GSF_E_INVALID,
                    "gsf_seed_first_hits: step, range, extinction, hit_alpha, color_steps or "
                    "opacity invalid");
    if (scratch_bytes < first_hit_scratch_bytes(nrays))
        return fail(ctx, GSF_E_INVALID, "gsf_seed_first_hits: scratch too small");
    if (((uintptr_t)scratch & 255u) != 0)
        return fail(ctx, GSF_E_INVALID, "gsf_seed_first_hits: scratch must be 256-byte aligned");
    GSF_HIP(ctx, run_first_hits(ctx->stream, vol, n, cams, n_views, widths, heights, step,
                                extinction, threshold, range, lo, hi, hit_alpha, color_steps,
                                opacity, cap, seed, params, count, ray_ids, scratch));
    return GSF_OK;
}

gsf_status gsf_reproject(gsf_ctx *ctx, const float *depth, int32_t width, int32_t height,
                         const float *p_old, const float *v_old, const float *pos_old,
                         const float *p_new, const float *v_new, float *clip) {
    if (!ctx) return GSF_E_INVALID;
    if (!depth || !p_old || !v_old || !pos_old || !p_new || !v_new || !clip)
        return fail(ctx, GSF_E_INVALID, "gsf_reproject: null argument");
    if (width < 1 || height < 1 || width > 16384 || height > 16384)
        return fail(ctx, GSF_E_INVALID, "gsf_reproject: image size out of range");
    ReprojConstOpaque k;
    if (!make_reproj(p_old, v_old, pos_old, p_new, v_new, width, height, &k))
        return fail(ctx, GSF_E_INVALID, "gsf_reproject: singular P_old V_old or a non-finite value");
    launch_reproject(ctx->stream, k, depth, clip);
    GSF_LAUNCHED(ctx);
    return GSF_OK;
}

gsf_status gsf_reproject_warp(gsf_ctx *ctx, const float *rgba, const float *depth, int32_t width,
                              int32_t height, const float *p_old, const float *v_old,
                              const float *pos_old, const float *p_new, const float *v_new,
                              int32_t out_width, int32_t out_height, uint64_t *zbuf,
                              float *out_rgba, int32_t *out_src) {
    if (!ctx) return GSF_E_INVALID;
    if (!rgba || !depth || !p_old || !v_old || !pos_old || !p_new || !v_new || !zbuf || !out_rgba ||
        !out_src)
        return fail(ctx, GSF_E_INVALID, "gsf_reproject_warp: null argument");
    if (width < 1 || height < 1 || width > 16384 || height > 16384 || out_width < 1 ||
        out_height < 1 || out_width > 16384 || out_height > 16384)
        return fail(ctx, GSF_E_INVALID, "gsf_reproject_warp: image size out of range");
    if (((uintptr_t)zbuf & 7u) != 0)
        return fail(ctx, GSF_E_INVALID, "gsf_reproject_warp: zbuf must be 8-byte aligned");
    ReprojConstOpaque k;
    if (!make_reproj(p_old, v_old, pos_old, p_new, v_new, width, height, &k))
        return fail(ctx, GSF_E_INVALID,
                    "gsf_reproject_warp: singular P_old V_old or a non-finite value");
    launch_reproject_warp(ctx->stream, k, rgba, depth, out_width, out_height,
                          (unsigned long long *)zbuf, out_rgba, out_src);
    GSF_LAUNCHED(ctx);
    return GSF_OK;
}

gsf_status gsf_reproject_warp_noalloc(gsf_ctx *ctx, const float *rgba, const float *depth,
                                      int32_t width, int32_t height, const float *p_old,
                                      const float *v_old, const float *pos_old, const float *p_new,
                                      const float *v_new, int32_t out_width, int32_t out_height,
                                      float *out_rgba, int32_t *out_src) {
    if (!ctx) return GSF_E_INVALID;
    if (!rgba || !depth || !p_old || !v_old || !pos_old || !p_new || !v_new || !out_rgba || !out_src)
        return fail(ctx, GSF_E_INVALID, "gsf_reproject_warp_noalloc: null argument");
    if (width < 1 || height < 1 || width > 16384 || height > 16384 || out_width < 1 ||
        out_height < 1 || out_width > 16384 || out_height > 16384)
        return fail(ctx, GSF_E_INVALID, "gsf_reproject_warp_noalloc: image size out of range");
    if ((int64_t)out_width * out_height > kWarpScratchPixels)
        return fail(ctx, GSF_E_INVALID,
                    "gsf_reproject_warp_noalloc: out_width * out_height exceeds the device "
                    "z-buffer (2048 * 2304 pixels); use gsf_reproject_warp with a caller buffer");
    if (ctx->warp_scratch_err != hipSuccess || !ctx->warp_scratch)
        return fail(ctx, GSF_E_HIP, std::string("gsf_reproject_warp_noalloc: z-buffer address: ") +
                                        hipGetErrorString(ctx->warp_scratch_err));
    ReprojConstOpaque k;
    if (!make_reproj(p_old, v_old, pos_old, p_new, v_new, width, height, &k))
        return fail(ctx, GSF_E_INVALID,
                    "gsf_reproject_warp_noalloc: singular P_old V_old or a non-finite value");
    launch_reproject_warp(ctx->stream, k, rgba, depth, out_width, out_height, ctx->warp_scratch,
                          out_rgba, out_src);
    GSF_LAUNCHED(ctx);
    return GSF_OK;
}

gsf_status gsf_step(gsf_plan *p, const gsf_step_args *a) {
    gsf_status st = check_ready(p);
    if (st != GSF_OK) return st;
    st = check_step(p, a);
    if (st != GSF_OK) return st;
    return enqueue_step(p, a);
}

gsf_status gsf_step_capture(gsf_plan *p, const gsf_step_args *a) {
    gsf_status st = check_ready(p);
    if (st != GSF_OK) return st;
    if (p->host_sized) return fail(p->ctx, GSF_E_STATE, "capture needs a plan with host_sized = 0");
    if (!p->ctx->stream) return fail(p->ctx, GSF_E_STATE, "capture needs a non-null stream");
    if (p->timing) return fail(p->ctx, GSF_E_STATE, "disable stage timing before capturing");
    st = check_step(p, a);
    if (st != GSF_OK) return st;
    if (p->exec) {
        hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    if (p->graph) {
        hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    GSF_HIP(p->ctx, hipStreamBeginCapture(p->ctx->stream, hipStreamCaptureModeThreadLocal));
    gsf_status est = enqueue_step(p, a);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->ctx->stream, &g);
    if (est != GSF_OK) {
        if (g) hipGraphDestroy(g);
        return est;
    }
    if (e != hipSuccess) return fail(p->ctx, GSF_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    p->graph = g;
    GSF_HIP(p->ctx, hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return GSF_OK;
}

gsf_status gsf_step_replay(gsf_plan *p) {
    if (!p) return GSF_E_INVALID;
    if (!p->exec) return fail(p->ctx, GSF_E_STATE, "no captured step");
    GSF_HIP(p->ctx, hipGraphLaunch(p->exec, p->ctx->stream));
    return GSF_OK;
}

namespace {

gsf_status check_tune_space(gsf_ctx *ctx, const gsf_plan_desc *base, const gsf_tune_space *t) {
    if (!base || !t) return fail(ctx, GSF_E_INVALID, "gsf_autotune: null argument");
    if (t->n_tiles < 1 || t->n_tiles > 3 || t->n_batches < 1 || t->n_batches > 3 ||
        t->n_t_modes < 1 || t->n_t_modes > 3)
        return fail(ctx, GSF_E_INVALID, "gsf_autotune: 1..3 tiles, LDS batches and transmittance modes");
    for (int k = 0; k < t->n_tiles; k++) {
        if (t->tiles[k] != 8 && t->tiles[k] != 16 && t->tiles[k] != 32)
            return fail(ctx, GSF_E_INVALID, "gsf_autotune: tiles must be 8, 16 or 32");
        if (t->key_capacity[k] < 0) return fail(ctx, GSF_E_INVALID, "gsf_autotune: negative key capacity");
    }
    for (int j = 0; j < t->n_batches; j++)
        if (t->batches[j] != 64 && t->batches[j] != 128 && t->batches[j] != 256)
            return fail(ctx, GSF_E_INVALID, "gsf_autotune: LDS batches must be 64, 128 or 256");
    for (int m = 0; m < t->n_t_modes; m++)
        if (t->t_modes[m] < 0 || t->t_modes[m] > 2)
            return fail(ctx, GSF_E_INVALID, "gsf_autotune: transmittance modes must be 0, 1 or 2");
    if (t->warmup < 0 || t->reps < 1) return fail(ctx, GSF_E_INVALID, "gsf_autotune: warmup >= 0, reps >= 1");
    return GSF_OK;
}

gsf_plan_desc tune_desc(const gsf_plan_desc *base, const gsf_tune_space *t, int k, int j, int m) {
    gsf_plan_desc d = *base;
    d.tile = t->tiles[k];
    d.lds_batch = t->batches[j];
    d.t_mode = t->t_modes[m];
    d.host_sized = 0;
    d.key_capacity = t->key_capacity[k];
    return d;
}

// The autotune workspace starts with the candidates' private step counter.
constexpr size_t kTuneHead = 256;

}  // namespace

gsf_status gsf_autotune_workspace_bytes(gsf_ctx *ctx, const gsf_plan_desc *base,
                                        const gsf_tune_space *space, size_t *bytes) {
    if (!ctx) return GSF_E_INVALID;
    gsf_status st = check_tune_space(ctx, base, space);
    if (st != GSF_OK) return st;
    if (!bytes) return fail(ctx, GSF_E_INVALID, "gsf_autotune_workspace_bytes: null bytes");
    size_t most = 0;
    for (int k = 0; k < space->n_tiles; k++)
        for (int j = 0; j < space->n_batches; j++)
            for (int m = 0; m < space->n_t_modes; m++) {
                const gsf_plan_desc d = tune_desc(base, space, k, j, m);
                gsf_plan *p = nullptr;
                st = gsf_plan_create(ctx, &d, &p);
                if (st != GSF_OK) return st;
                most = std::max(most, p->ws_bytes);
                gsf_plan_destroy(p);
            }
    *bytes = kTuneHead + most;
    return GSF_OK;
}

gsf_status gsf_autotune(gsf_ctx *ctx, const gsf_plan_desc *base, const gsf_tune_space *space,
                        const gsf_step_args *args, void *workspace, size_t bytes,
                        gsf_tune_result *out) {
    if (!ctx) return GSF_E_INVALID;
    gsf_status st = check_tune_space(ctx, base, space);
    if (st != GSF_OK) return st;
    if (!args || !workspace || !out) return fail(ctx, GSF_E_INVALID, "gsf_autotune: null argument");
    if (((uintptr_t)workspace & 255u) != 0)
        return fail(ctx, GSF_E_INVALID, "gsf_autotune: workspace must be 256-byte aligned");
    if (bytes <= kTuneHead) return fail(ctx, GSF_E_INVALID, "gsf_autotune: workspace too small");
    if (!ctx->stream) return fail(ctx, GSF_E_STATE, "gsf_autotune captures graphs: needs a non-null stream");
    std::memset(out, 0, sizeof *out);
    for (int e = 0; e < 27; e++) out->ms[e] = -1.f;
    hipStream_t s = ctx->stream;
    int32_t *counter = (int32_t *)workspace;
    char *ws = (char *)workspace + kTuneHead;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GSF_HIP(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(ctx, GSF_E_HIP, "gsf_autotune: hipEventCreate failed");
    }
    float best = INFINITY;
    gsf_status result = GSF_OK;
    for (int k = 0; k < space->n_tiles && result == GSF_OK; k++)
        for (int j = 0; j < space->n_batches && result == GSF_OK; j++)
            for (int m = 0; m < space->n_t_modes && result == GSF_OK; m++) {
                const gsf_plan_desc d = tune_desc(base, space, k, j, m);
                gsf_plan *p = nullptr;
                result = gsf_plan_create(ctx, &d, &p);
                if (result != GSF_OK) break;
                float ms = INFINITY;
                do {
                    if ((result = gsf_plan_bind_workspace(p, ws, bytes - kTuneHead)) != GSF_OK) break;
                    gsf_step_args a = *args;
                    a.step_dev = counter;   // private: the caller's step count is not advanced
                    if ((result = check_step(p, &a)) != GSF_OK) break;
                    launch_fill_u32(s, (uint32_t *)counter, 1, 0u);
                    hipGraph_t g = nullptr;
                    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                        result = fail(ctx, GSF_E_HIP, "gsf_autotune: hipStreamBeginCapture failed");
                        break;
                    }
                    gsf_status est = enqueue_step(p, &a, false);
                    const hipError_t ce = hipStreamEndCapture(s, &g);
                    if (est != GSF_OK || ce != hipSuccess) {
                        if (g) hipGraphDestroy(g);
                        result = est != GSF_OK ? est : fail(ctx, GSF_E_HIP, "gsf_autotune: capture failed");
                        break;
                    }
                    p->graph = g;
                    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
                        result = fail(ctx, GSF_E_HIP, "gsf_autotune: hipGraphInstantiate failed");
                        break;
                    }
                    bool ok = true;
                    for (int w = 0; w < space->warmup && ok; w++) ok = hipGraphLaunch(p->exec, s) == hipSuccess;
                    ok = ok && hipEventRecord(e0, s) == hipSuccess;
                    for (int r = 0; r < space->reps && ok; r++) ok = hipGraphLaunch(p->exec, s) == hipSuccess;
                    ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
                    float el = 0.f;
                    ok = ok && hipEventElapsedTime(&el, e0, e1) == hipSuccess;
                    uint32_t f = 0;
                    ok = ok && hipMemcpy(&f, p->b.flags, 4, hipMemcpyDeviceToHost) == hipSuccess;
                    if (!ok) {
                        result = fail(ctx, GSF_E_HIP, "gsf_autotune: timing a candidate failed");
                        break;
                    }
                    if (!(f & GSF_FLAG_CAPACITY)) ms = el / (float)space->reps;   // else: overflowed
                } while (false);
                gsf_plan_destroy(p);
                out->ms[9 * k + 3 * j + m] = ms;
                if (result == GSF_OK && ms < best) {
                    best = ms;
                    out->tile = d.tile;
                    out->lds_batch = d.lds_batch;
                    out->t_mode = d.t_mode;
                }
            }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (result != GSF_OK) return result;
    if (!(best < INFINITY))
        return fail(ctx, GSF_E_CAPACITY, "gsf_autotune: every candidate overflowed its key capacity");
    return GSF_OK;
}

gsf_status gsf_poll(gsf_plan *p, uint32_t *flags, int64_t *m_keys) {
    gsf_status st = check_ready(p);
    if (st != GSF_OK) return st;
    if (!flags) return fail(p->ctx, GSF_E_INVALID, "gsf_poll: null flags");
    hipStream_t s = p->ctx->stream;
    uint32_t f = 0;
    unsigned long long m = 0;
    GSF_HIP(p->ctx, hipStreamSynchronize(s));
    GSF_HIP(p->ctx, hipMemcpy(&f, p->b.flags, 4, hipMemcpyDeviceToHost));
    GSF_HIP(p->ctx, hipMemcpy(&m, p->b.m_total, 8, hipMemcpyDeviceToHost));
    launch_fill_u32(s, p->b.flags, 1, 0u);
    GSF_LAUNCHED(p->ctx);
    GSF_HIP(p->ctx, hipStreamSynchronize(s));
    *flags = f;
    if (m_keys) *m_keys = (int64_t)m;
    return GSF_OK;
}

gsf_status gsf_plan_set_timing(gsf_plan *p, int enable) {
    if (!p) return GSF_E_INVALID;
    gsf_status st = flush_timing(p);
    if (st != GSF_OK) return st;
    p->timing = enable != 0;
    for (int k = 0; k < GSF_STAGE_COUNT; k++) {
        p->stage_ms[k] = 0.0;
        p->stage_calls[k] = 0;
    }
    return GSF_OK;
}

gsf_status gsf_plan_stage_times(gsf_plan *p, double *total_ms, int64_t *calls) {
    if (!p) return GSF_E_INVALID;
    gsf_status st = flush_timing(p);
    if (st != GSF_OK) return st;
    for (int k = 0; k < GSF_STAGE_COUNT; k++) {
        if (total_ms) total_ms[k] = p->stage_ms[k];
        if (calls) calls[k] = p->stage_calls[k];
    }
    return GSF_OK;
}

gsf_status gsf_count_pairs(gsf_plan *p, int64_t *out) {
    gsf_status st = check_ready(p);
    if (st != GSF_OK) return st;
    if (!out) return fail(p->ctx, GSF_E_INVALID, "gsf_count_pairs: null output");
    if (!p->have_forward) return fail(p->ctx, GSF_E_STATE, "gsf_count_pairs before gsf_forward");
    launch_count_pairs(p->ctx->stream, p->tile, (int)p->fwd_tiles, p->b.ranges, p->b.vals,
                       splats(p), p->b.views, p->V, p->fwd_tm, p->fwd_cull_gaze,
                       p->fwd_cull_radius, p->b.counters);
    GSF_LAUNCHED(p->ctx);
    unsigned long long c[3] = {0, 0, 0};
    GSF_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
    GSF_HIP(p->ctx, hipMemcpy(c, p->b.counters, sizeof c, hipMemcpyDeviceToHost));
    for (int k = 0; k < 3; k++) out[k] = (int64_t)c[k];
    return GSF_OK;
}

namespace {

// The last forward's ranges per global tile and its compositing order as
// global tile ids (after a fovea-culled forward: its composited tiles only).
// Compact fovea-box ranges are mapped back; a tile without keys gets [lb, lb),
// lb being its lower bound among the sorted keys.
gsf_status global_tiles(gsf_plan *p, std::vector<uint2> *ranges, std::vector<uint32_t> *order) {
    const int64_t L = p->fwd_tiles > 0 ? p->fwd_tiles : p->total_tiles;
    std::vector<uint2> lr((size_t)L);
    std::vector<uint32_t> lo((size_t)L);
    if (L) {
        GSF_HIP(p->ctx, hipMemcpy(lr.data(), p->b.ranges, (size_t)L * 8, hipMemcpyDeviceToHost));
        GSF_HIP(p->ctx, hipMemcpy(lo.data(), p->b.order, (size_t)L * 4, hipMemcpyDeviceToHost));
    }
    const TileMap tm = p->fwd_tm;
    if (!tm.gaze) {
        *ranges = std::move(lr);
        *order = std::move(lo);
        return GSF_OK;
    }
    std::vector<float> gz(2 * (size_t)p->V);
    GSF_HIP(p->ctx, hipMemcpy(gz.data(), tm.gaze, gz.size() * 4, hipMemcpyDeviceToHost));
    const int64_t area = (int64_t)tm.box * tm.box;
    std::vector<int64_t> glob((size_t)L, -1);   // global id of each launch tile (-1: none)
    for (int v = 0; v < p->V; v++) {
        const ViewDesc &vd = p->views[v];
        const FoveaTiles f = fovea_tiles(gz.data(), v, tm.radius, vd.width, vd.height, tm.tile);
        for (int64_t l = 0; l < area; l++) {
            const int ty = f.ty0 + (int)(l / tm.box), tx = f.tx0 + (int)(l % tm.box);
            if (tx <= f.tx1 && ty <= f.ty1)
                glob[(size_t)(v * area + l)] = vd.tile_off + (int64_t)ty * vd.tiles_x + tx;
        }
    }
    ranges->assign((size_t)p->total_tiles, make_uint2(0u, 0u));
    std::vector<char> has((size_t)p->total_tiles, 0);
    for (size_t c = 0; c < glob.size(); c++)
        if (glob[c] >= 0) {
            (*ranges)[(size_t)glob[c]] = lr[c];
            has[(size_t)glob[c]] = 1;
        }
    uint32_t pos = 0;
    for (size_t t = 0; t < has.size(); t++) {
        if (has[t]) pos = (*ranges)[t].y;
        else (*ranges)[t] = make_uint2(pos, pos);
    }
    order->clear();
    for (uint32_t c : lo)
        if (c < glob.size() && glob[c] >= 0) order->push_back((uint32_t)glob[c]);
    return GSF_OK;
}

}  // namespace

gsf_status gsf_debug_copy(gsf_plan *p, int which, void *host_dst, size_t cap, size_t *written) {
    gsf_status st = check_ready(p);
    if (st != GSF_OK) return st;
    if (!host_dst || !written) return fail(p->ctx, GSF_E_INVALID, "gsf_debug_copy: null argument");
    GSF_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
    const size_t R = (size_t)(p->fwd_n * p->V);
    unsigned long long mt = 0;
    uint32_t md = 0;
    GSF_HIP(p->ctx, hipMemcpy(&mt, p->b.m_total, 8, hipMemcpyDeviceToHost));
    GSF_HIP(p->ctx, hipMemcpy(&md, p->b.m_dev, 4, hipMemcpyDeviceToHost));
    const size_t M = p->host_sized ? (mt > (unsigned long long)p->cap ? 0 : (size_t)mt) : md;
    const void *src = nullptr;
    size_t bytes = 0;
    std::vector<float> proj;
    switch (which) {
    case GSF_DBG_RECT: src = p->b.rect; bytes = R * 8; break;
    case GSF_DBG_COUNT: src = p->b.count; bytes = R * 4; break;
    case GSF_DBG_DEPTH: src = p->b.depth_key; bytes = R * 4; break;
    case GSF_DBG_KEYS: {   // the tile id of every key position, from the ranges
        std::vector<uint2> rg;
        std::vector<uint32_t> od;
        st = global_tiles(p, &rg, &od);
        if (st != GSF_OK) return st;
        std::vector<uint32_t> keys(M);
        for (size_t t = 0; t < rg.size(); t++)
            for (uint32_t k = rg[t].x; k < rg[t].y && k < M; k++) keys[k] = (uint32_t)t;
        bytes = M * 4;
        if (bytes > cap) return fail(p->ctx, GSF_E_INVALID, "gsf_debug_copy: destination too small");
        if (bytes) std::memcpy(host_dst, keys.data(), bytes);
        *written = bytes;
        return GSF_OK;
    }
    case GSF_DBG_VALS: src = p->b.vals; bytes = M * 4; break;
    case GSF_DBG_RANGES:
    case GSF_DBG_ORDER: {
        std::vector<uint2> rg;
        std::vector<uint32_t> od;
        st = global_tiles(p, &rg, &od);
        if (st != GSF_OK) return st;
        const void *data = which == GSF_DBG_RANGES ? (const void *)rg.data() : (const void *)od.data();
        bytes = which == GSF_DBG_RANGES ? rg.size() * 8 : od.size() * 4;
        if (bytes > cap) return fail(p->ctx, GSF_E_INVALID, "gsf_debug_copy: destination too small");
        if (bytes) std::memcpy(host_dst, data, bytes);
        *written = bytes;
        return GSF_OK;
    }
    case GSF_DBG_BG: src = p->b.bg; bytes = p->views.size() * 3 * sizeof(float); break;
    case GSF_DBG_VIS: src = p->b.vis; bytes = (size_t)p->fwd_n; break;
    case GSF_DBG_TFINAL: src = p->b.tfinal; bytes = (size_t)p->total_pix * 4; break;
    case GSF_DBG_NCONTRIB: src = p->b.ncontrib; bytes = (size_t)p->total_pix * 4; break;
    case GSF_DBG_G2D: {   // the per-record sums of the last adjoint's per-key gradients
        RenderArgs ra = render_args(p, nullptr, p->fwd_n);
        launch_grad_sum(p->ctx->stream, ra.kp, (int)R, p->b.g2d);
        GSF_LAUNCHED(p->ctx);
        GSF_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
        src = p->b.g2d;
        bytes = 9 * R * 4;
        break;
    }
    case GSF_DBG_PROJ: {
        std::vector<float4> rec(R * kRecF4);
        std::vector<uint32_t> dk(R);
        if (R) {
            GSF_HIP(p->ctx, hipMemcpy(rec.data(), p->b.rec, R * kRecF4 * 16, hipMemcpyDeviceToHost));
            GSF_HIP(p->ctx, hipMemcpy(dk.data(), p->b.depth_key, R * 4, hipMemcpyDeviceToHost));
        }
        std::vector<float4> a(R), b(R), c(R);
        for (size_t r = 0; r < R; r++) {
            a[r] = rec[r * kRecF4 + kRecA];
            b[r] = rec[r * kRecF4 + kRecB];
            c[r] = rec[r * kRecF4 + kRecC];
        }
        proj.resize(R * 11);
        // the stored conic is pre-scaled by -log2(e)/2 (A, C) and -log2(e) (B)
        const double half = -0.5 * 1.4426950408889634, full = -1.4426950408889634;
        for (size_t r = 0; r < R; r++) {
            float *o = proj.data() + 11 * r;
            const bool valid = dk[r] != 0xFFFFFFFFu;
            float depth;
            std::memcpy(&depth, &dk[r], 4);
            // the mean is stored as an integer pixel plus the offset of the mean from its centre
            const float mx = (float)((double)c[r].z + 0.5 - (double)a[r].x);
            const float my = (float)((double)c[r].w + 0.5 - (double)a[r].y);
            const float vals[11] = {mx, my, (float)(a[r].z / half), (float)(a[r].w / full),
                                    (float)(b[r].x / half), b[r].y, b[r].z, b[r].w, c[r].x,
                                    valid ? depth : 0.f, valid ? 1.f : 0.f};
            std::memcpy(o, vals, sizeof vals);
        }
        bytes = proj.size() * 4;
        if (bytes > cap) return fail(p->ctx, GSF_E_INVALID, "gsf_debug_copy: destination too small");
        std::memcpy(host_dst, proj.data(), bytes);
        *written = bytes;
        return GSF_OK;
    }
    default: return fail(p->ctx, GSF_E_INVALID, "gsf_debug_copy: unknown buffer");
    }
    if (bytes > cap) return fail(p->ctx, GSF_E_INVALID, "gsf_debug_copy: destination too small");
    if (bytes) GSF_HIP(p->ctx, hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost));
    *written = bytes;
    return GSF_OK;
}

}  // extern "C"

// Context, workspace and the C ABI declared in include/vgr.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <map>
#include <vector>

#include "vgr_internal.h"

using namespace vgr;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

enum Stage {
    ST_PREPROCESS, ST_SORT_DEPTH, ST_SCAN_EMIT, ST_SORT_TILES, ST_RANGES, ST_RASTER_FWD,
    ST_ZERO_GRAD, ST_RASTER_BWD, ST_PREPROCESS_BWD, ST_COUNT
};
const char *kStageNames[ST_COUNT] = {
    "preprocess_fwd", "sort_depth", "scan_emit", "sort_tiles", "tile_ranges_order", "raster_fwd",
    "zero_record_grads", "raster_bwd", "preprocess_bwd"
};

// Workload class of the autotuner's cache: total pixels and Gaussians in
// powers of two, and the rules that change the rasterisers' work.
struct TuneKey {
    int32_t pix_log2, n_log2, mode, alpha_model, kernel, tile_resort, near_segment;
    bool operator<(const TuneKey &o) const
    {
        const int32_t a[7] = { pix_log2, n_log2, mode, alpha_model, kernel, tile_resort, near_segment };
        const int32_t b[7] = { o.pix_log2, o.n_log2, o.mode, o.alpha_model, o.kernel, o.tile_resort,
                               o.near_segment };
        for (int k = 0; k < 7; ++k)
            if (a[k] != b[k]) return a[k] < b[k];
        return false;
    }
};
struct TuneVal {
    int32_t tile_w, tile_h, batch;
    float ms;
};

int32_t log2_bucket(int64_t v)
{
    return v <= 1 ? 0 : (int32_t)lround(log2((double)v));
}

TuneKey tune_key(const vgr_settings *st, int64_t n, int32_t n_views, const vgr_camera *cams)
{
    int64_t pix = 0;
    for (int v = 0; v < n_views; ++v) pix += (int64_t)cams[v].width * cams[v].height;
    return TuneKey{ log2_bucket(pix), log2_bucket(n), st->mode, st->alpha_model, st->kernel,
                    st->tile_resort, st->near_segment };
}

}  // namespace

// Scratch of vgr_sort_pairs_static, one array per device (file scope, so
// every GPU the library runs on holds its own copy until the process ends):
// the ping-pong halves of keys and values and the radix tables, followed by
// the element-count word the sort kernels read.  Host code never uses the
// array's name as an address: vgr_create looks up each device's copy with
// hipGetSymbolAddress and keeps that pointer in the context.
constexpr int64_t kStaticSortMax = VGR_STATIC_SORT_MAX;
constexpr int kMaxGraphCalls = VGR_MAX_GRAPH_CALLS;
constexpr int64_t kStaticRadixWords = 256 * (kStaticSortMax / 1024) + 256;
constexpr int64_t kStaticScratchWords = 4 * kStaticSortMax + kStaticRadixWords + 64;
static __device__ __align__(256) uint32_t scratch[kStaticScratchWords];

struct vgr_ctx {
    int device = 0;
    uint32_t *static_scratch = nullptr;   // this device's copy of `scratch`
    hipStream_t stream = nullptr;
    std::string err;

    // workspace
    DevBuf geom, depth_key, item_ids, key2, item2, counts, cnt_sorted, offsets, rect;
    DevBuf inst_key, inst_val, inst_key2, inst_val2, ranges, T_final, last_pos, last_id, pmask;
    DevBuf tile_key, tile_order, tile_key2, tile_order2;
    DevBuf rgrad, scan_tmp, sort_tmp, words, counters, views, views_b, blk_counts, wg_time;
    DevBuf rs_key, rs_idx, rs_key2, rs_idx2;   // per-tile re-sorting (instance-sized)
    DevBuf wseq, wpair, wcount;                // per-pixel window (pair slots, pixels)
    ViewInfo *h_views = nullptr;      // pinned staging: [0] forward, [kMaxViews] backward
    hipEvent_t stage_ev[2] = {};      // recorded after each staging copy
    // the table last uploaded through each slot (forward: views, backward:
    // views_b); an identical table is not copied again
    std::vector<ViewInfo> uploaded[2];
    hipEvent_t k_ev = nullptr;        // recorded after the instance count copy
    bool stage_pending[2] = { false, false };
    uint32_t *h_words = nullptr;      // pinned, 8 words
    uint32_t *h_words_dev = nullptr;  // the same words as the device addresses them
    int64_t inst_capacity = 0;

    // saved forward
    bool have_fwd = false;
    RenderParams rp{};
    Buffers buf{};
    int64_t K = 0;
    int64_t total_pix = 0;
    std::vector<ViewInfo> vinfo;
    const float *means = nullptr, *quats = nullptr, *scales = nullptr, *dens = nullptr,
                *sh = nullptr;

    // densification statistics (vgr_set_densify_stats)
    float *dn_norm = nullptr;
    int32_t *dn_count = nullptr;
    int64_t dn_cap = 0;

    bool counting = false;
    bool wg_timing = false;     // time each rasteriser workgroup (load balance)
    bool wg_timed = false;      // the last forward was timed so
    bool timing = false;
    // timing: one set of events per forward / backward call since timing was
    // switched on; stage st spans events [st] .. [st + 1] of its set
    struct EvSet { hipEvent_t ev[ST_COUNT + 1]; bool used[ST_COUNT]; };
    std::vector<EvSet> evsets;
    size_t ev_next = 0;
    EvSet *cur = nullptr;
    // launch shape of calls that leave it to the library (tile_w = tile_h = 0,
    // batch = 0): the tuner's choice for the call's workload class, else the
    // last tuned shape (8x8 tiles, 64-record batches until vgr_autotune)
    int tuned_w = 8, tuned_h = 8, tuned_b = 64;
    std::map<TuneKey, TuneVal> tune_cache;

    // captured forward + backward (hipGraph)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool graph_valid = false;
    hipStream_t own_stream = nullptr;   // capture stream when the caller uses the null stream
    DevBuf views_graph;
    int64_t graph_cap = 0;
};

namespace {

int fail(vgr_ctx *c, int code, const char *fmt, ...)
{
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    if (c) c->err = msg;
    return code;
}

#define HIP_TRY(c, expr)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((c), VGR_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                              \
    } while (0)

// Grow-only device buffer; contents are not preserved.
int ensure(vgr_ctx *c, DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return VGR_OK;
    size_t want = bytes + bytes / 4;
    if (b.p) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess && c->own_stream) e = hipStreamSynchronize(c->own_stream);
        if (e != hipSuccess) return fail(c, VGR_ERR_HIP, "sync: %s", hipGetErrorString(e));
        c->graph_valid = false;   // a captured graph holds the old addresses
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        e = hipMalloc(&p, bytes);
        want = bytes;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, VGR_ERR_OOM, "hipMalloc(%zu) failed", bytes);
    }
    b.p = p;
    b.bytes = want;
    return VGR_OK;
}

template <class T>
T *ptr(DevBuf &b)
{
    return reinterpret_cast<T *>(b.p);
}

bool valid_tile(int w, int h)
{
    return (w == 8 && h == 8) || (w == 16 && h == 8) || (w == 16 && h == 16) || (w == 32 && h == 8);
}

void inverse3(const float *Rf, double *Ri)
{
    double R[9];
    for (int k = 0; k < 9; ++k) R[k] = Rf[k];
    double c0 = R[4] * R[8] - R[5] * R[7];
    double c1 = R[5] * R[6] - R[3] * R[8];
    double c2 = R[3] * R[7] - R[4] * R[6];
    double det = R[0] * c0 + R[1] * c1 + R[2] * c2;
    Ri[0] = c0 / det; Ri[1] = (R[2] * R[7] - R[1] * R[8]) / det; Ri[2] = (R[1] * R[5] - R[2] * R[4]) / det;
    Ri[3] = c1 / det; Ri[4] = (R[0] * R[8] - R[2] * R[6]) / det; Ri[5] = (R[2] * R[3] - R[0] * R[5]) / det;
    Ri[6] = c2 / det; Ri[7] = (R[1] * R[6] - R[0] * R[7]) / det; Ri[8] = (R[0] * R[4] - R[1] * R[3]) / det;
}

// Start a timed call: take the next event set (created on first use).
int timing_begin(vgr_ctx *c)
{
    c->cur = nullptr;
    if (!c->timing) return VGR_OK;
    if (c->ev_next == c->evsets.size()) {
        vgr_ctx::EvSet es{};
        for (auto &e : es.ev) HIP_TRY(c, hipEventCreate(&e));
        c->evsets.push_back(es);
    }
    c->cur = &c->evsets[c->ev_next++];
    for (bool &u : c->cur->used) u = false;
    return VGR_OK;
}

void mark(vgr_ctx *c, int st)
{
    if (!c->cur) return;
    (void)hipEventRecord(c->cur->ev[st], c->stream);
    c->cur->used[st] = true;
}

void mark_end(vgr_ctx *c, int st)
{
    if (!c->cur) return;
    (void)hipEventRecord(c->cur->ev[st + 1], c->stream);
}

int bits_for(int64_t v)
{
    int b = 1;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

// Device view table of slot 0 (forward) or 1 (backward).
ViewInfo *view_table(vgr_ctx *c, int slot)
{
    return ptr<ViewInfo>(slot == 0 ? c->views : c->views_b);
}

// Copy the view table to slot `slot`'s device table through pinned staging,
// waiting first for the previous copy out of that slot to finish; skipped
// when the table equals the one that slot holds (a loop over the same
// cameras and buffers uploads once).
int upload_views(vgr_ctx *c, int slot, const std::vector<ViewInfo> &vinfo)
{
    std::vector<ViewInfo> &last = c->uploaded[slot];
    const size_t bytes = sizeof(ViewInfo) * vinfo.size();
    if (last.size() == vinfo.size() && memcmp(last.data(), vinfo.data(), bytes) == 0)
        return VGR_OK;
    ViewInfo *h = c->h_views + slot * kMaxViews;
    if (c->stage_pending[slot]) HIP_TRY(c, hipEventSynchronize(c->stage_ev[slot]));
    memcpy(h, vinfo.data(), bytes);
    last.clear();
    HIP_TRY(c, hipMemcpyAsync(view_table(c, slot), h, bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipEventRecord(c->stage_ev[slot], c->stream));
    c->stage_pending[slot] = true;
    last = vinfo;
    return VGR_OK;
}

Buffers make_buffers(vgr_ctx *c)
{
    Buffers b{};
    b.geom = ptr<float4>(c->geom);
    b.depth_key = ptr<uint32_t>(c->depth_key);
    b.item_ids = ptr<uint32_t>(c->item_ids);
    b.key2 = ptr<uint32_t>(c->key2);
    b.item2 = ptr<uint32_t>(c->item2);
    b.counts = ptr<uint32_t>(c->counts);
    b.cnt_sorted = ptr<uint32_t>(c->cnt_sorted);
    b.offsets = ptr<uint32_t>(c->offsets);
    b.rect = ptr<ushort4>(c->rect);
    b.inst_key = ptr<uint32_t>(c->inst_key);
    b.inst_val = ptr<uint32_t>(c->inst_val);
    b.inst_key2 = ptr<uint32_t>(c->inst_key2);
    b.inst_val2 = ptr<uint32_t>(c->inst_val2);
    b.pmask = ptr<uint64_t>(c->pmask);
    b.ranges = ptr<uint2>(c->ranges);
    b.tile_key = ptr<uint32_t>(c->tile_key);
    b.tile_order = ptr<uint32_t>(c->tile_order);
    b.tile_key2 = ptr<uint32_t>(c->tile_key2);
    b.tile_order2 = ptr<uint32_t>(c->tile_order2);
    b.T_final = ptr<float>(c->T_final);
    b.last_pos = ptr<int32_t>(c->last_pos);
    b.last_id = ptr<int32_t>(c->last_id);
    b.rgrad = ptr<float4>(c->rgrad);
    b.wseq = ptr<int2>(c->wseq);
    b.wpair = ptr<float2>(c->wpair);
    b.wcount = ptr<int32_t>(c->wcount);
    b.d_total = ptr<uint32_t>(c->words);
    b.blk_counts = ptr<uint32_t>(c->blk_counts);
    b.counters = ptr<unsigned long long>(c->counters);
    b.wg_time = nullptr;   // set by a forward that times its workgroups
    b.views = ptr<ViewInfo>(c->views);
    return b;
}

int check_ptr(vgr_ctx *c, const void *p, const char *name)
{
    if (!p) return fail(c, VGR_ERR_INVALID_ARG, "%s is NULL", name);
    return VGR_OK;
}

}  // namespace

extern "C" {

void vgr_default_settings(vgr_settings *s)
{
    if (!s) return;
    memset(s, 0, sizeof *s);
    s->mode = VGR_MODE_COLOR;
    s->sh_degree = 0;
    s->alpha_min = 1.0f / 255.0f;
    s->alpha_max = 0.99f;
    s->T_min = 1e-4f;
    s->x_min_xray = 1e-6f;
    s->act = VGR_ACT_CLAMP0;
}

int vgr_create(vgr_ctx **out, int device)
{
    if (!out) return VGR_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return VGR_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return VGR_ERR_HIP;
    vgr_ctx *c = new vgr_ctx();
    c->device = device;
    int rc;
    if (hipHostMalloc((void **)&c->h_views, sizeof(ViewInfo) * 2 * kMaxViews, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->stage_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->stage_ev[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->k_ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&c->h_words, sizeof(uint32_t) * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->h_words_dev, c->h_words, 0) != hipSuccess) {
        vgr_destroy(c);
        return VGR_ERR_HIP;
    }
    if ((rc = ensure(c, c->views, sizeof(ViewInfo) * kMaxViews)) ||
        (rc = ensure(c, c->views_b, sizeof(ViewInfo) * kMaxViews)) ||
        (rc = ensure(c, c->words, sizeof(uint32_t) * 8)) ||
        (rc = ensure(c, c->counters, sizeof(unsigned long long) * 16))) {
        vgr_destroy(c);
        return rc;
    }
    // this device's copy of the static scratch (the device is current here)
    void *sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
        vgr_destroy(c);
        return VGR_ERR_HIP;
    }
    c->static_scratch = static_cast<uint32_t *>(sp);
    *out = c;
    return VGR_OK;
}

void vgr_destroy(vgr_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->own_stream) (void)hipStreamSynchronize(c->own_stream);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    DevBuf *all[] = { &c->views_graph, &c->geom, &c->depth_key, &c->item_ids, &c->key2, &c->item2,
                      &c->counts, &c->cnt_sorted, &c->offsets, &c->rect, &c->inst_key,
                      &c->inst_val, &c->inst_key2, &c->inst_val2, &c->pmask, &c->ranges, &c->T_final,
                      &c->last_pos, &c->last_id, &c->tile_key, &c->tile_order, &c->tile_key2,
                      &c->tile_order2, &c->rgrad, &c->scan_tmp, &c->sort_tmp,
                      &c->words, &c->counters, &c->views, &c->views_b, &c->blk_counts,
                      &c->wg_time,
                      &c->rs_key, &c->rs_idx, &c->rs_key2, &c->rs_idx2,
                      &c->wseq, &c->wpair, &c->wcount };
    for (DevBuf *b : all)
        if (b->p) (void)hipFree(b->p);
    if (c->h_views) (void)hipHostFree(c->h_views);
    for (auto &e : c->stage_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->k_ev) (void)hipEventDestroy(c->k_ev);
    if (c->h_words) (void)hipHostFree(c->h_words);
    for (auto &es : c->evsets)
        for (auto &e : es.ev) (void)hipEventDestroy(e);
    delete c;
}

int vgr_set_stream(vgr_ctx *c, void *stream)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    return VGR_OK;
}

const char *vgr_last_error(const vgr_ctx *c)
{
    return c ? c->err.c_str() : "null context";
}

int vgr_set_counting(vgr_ctx *c, int enable)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    c->counting = (enable & 1) != 0;
    c->wg_timing = (enable & 2) != 0;
    return VGR_OK;
}

int vgr_set_densify_stats(vgr_ctx *c, float *grad_norm_sum, int32_t *view_count,
                          int64_t capacity)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    c->err.clear();
    if (capacity < 0) return fail(c, VGR_ERR_INVALID_ARG, "negative capacity");
    c->dn_norm = grad_norm_sum;
    c->dn_count = view_count;
    c->dn_cap = (grad_norm_sum || view_count) ? capacity : 0;
    return VGR_OK;
}

int vgr_set_timing(vgr_ctx *c, int enable)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->timing = enable != 0;
    c->ev_next = 0;
    c->cur = nullptr;
    return VGR_OK;
}

int vgr_get_timing(vgr_ctx *c, int32_t cap, const char **names, float *ms, int32_t *count)
{
    if (!c || !count) return VGR_ERR_INVALID_ARG;
    *count = 0;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int n = 0;
    for (int st = 0; st < ST_COUNT && n < cap; ++st) {
        double tot = 0.0;
        int calls = 0;
        for (size_t k = 0; k < c->ev_next; ++k) {
            const vgr_ctx::EvSet &es = c->evsets[k];
            if (!es.used[st]) continue;
            float t = 0.f;
            if (hipEventElapsedTime(&t, es.ev[st], es.ev[st + 1]) != hipSuccess) {
                (void)hipGetLastError();
                continue;
            }
            tot += t;
            ++calls;
        }
        if (!calls) continue;
        if (names) names[n] = kStageNames[st];
        if (ms) ms[n] = (float)(tot / calls);
        ++n;
    }
    *count = n;
    return VGR_OK;
}

}  // extern "C"

namespace {

// Validated call: render rules, per-view tables and workspace sizes.
struct Prepared {
    RenderParams rp{};
    std::vector<ViewInfo> vinfo;
    int64_t m = 0, tiles = 0, pix = 0, sort_n = 0;
};

int prepare(vgr_ctx *c, const vgr_settings *st, int64_t n, const float *means,
            const float *quats, const float *scales, const float *dens, const float *sh,
            int32_t n_views, const vgr_camera *cams, float *const *out, Prepared &p)
{
    if (!st) return fail(c, VGR_ERR_INVALID_ARG, "settings is NULL");
    if (n < 0 || n > (int64_t)0x7FFFFFFF) return fail(c, VGR_ERR_INVALID_ARG, "bad n %lld", (long long)n);
    if (n_views < 1 || n_views > kMaxViews)
        return fail(c, VGR_ERR_INVALID_ARG, "n_views must be in [1, %d]", kMaxViews);
    if ((int64_t)n * n_views >= (int64_t)0xFFFFFFFF)
        return fail(c, VGR_ERR_INVALID_ARG, "n * n_views too large");
    if (st->mode != VGR_MODE_COLOR && st->mode != VGR_MODE_XRAY)
        return fail(c, VGR_ERR_INVALID_ARG, "bad mode");
    if (st->mode == VGR_MODE_COLOR && (st->sh_degree < 0 || st->sh_degree > 3))
        return fail(c, VGR_ERR_INVALID_ARG, "sh_degree must be 0..3");
    if (st->act != VGR_ACT_CLAMP0 && st->act != VGR_ACT_SOFTPLUS10)
        return fail(c, VGR_ERR_INVALID_ARG, "bad act");
    if (st->density != VGR_DENSITY_KAPPA && st->density != VGR_DENSITY_THETA)
        return fail(c, VGR_ERR_INVALID_ARG, "bad density");
    if (st->alpha_model != VGR_ALPHA_VOLUMETRIC && st->alpha_model != VGR_ALPHA_SPLAT)
        return fail(c, VGR_ERR_INVALID_ARG, "bad alpha_model");
    if (st->alpha_model == VGR_ALPHA_SPLAT &&
        (st->mode != VGR_MODE_COLOR || st->density != VGR_DENSITY_KAPPA))
        return fail(c, VGR_ERR_INVALID_ARG,
                    "the splatting model needs colour mode and the plain density input");
    if (st->near_segment != 0 && st->near_segment != 1)
        return fail(c, VGR_ERR_INVALID_ARG, "bad near_segment");
    if (st->near_segment && st->alpha_model == VGR_ALPHA_SPLAT)
        return fail(c, VGR_ERR_INVALID_ARG, "the near-plane segment needs the volumetric model");
    if (st->tile_resort != 0 && st->tile_resort != 1)
        return fail(c, VGR_ERR_INVALID_ARG, "bad tile_resort");
    if (st->tile_resort && (st->mode != VGR_MODE_COLOR || st->alpha_model != VGR_ALPHA_VOLUMETRIC))
        return fail(c, VGR_ERR_INVALID_ARG, "tile_resort needs colour mode and the volumetric model");
    if (st->kernel != VGR_KERNEL_GAUSSIAN && st->kernel != VGR_KERNEL_EPANECHNIKOV)
        return fail(c, VGR_ERR_INVALID_ARG, "bad kernel");
    if (st->kernel == VGR_KERNEL_EPANECHNIKOV &&
        (st->alpha_model != VGR_ALPHA_VOLUMETRIC || st->near_segment))
        return fail(c, VGR_ERR_INVALID_ARG,
                    "the Epanechnikov kernel needs the volumetric model without the near-plane segment");
    if (!(st->alpha_min > 0.f && st->alpha_min < 1.f) || !(st->alpha_max > st->alpha_min) ||
        !(st->alpha_max < 1.f) || !(st->T_min >= 0.f) || !(st->x_min_xray > 0.f))
        return fail(c, VGR_ERR_INVALID_ARG, "bad thresholds");
    if (!cams || !out) return fail(c, VGR_ERR_INVALID_ARG, "cams/out is NULL");
    int rc;
    if (n > 0) {
        if ((rc = check_ptr(c, means, "means")) || (rc = check_ptr(c, quats, "quats")) ||
            (rc = check_ptr(c, scales, "scales")) || (rc = check_ptr(c, dens, "dens")))
            return rc;
        if (st->mode == VGR_MODE_COLOR && (rc = check_ptr(c, sh, "sh"))) return rc;
    }
    if (st->batch != 0 && st->batch != 32 && st->batch != 64)
        return fail(c, VGR_ERR_INVALID_ARG, "batch must be 0, 32 or 64");
    if (st->pixel_window < 0 || st->pixel_window > VGR_MAX_PIXEL_WINDOW)
        return fail(c, VGR_ERR_INVALID_ARG, "pixel_window must be in [0, %d]", VGR_MAX_PIXEL_WINDOW);
    int tw = st->tile_w, th = st->tile_h, tb = st->batch;
    if (st->pixel_window > 0) {
        // one pixel per lane and the 64-record batch layout of the pair slots
        if (!st->tile_resort)
            return fail(c, VGR_ERR_INVALID_ARG, "pixel_window needs tile_resort");
        if (!((tw == 0 && th == 0) || (tw == 8 && th == 8)) || !(tb == 0 || tb == 64))
            return fail(c, VGR_ERR_INVALID_ARG, "pixel_window needs 8x8 tiles and 64-record batches");
        tw = th = 8;
        tb = 64;
    }
    if ((tw == 0 && th == 0) || tb == 0) {
        const auto it = c->tune_cache.find(tune_key(st, n, n_views, cams));
        const bool hit = it != c->tune_cache.end();
        if (tw == 0 && th == 0) {
            tw = hit ? it->second.tile_w : c->tuned_w;
            th = hit ? it->second.tile_h : c->tuned_h;
        }
        if (tb == 0) tb = hit ? it->second.batch : c->tuned_b;
    }
    if (!valid_tile(tw, th)) return fail(c, VGR_ERR_INVALID_ARG, "unsupported tile %dx%d", tw, th);

    RenderParams &rp = p.rp;
    rp.mode = st->mode;
    rp.sh_degree = st->mode == VGR_MODE_COLOR ? st->sh_degree : 0;
    rp.act = st->act;
    rp.density = st->density;
    rp.alpha_model = st->alpha_model;
    rp.amin = st->alpha_min;
    rp.amax = st->alpha_max;
    rp.near_segment = st->near_segment;
    rp.tile_resort = st->tile_resort;
    rp.kernel = st->kernel;
    rp.n_views = n_views;
    rp.n = n;
    rp.tau = st->mode == VGR_MODE_COLOR ? (float)(-log1p(-(double)st->alpha_min)) : st->x_min_xray;
    rp.tau2 = (float)((double)rp.tau * 1.4426950408889634);
    rp.ymax = (float)(-log2(1.0 - (double)st->alpha_max));
    rp.T_min = st->T_min;
    for (int k = 0; k < 3; ++k) rp.bg[k] = st->bg[k];
    rp.tile_w = tw;
    rp.tile_h = th;
    rp.batch = tb;
    rp.pixel_window = st->pixel_window;

    p.vinfo.assign(n_views, ViewInfo{});
    int64_t tiles = 0, pix = 0;
    for (int v = 0; v < n_views; ++v) {
        const vgr_camera &cm = cams[v];
        if (cm.width <= 0 || cm.height <= 0 || cm.width > 16384 || cm.height > 16384)
            return fail(c, VGR_ERR_INVALID_ARG, "view %d: bad size %dx%d", v, cm.width, cm.height);
        if (!(cm.fx > 0.f) || !(cm.fy > 0.f))
            return fail(c, VGR_ERR_INVALID_ARG, "view %d: bad focal length", v);
        if (!out[v]) return fail(c, VGR_ERR_INVALID_ARG, "out[%d] is NULL", v);
        ViewInfo &vi = p.vinfo[v];
        memcpy(vi.R, cm.R, sizeof vi.R);
        memcpy(vi.t, cm.t, sizeof vi.t);
        vi.fx = cm.fx; vi.fy = cm.fy; vi.cx = cm.cx; vi.cy = cm.cy;
        vi.znear = cm.znear;
        double Ri[9];
        inverse3(cm.R, Ri);
        for (int a = 0; a < 3; ++a)
            vi.o[a] = (float)-(Ri[a * 3] * cm.t[0] + Ri[a * 3 + 1] * cm.t[1] + Ri[a * 3 + 2] * cm.t[2]);
        vi.width = cm.width;
        vi.height = cm.height;
        vi.tiles_x = (cm.width + tw - 1) / tw;
        vi.tiles_y = (cm.height + th - 1) / th;
        vi.tile_off = (int32_t)tiles;
        vi.pix_off = pix;
        vi.out = out[v];
        vi.dL = nullptr;
        tiles += (int64_t)vi.tiles_x * vi.tiles_y;
        pix += (int64_t)cm.width * cm.height;
    }
    if (tiles >= (int64_t)1 << 30) return fail(c, VGR_ERR_INVALID_ARG, "too many tiles");
    rp.total_tiles = (int32_t)tiles;
    p.m = n * n_views;
    p.tiles = tiles;
    p.pix = pix;
    p.sort_n = p.m > tiles ? p.m : tiles;
    const int64_t m = p.m;
    if ((rc = ensure(c, c->geom, sizeof(float4) * kRecVec * (m > 0 ? m : 1))) ||
        (rc = ensure(c, c->blk_counts, 4 * (preprocess_blocks(n, n_views) + 1))) ||
        (rc = ensure(c, c->depth_key, 4 * m)) || (rc = ensure(c, c->item_ids, 4 * m)) ||
        (rc = ensure(c, c->key2, 4 * m)) || (rc = ensure(c, c->item2, 4 * m)) ||
        (rc = ensure(c, c->counts, 4 * m)) || (rc = ensure(c, c->cnt_sorted, 4 * m)) ||
        (rc = ensure(c, c->offsets, 4 * (m + 1))) || (rc = ensure(c, c->rect, 8 * m)) ||
        (rc = ensure(c, c->ranges, 8 * tiles)) || (rc = ensure(c, c->T_final, 4 * pix)) ||
        (rc = ensure(c, c->tile_key, 4 * (tiles > 64 ? tiles : 64))) ||
        (rc = ensure(c, c->tile_order, 4 * tiles)) ||
        (rc = ensure(c, c->tile_key2, 4 * tiles)) || (rc = ensure(c, c->tile_order2, 4 * tiles)) ||
        (rc = ensure(c, c->last_pos, 4 * pix)) || (rc = ensure(c, c->last_id, 4 * pix)) ||
        (rc = ensure(c, c->scan_tmp, 4 * scan_tmp_words(m > 0 ? m : 1))) ||
        (rc = ensure(c, c->sort_tmp, 4 * radix_tmp_words(p.sort_n > 0 ? p.sort_n : 1))) ||
        (rc = ensure(c, c->inst_key, 4)) || (rc = ensure(c, c->inst_val, 4)) ||
        (rc = ensure(c, c->inst_key2, 4)) || (rc = ensure(c, c->inst_val2, 4)))
        return rc;
    return VGR_OK;
}

// Enqueue the forward on stream s.  cap < 0 (eager): wait on an event for the
// instance count and size the lists exactly.  cap >= 0 (graph capture): the
// lists have `cap` entries, nothing waits, overflow is flagged on the device.
int enqueue_forward(vgr_ctx *c, const Prepared &p, const float *means, const float *quats,
                    const float *scales, const float *dens, const float *sh,
                    const ViewInfo *views_dev, int64_t cap, hipStream_t s, Buffers &out_b,
                    int64_t &out_K)
{
    const RenderParams &rp = p.rp;
    const int64_t m = p.m;
    int rc;
    Buffers b = make_buffers(c);
    b.views = views_dev;
    int64_t K = 0;
    if (m > 0) {
        mark(c, ST_PREPROCESS);
        // eager: the totals kernel also stores the instance count K and the
        // number of items with instances in the pinned words, which the host
        // reads (after k_ev) while the depth sort runs
        b.h_total = cap < 0 ? c->h_words_dev : nullptr;
        HIP_TRY(c, launch_preprocess(rp, b, means, quats, scales, dens, sh, s));
        b.h_total = nullptr;
        if (cap < 0) HIP_TRY(c, hipEventRecord(c->k_ev, s));
        mark_end(c, ST_PREPROCESS);
        // depth order of the (view, Gaussian) items that have instances (about
        // half of them in a wide scene: the others are culled or out of view);
        // ties keep the item order
        mark(c, ST_SORT_DEPTH);
        // (their number, d_total[6], comes from the preprocess's totals kernel)
        HIP_TRY(c, launch_compact_items(rp, b, s));
        HIP_TRY(c, launch_radix_sort(b.depth_key, b.item_ids, b.key2, b.item2, b.d_total + 6, m, 32,
                                     ptr<uint32_t>(c->sort_tmp), s));
        mark_end(c, ST_SORT_DEPTH);
        mark(c, ST_SCAN_EMIT);
        // eager: the items with instances come first in depth order, and their
        // number mv (with K) is on the host by now, so the scan and the
        // emission cover only them; a capture covers all m items
        int64_t mv = m;
        if (cap < 0) {
            HIP_TRY(c, hipEventSynchronize(c->k_ev));
            mv = c->h_words[2] < (uint64_t)m ? (int64_t)c->h_words[2] : m;
            K = c->h_words[0];
            if ((rc = ensure(c, c->inst_key, 4 * K)) || (rc = ensure(c, c->inst_val, 4 * K)) ||
                (rc = ensure(c, c->inst_key2, 4 * K)) || (rc = ensure(c, c->inst_val2, 4 * K)) ||
                (rc = ensure(c, c->sort_tmp, 4 * radix_tmp_words(K > p.sort_n ? K : p.sort_n))))
                return rc;
            if (rp.tile_resort &&
                ((rc = ensure(c, c->rs_key, 4 * K)) || (rc = ensure(c, c->rs_idx, 4 * K)) ||
                 (rc = ensure(c, c->rs_key2, 4 * K)) || (rc = ensure(c, c->rs_idx2, 4 * K))))
                return rc;
            c->inst_capacity = (int64_t)(c->inst_key.bytes / 4);
            b = make_buffers(c);
            b.views = views_dev;
        } else {
            K = cap;
        }
        // per-item counts in depth order with their block sums, then their
        // scan, whose total is the instance count (clamped to the capacity K)
        HIP_TRY(c, launch_gather_counts(b, mv, rp.total_tiles, ptr<uint32_t>(c->scan_tmp), s));
        HIP_TRY(c, launch_count_scan(b.cnt_sorted, b.offsets, mv, ptr<uint32_t>(c->scan_tmp),
                                     b.d_total, K, s));
        HIP_TRY(c, launch_emit(rp, b, mv, K, s));
        mark_end(c, ST_SCAN_EMIT);
        mark(c, ST_SORT_TILES);
        if (rp.tile_resort) {
            // order the instances by the depth of each maximum on its tile-centre
            // ray; the stable tile sort below keeps that order within each tile
            uint32_t *k1 = ptr<uint32_t>(c->rs_key), *i1 = ptr<uint32_t>(c->rs_idx);
            uint32_t *k2 = ptr<uint32_t>(c->rs_key2), *i2 = ptr<uint32_t>(c->rs_idx2);
            HIP_TRY(c, launch_resort_keys(rp, b, k1, i1, K, s));
            HIP_TRY(c, launch_radix_sort(k1, i1, k2, i2, b.d_total, K, 32,
                                         ptr<uint32_t>(c->sort_tmp), s));
            HIP_TRY(c, launch_resort_permute(b, i1, k2, i2, K, s));
        }
        HIP_TRY(c, launch_radix_sort(b.inst_key, b.inst_val, b.inst_key2, b.inst_val2, b.d_total, K,
                                     bits_for(p.tiles), ptr<uint32_t>(c->sort_tmp), s));
        mark_end(c, ST_SORT_TILES);
    } else {
        HIP_TRY(c, launch_fill_u32(b.d_total, 0u, 2, s));
    }
    mark(c, ST_RANGES);
    // with items, the count gather cleared the ranges and the tile-order counters
    HIP_TRY(c, launch_ranges(b, K, rp.total_tiles, m == 0, s));
    HIP_TRY(c, launch_tile_order(b, rp.total_tiles, m == 0, s));
    mark_end(c, ST_RANGES);
    if (cap < 0 && raster_keeps_masks(rp.mode, rp.tile_w, rp.tile_h)) {
        // (a capture sizes this buffer for its capacity before it starts)
        if ((rc = ensure(c, c->pmask,
                         8 * (size_t)pmask_words(K, rp.total_tiles, rp.tile_w, rp.tile_h, rp.batch))))
            return rc;
        b.pmask = ptr<uint64_t>(c->pmask);
    }
    if (rp.pixel_window > 0) {
        // (a capture sizes these buffers before it starts)
        if (cap < 0 && ((rc = ensure(c, c->wcount, 4 * (size_t)(p.pix > 0 ? p.pix : 1))) ||
                        (rc = ensure(c, c->wseq, 8 * 64 * (size_t)K)) ||
                        (rc = ensure(c, c->wpair, 8 * 64 * (size_t)K))))
            return rc;
        b.wseq = ptr<int2>(c->wseq);
        b.wpair = ptr<float2>(c->wpair);
        b.wcount = ptr<int32_t>(c->wcount);
    }
    if (c->counting)
        HIP_TRY(c, launch_fill_u32(reinterpret_cast<uint32_t *>(b.counters), 0u, 16, s));
    b.wg_time = nullptr;
    c->wg_timed = false;
    if (c->wg_timing && cap < 0) {
        if ((rc = ensure(c, c->wg_time, 16 * (size_t)(rp.total_tiles > 0 ? rp.total_tiles : 1))))
            return rc;
        b.wg_time = ptr<uint2>(c->wg_time);
        HIP_TRY(c, launch_fill_u32(reinterpret_cast<uint32_t *>(b.wg_time), 0u,
                                   4 * (int64_t)rp.total_tiles, s));
        c->wg_timed = true;
    }
    mark(c, ST_RASTER_FWD);
    HIP_TRY(c, launch_raster_fwd(rp, b, c->counting, s));
    mark_end(c, ST_RASTER_FWD);
    out_b = b;
    out_K = K;
    return VGR_OK;
}

int enqueue_backward(vgr_ctx *c, const RenderParams &rp, const Buffers &b_fwd,
                     const ViewInfo *views_dev, const float *means, const float *quats,
                     const float *scales, const float *dens, const float *sh, float *d_means,
                     float *d_quats, float *d_scales, float *d_dens, float *d_sh, bool accumulate,
                     hipStream_t s)
{
    const int64_t m = rp.n * rp.n_views;
    if (m == 0) return VGR_OK;
    Buffers b = b_fwd;
    b.rgrad = ptr<float4>(c->rgrad);
    b.views = views_dev;
    mark(c, ST_ZERO_GRAD);
    HIP_TRY(c, launch_fill_f32(reinterpret_cast<float *>(b.rgrad), 0.0f, 16 * m, s));
    mark_end(c, ST_ZERO_GRAD);
    mark(c, ST_RASTER_BWD);
    if (c->counting)
        HIP_TRY(c, launch_fill_u32(reinterpret_cast<uint32_t *>(b.counters) + 16, 0u, 16, s));
    HIP_TRY(c, launch_raster_bwd(rp, b, c->counting, s));
    mark_end(c, ST_RASTER_BWD);
    mark(c, ST_PREPROCESS_BWD);
    HIP_TRY(c, launch_preprocess_bwd(rp, b, means, quats, scales, dens, sh, d_means, d_quats,
                                     d_scales, d_dens, d_sh, accumulate, c->dn_norm,
                                     c->dn_count, s));
    mark_end(c, ST_PREPROCESS_BWD);
    return VGR_OK;
}

int check_grads(vgr_ctx *c, const RenderParams &rp, float *d_means, float *d_quats,
                float *d_scales, float *d_dens, float *d_sh)
{
    int rc;
    if (rp.n > 0) {
        if ((rc = check_ptr(c, d_means, "d_means")) || (rc = check_ptr(c, d_quats, "d_quats")) ||
            (rc = check_ptr(c, d_scales, "d_scales")) || (rc = check_ptr(c, d_dens, "d_dens")))
            return rc;
        if (rp.mode == VGR_MODE_COLOR && (rc = check_ptr(c, d_sh, "d_sh"))) return rc;
    }
    if ((c->dn_norm || c->dn_count) && rp.n > c->dn_cap)
        return fail(c, VGR_ERR_INVALID_ARG, "n = %lld exceeds the densification arrays (%lld)",
                    (long long)rp.n, (long long)c->dn_cap);
    return VGR_OK;
}

}  // namespace

extern "C" {

int vgr_render_forward(vgr_ctx *c, const vgr_settings *st, int64_t n, const float *means,
                       const float *quats, const float *scales, const float *dens,
                       const float *sh, int32_t n_views, const vgr_camera *cams,
                       float *const *out)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    c->err.clear();
    c->have_fwd = false;
    HIP_TRY(c, hipSetDevice(c->device));
    Prepared p;
    int rc;
    if ((rc = prepare(c, st, n, means, quats, scales, dens, sh, n_views, cams, out, p))) return rc;
    if ((rc = upload_views(c, 0, p.vinfo))) return rc;
    if ((rc = timing_begin(c))) return rc;
    Buffers b;
    int64_t K;
    if ((rc = enqueue_forward(c, p, means, quats, scales, dens, sh, view_table(c, 0), -1,
                              c->stream, b, K)))
        return rc;
    c->rp = p.rp;
    c->buf = b;
    c->K = K;
    c->total_pix = p.pix;
    c->vinfo = p.vinfo;
    c->means = means; c->quats = quats; c->scales = scales; c->dens = dens; c->sh = sh;
    c->have_fwd = true;
    return VGR_OK;
}

int vgr_render_backward(vgr_ctx *c, const float *const *dL, float *d_means, float *d_quats,
                        float *d_scales, float *d_dens, float *d_sh, int32_t accumulate)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    c->err.clear();
    if (!c->have_fwd) return fail(c, VGR_ERR_NO_FORWARD, "no forward to differentiate");
    if (!dL) return fail(c, VGR_ERR_INVALID_ARG, "dL_dout is NULL");
    const RenderParams &rp = c->rp;
    int rc;
    if ((rc = check_grads(c, rp, d_means, d_quats, d_scales, d_dens, d_sh))) return rc;
    for (int v = 0; v < rp.n_views; ++v) {
        if (!dL[v]) return fail(c, VGR_ERR_INVALID_ARG, "dL_dout[%d] is NULL", v);
        c->vinfo[v].dL = dL[v];
    }
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t m = rp.n * rp.n_views;
    if ((rc = ensure(c, c->rgrad, sizeof(float4) * 4 * (m > 0 ? m : 1)))) return rc;
    if ((rc = upload_views(c, 1, c->vinfo))) return rc;
    if ((rc = timing_begin(c))) return rc;
    return enqueue_backward(c, rp, c->buf, view_table(c, 1), c->means, c->quats, c->scales,
                            c->dens, c->sh, d_means, d_quats, d_scales, d_dens, d_sh,
                            accumulate != 0, c->stream);
}

int vgr_get_aux(vgr_ctx *c, int32_t view, float *T_final, int32_t *last_index)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    if (!c->have_fwd) return fail(c, VGR_ERR_NO_FORWARD, "no forward");
    if (view < 0 || view >= c->rp.n_views) return fail(c, VGR_ERR_INVALID_ARG, "bad view");
    const ViewInfo &vi = c->vinfo[view];
    const size_t np = (size_t)vi.width * vi.height;
    if (T_final)
        HIP_TRY(c, hipMemcpyAsync(T_final, ptr<float>(c->T_final) + vi.pix_off, 4 * np,
                                  hipMemcpyDeviceToDevice, c->stream));
    if (last_index)
        HIP_TRY(c, hipMemcpyAsync(last_index, ptr<int32_t>(c->last_id) + vi.pix_off, 4 * np,
                                  hipMemcpyDeviceToDevice, c->stream));
    return VGR_OK;
}

int vgr_get_stats(vgr_ctx *c, vgr_stats *out)
{
    if (!c || !out) return VGR_ERR_INVALID_ARG;
    memset(out, 0, sizeof *out);
    if (!c->have_fwd) return fail(c, VGR_ERR_NO_FORWARD, "no forward");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    uint32_t words[8];
    HIP_TRY(c, hipMemcpy(words, c->words.p, sizeof words, hipMemcpyDeviceToHost));
    unsigned long long cnt[16] = {};
    if (c->counting) HIP_TRY(c, hipMemcpy(cnt, c->counters.p, sizeof cnt, hipMemcpyDeviceToHost));
    out->instances = words[0];
    out->overflow = (int32_t)words[1];
    out->emit_mismatch = c->rp.n > 0 && c->rp.n_views > 0 ? (int32_t)words[7] : 0;
    out->capacity = c->inst_capacity;
    out->pairs_tested = (int64_t)cnt[0];
    out->pairs_full = (int64_t)cnt[1];
    out->pairs_blended = (int64_t)cnt[2];
    out->visits = (int64_t)cnt[3];
    out->visits_full = (int64_t)cnt[4];
    out->bwd_pairs_tested = (int64_t)cnt[8];
    out->bwd_pairs_full = (int64_t)cnt[9];
    out->bwd_pairs_blended = (int64_t)cnt[10];
    out->bwd_visits = (int64_t)cnt[11];
    out->bwd_visits_full = (int64_t)cnt[12];
    out->tile_w = c->rp.tile_w;
    out->tile_h = c->rp.tile_h;
    out->n_views = c->rp.n_views;
    // load balance of the rasterisers: per compute unit, the summed durations
    // of its workgroups; max over mean
    const int32_t T = c->rp.total_tiles;
    if (c->wg_timed && T > 0 && c->wg_time.bytes >= 16 * (size_t)T) {
        std::vector<uint32_t> wt(4 * (size_t)T);
        HIP_TRY(c, hipMemcpy(wt.data(), c->wg_time.p, 16 * (size_t)T, hipMemcpyDeviceToHost));
        for (int dir = 0; dir < 2; ++dir) {
            std::map<uint32_t, double> busy;
            for (int32_t k = 0; k < T; ++k) {
                const uint32_t key = wt[2 * ((size_t)dir * T + k)];
                const uint32_t dur = wt[2 * ((size_t)dir * T + k) + 1];
                if (dur) busy[key] += dur;
            }
            double mx = 0.0, sum = 0.0;
            for (const auto &kv : busy) {
                mx = kv.second > mx ? kv.second : mx;
                sum += kv.second;
            }
            const double lb = busy.empty() || sum <= 0.0 ? 0.0 : mx / (sum / busy.size());
            (dir == 0 ? out->load_balance_fwd : out->load_balance_bwd) = lb;
        }
    }
    // visible (Gaussian, view) items = items with a nonzero tile count
    const int64_t m = c->rp.n * c->rp.n_views;
    if (m > 0) {
        std::vector<uint32_t> counts(m);
        HIP_TRY(c, hipMemcpy(counts.data(), c->counts.p, 4 * m, hipMemcpyDeviceToHost));
        int64_t vis = 0;
        for (uint32_t x : counts) vis += x > 0;
        out->visible = vis;
    }
    return VGR_OK;
}

int vgr_sort_pairs(vgr_ctx *c, uint32_t *keys, uint32_t *vals, int64_t n, int32_t bits)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    c->err.clear();
    if (n < 0 || n > (int64_t)0xFFFFFFF || bits < 1 || bits > 32)
        return fail(c, VGR_ERR_INVALID_ARG, "bad n or bits");
    if (n == 0) return VGR_OK;
    if (!keys || !vals) return fail(c, VGR_ERR_INVALID_ARG, "keys/vals NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc;
    if ((rc = ensure(c, c->sort_tmp, 4 * radix_tmp_words(n)))) return rc;
    // the ping-pong halves live in the instance buffers (not part of any saved forward)
    if ((rc = ensure(c, c->inst_key2, 4 * n)) || (rc = ensure(c, c->inst_val2, 4 * n))) return rc;
    c->have_fwd = false;
    hipStream_t s = c->stream;
    uint32_t *dn = ptr<uint32_t>(c->words) + 2;
    HIP_TRY(c, launch_fill_u32(dn, (uint32_t)n, 1, s));
    HIP_TRY(c, launch_radix_sort(keys, vals, ptr<uint32_t>(c->inst_key2), ptr<uint32_t>(c->inst_val2),
                                 dn, n, bits, ptr<uint32_t>(c->sort_tmp), s));
    return VGR_OK;
}

int vgr_sort_pairs_static(vgr_ctx *c, uint32_t *keys, uint32_t *vals, int64_t n, int32_t bits)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    c->err.clear();
    if (n < 0 || bits < 1 || bits > 32) return fail(c, VGR_ERR_INVALID_ARG, "bad n or bits");
    if (n > kStaticSortMax)
        return fail(c, VGR_ERR_INVALID_ARG, "n = %lld exceeds the static scratch (%lld pairs)",
                    (long long)n, (long long)kStaticSortMax);
    if (n == 0) return VGR_OK;
    if (!keys || !vals) return fail(c, VGR_ERR_INVALID_ARG, "keys/vals NULL");
    if (!c->static_scratch) return fail(c, VGR_ERR_HIP, "no static scratch on this device");
    if (radix_tmp_words(n) > kStaticRadixWords)
        return fail(c, VGR_ERR_INVALID_ARG, "radix tables exceed the static scratch");
    HIP_TRY(c, hipSetDevice(c->device));
    // layout: keys2 | vals2 | radix tables | count word (all overwritten by
    // every call before they are read: nothing needs clearing)
    uint32_t *k2 = c->static_scratch;
    uint32_t *v2 = k2 + kStaticSortMax;
    uint32_t *tmp = v2 + kStaticSortMax;
    uint32_t *dn = tmp + kStaticRadixWords;
    hipStream_t s = c->stream;
    HIP_TRY(c, launch_fill_u32(dn, (uint32_t)n, 1, s));
    HIP_TRY(c, launch_radix_sort(keys, vals, k2, v2, dn, n, bits, tmp, s));
    return VGR_OK;
}

int vgr_graph_capture_calls(vgr_ctx *c, const vgr_settings *st, int64_t n, const float *means,
                            const float *quats, const float *scales, const float *dens,
                            const float *sh, int32_t n_calls, const int32_t *views_per_call,
                            const vgr_camera *cams, float *const *out, const float *const *dL,
                            float *d_means, float *d_quats, float *d_scales, float *d_dens,
                            float *d_sh, float capacity_factor, int32_t zero_grads)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    c->err.clear();
    if (!dL) return fail(c, VGR_ERR_INVALID_ARG, "dL_dout is NULL");
    if (n_calls < 1 || n_calls > kMaxGraphCalls || !views_per_call)
        return fail(c, VGR_ERR_INVALID_ARG, "n_calls must be in [1, %d]", kMaxGraphCalls);
    std::vector<int32_t> off(n_calls + 1, 0);
    for (int k = 0; k < n_calls; ++k) {
        if (views_per_call[k] < 1 || views_per_call[k] > kMaxViews)
            return fail(c, VGR_ERR_INVALID_ARG, "call %d: views must be in [1, %d]", k, kMaxViews);
        off[k + 1] = off[k] + views_per_call[k];
    }
    if (!(capacity_factor >= 1.0f)) capacity_factor = 1.25f;
    int rc = VGR_OK;
    // one eager pass per call sizes every buffer and measures the instance counts
    const bool counting = c->counting, timing = c->timing;
    c->counting = false;
    c->timing = false;
    c->cur = nullptr;
    int64_t kmax = 0;
    for (int k = 0; k < n_calls && !rc; ++k) {
        rc = vgr_render_forward(c, st, n, means, quats, scales, dens, sh, views_per_call[k],
                                cams + off[k], out + off[k]);
        if (!rc)
            rc = vgr_render_backward(c, dL + off[k], d_means, d_quats, d_scales, d_dens, d_sh,
                                     (zero_grads && k == 0) ? 0 : 1);
        if (!rc) kmax = c->K > kmax ? c->K : kmax;
    }
    c->counting = counting;
    c->timing = timing;
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::vector<Prepared> ps(n_calls);
    for (int k = 0; k < n_calls; ++k)
        if ((rc = prepare(c, st, n, means, quats, scales, dens, sh, views_per_call[k],
                          cams + off[k], out + off[k], ps[k])))
            return rc;
    const int64_t cap = (int64_t)ceil((double)kmax * capacity_factor) + 4096;
    int64_t mmax = 0, sort_n = 0, pmw = 0;
    for (const Prepared &p : ps) {
        mmax = p.m > mmax ? p.m : mmax;
        sort_n = p.sort_n > sort_n ? p.sort_n : sort_n;
        if (raster_keeps_masks(p.rp.mode, p.rp.tile_w, p.rp.tile_h)) {
            const int64_t w = pmask_words(cap, p.rp.total_tiles, p.rp.tile_w, p.rp.tile_h, p.rp.batch);
            pmw = w > pmw ? w : pmw;
        }
    }
    if (ps[0].rp.tile_resort &&
        ((rc = ensure(c, c->rs_key, 4 * cap)) || (rc = ensure(c, c->rs_idx, 4 * cap)) ||
         (rc = ensure(c, c->rs_key2, 4 * cap)) || (rc = ensure(c, c->rs_idx2, 4 * cap))))
        return rc;
    if ((rc = ensure(c, c->inst_key, 4 * cap)) || (rc = ensure(c, c->inst_val, 4 * cap)) ||
        (rc = ensure(c, c->inst_key2, 4 * cap)) || (rc = ensure(c, c->inst_val2, 4 * cap)) ||
        (rc = ensure(c, c->sort_tmp, 4 * radix_tmp_words(cap > sort_n ? cap : sort_n))) ||
        (rc = ensure(c, c->rgrad, sizeof(float4) * 4 * (mmax > 0 ? mmax : 1))) ||
        (rc = ensure(c, c->views_graph, sizeof(ViewInfo) * (size_t)off[n_calls])))
        return rc;
    if (pmw > 0 && (rc = ensure(c, c->pmask, 8 * (size_t)pmw))) return rc;
    int64_t pixmax = 1;
    for (const Prepared &p : ps) pixmax = p.pix > pixmax ? p.pix : pixmax;
    if (ps[0].rp.pixel_window > 0 &&
        ((rc = ensure(c, c->wcount, 4 * (size_t)pixmax)) ||
         (rc = ensure(c, c->wseq, 8 * 64 * (size_t)cap)) ||
         (rc = ensure(c, c->wpair, 8 * 64 * (size_t)cap))))
        return rc;
    c->inst_capacity = (int64_t)(c->inst_key.bytes / 4);
    for (int k = 0; k < n_calls; ++k) {
        for (int v = 0; v < views_per_call[k]; ++v) {
            if (!dL[off[k] + v]) return fail(c, VGR_ERR_INVALID_ARG, "dL_dout[%d] is NULL", off[k] + v);
            ps[k].vinfo[v].dL = dL[off[k] + v];
        }
        HIP_TRY(c, hipMemcpy(ptr<ViewInfo>(c->views_graph) + off[k], ps[k].vinfo.data(),
                             sizeof(ViewInfo) * views_per_call[k], hipMemcpyHostToDevice));
    }
    HIP_TRY(c, launch_fill_u32(ptr<uint32_t>(c->words) + 5, 0u, 1, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
    if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
    c->graph_valid = false;
    hipStream_t s = c->stream;
    if (!s) {
        if (!c->own_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
        s = c->own_stream;
    }
    const bool counting2 = c->counting;
    c->counting = false;
    c->cur = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    Buffers b;
    int64_t K;
    rc = VGR_OK;
    // the calls run one after the other on the one workspace: each backward
    // consumes its own forward before the next forward overwrites it
    for (int k = 0; k < n_calls && !rc; ++k) {
        const ViewInfo *vg = ptr<ViewInfo>(c->views_graph) + off[k];
        rc = enqueue_forward(c, ps[k], means, quats, scales, dens, sh, vg, cap, s, b, K);
        if (!rc)
            rc = enqueue_backward(c, ps[k].rp, b, vg, means, quats, scales, dens, sh, d_means,
                                  d_quats, d_scales, d_dens, d_sh, !(zero_grads && k == 0), s);
    }
    c->counting = counting2;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(c, VGR_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(c, VGR_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    c->graph = g;
    c->graph_cap = cap;
    c->graph_valid = true;
    // the last captured call also serves as the saved forward of this context
    c->rp = ps[n_calls - 1].rp;
    c->buf = b;
    c->K = cap;
    c->vinfo = ps[n_calls - 1].vinfo;
    c->means = means; c->quats = quats; c->scales = scales; c->dens = dens; c->sh = sh;
    c->have_fwd = false;
    return VGR_OK;
}

int vgr_graph_capture(vgr_ctx *c, const vgr_settings *st, int64_t n, const float *means,
                      const float *quats, const float *scales, const float *dens, const float *sh,
                      int32_t n_views, const vgr_camera *cams, float *const *out,
                      const float *const *dL, float *d_means, float *d_quats, float *d_scales,
                      float *d_dens, float *d_sh, float capacity_factor, int32_t zero_grads)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    if (n_views < 1 || n_views > kMaxViews)
        return fail(c, VGR_ERR_INVALID_ARG, "n_views must be in [1, %d]", kMaxViews);
    return vgr_graph_capture_calls(c, st, n, means, quats, scales, dens, sh, 1, &n_views, cams, out,
                                   dL, d_means, d_quats, d_scales, d_dens, d_sh, capacity_factor,
                                   zero_grads);
}

int vgr_graph_launch(vgr_ctx *c)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    if (!c->graph_valid || !c->graph_exec)
        return fail(c, VGR_ERR_NOT_CAPTURED, "no valid captured graph (re-capture after reallocation)");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream ? c->stream : c->own_stream));
    return VGR_OK;
}

int vgr_graph_check(vgr_ctx *c, int64_t *instances)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    if (!c->graph_exec) return fail(c, VGR_ERR_NOT_CAPTURED, "no captured graph");
    hipStream_t s = c->stream ? c->stream : c->own_stream;
    HIP_TRY(c, hipStreamSynchronize(s));
    uint32_t words[6];
    HIP_TRY(c, hipMemcpy(words, c->words.p, sizeof words, hipMemcpyDeviceToHost));
    if (instances) *instances = words[0];
    if (words[5]) {
        const uint32_t zero = 0;
        HIP_TRY(c, hipMemcpy(ptr<uint32_t>(c->words) + 5, &zero, 4, hipMemcpyHostToDevice));
        return fail(c, VGR_ERR_CAPACITY,
                    "a graph launch needed more than %lld instances; re-capture",
                    (long long)c->graph_cap);
    }
    return VGR_OK;
}

int vgr_autotune(vgr_ctx *c, const vgr_settings *st, int64_t n, const float *means,
                 const float *quats, const float *scales, const float *dens, const float *sh,
                 int32_t n_views, const vgr_camera *cams, float *const *out,
                 const float *const *dL, float *d_means, float *d_quats, float *d_scales,
                 float *d_dens, float *d_sh, int32_t iters, int32_t *best_w, int32_t *best_h,
                 int32_t *best_batch, float *ms_per_candidate)
{
    if (!c || !st) return VGR_ERR_INVALID_ARG;
    if (n_views < 1 || n_views > kMaxViews || !cams)
        return fail(c, VGR_ERR_INVALID_ARG, "bad views");
    if (st->pixel_window > 0)
        return fail(c, VGR_ERR_INVALID_ARG, "pixel_window fixes the launch shape: nothing to tune");
    static const int cand[VGR_TUNE_CANDIDATES][3] = {
        { 8, 8, 64 }, { 16, 8, 64 }, { 16, 16, 64 }, { 32, 8, 64 },
        { 8, 8, 32 }, { 16, 8, 32 }, { 16, 16, 32 }, { 32, 8, 32 } };
    if (iters < 1) iters = 3;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    const bool timing = c->timing;
    c->timing = false;
    float best = 1e30f;
    int bi = -1, rc = VGR_OK;
    for (int k = 0; k < VGR_TUNE_CANDIDATES && !rc; ++k) {
        vgr_settings s2 = *st;
        s2.tile_w = cand[k][0];
        s2.tile_h = cand[k][1];
        s2.batch = cand[k][2];
        float ms = 0.f;
        for (int it = 0; it <= iters && !rc; ++it) {   // the first pass warms up
            if (it == 1) (void)hipEventRecord(e0, c->stream);
            rc = vgr_render_forward(c, &s2, n, means, quats, scales, dens, sh, n_views, cams, out);
            if (!rc && dL)
                rc = vgr_render_backward(c, dL, d_means, d_quats, d_scales, d_dens, d_sh, 1);
        }
        if (rc) break;
        (void)hipEventRecord(e1, c->stream);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= iters;
        if (ms_per_candidate) ms_per_candidate[k] = ms;
        if (ms < best) { best = ms; bi = k; }
    }
    c->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    c->tuned_w = cand[bi][0];
    c->tuned_h = cand[bi][1];
    c->tuned_b = cand[bi][2];
    c->tune_cache[tune_key(st, n, n_views, cams)] = TuneVal{ c->tuned_w, c->tuned_h, c->tuned_b, best };
    if (best_w) *best_w = c->tuned_w;
    if (best_h) *best_h = c->tuned_h;
    if (best_batch) *best_batch = c->tuned_b;
    return VGR_OK;
}

int vgr_tune_export(vgr_ctx *c, char *buf, int64_t cap, int64_t *len)
{
    if (!c) return VGR_ERR_INVALID_ARG;
    c->err.clear();
    std::string txt;
    char line[160];
    for (const auto &kv : c->tune_cache) {
        const TuneKey &k = kv.first;
        const TuneVal &v = kv.second;
        snprintf(line, sizeof line, "%d %d %d %d %d %d %d %d %d %d %.6g\n", k.pix_log2, k.n_log2,
                 k.mode, k.alpha_model, k.kernel, k.tile_resort, k.near_segment, v.tile_w, v.tile_h,
                 v.batch, (double)v.ms);
        txt += line;
    }
    if (len) *len = (int64_t)txt.size() + 1;
    if (!buf) return VGR_OK;
    if (cap < (int64_t)txt.size() + 1)
        return fail(c, VGR_ERR_INVALID_ARG, "buffer too small (%lld bytes needed)",
                    (long long)txt.size() + 1);
    memcpy(buf, txt.c_str(), txt.size() + 1);
    return VGR_OK;
}

int vgr_tune_import(vgr_ctx *c, const char *text)
{
    if (!c || !text) return VGR_ERR_INVALID_ARG;
    c->err.clear();
    std::map<TuneKey, TuneVal> add;
    const char *p = text;
    int lineno = 0;
    while (*p) {
        const char *e = strchr(p, '\n');
        const size_t L = e ? (size_t)(e - p) : strlen(p);
        ++lineno;
        std::string ln(p, L);
        p += L + (e ? 1 : 0);
        if (ln.find_first_not_of(" \t\r") == std::string::npos) continue;
        TuneKey k{};
        TuneVal v{};
        double ms = 0.0;
        if (sscanf(ln.c_str(), "%d %d %d %d %d %d %d %d %d %d %lf", &k.pix_log2, &k.n_log2, &k.mode,
                   &k.alpha_model, &k.kernel, &k.tile_resort, &k.near_segment, &v.tile_w, &v.tile_h,
                   &v.batch, &ms) != 11 ||
            !valid_tile(v.tile_w, v.tile_h) || (v.batch != 32 && v.batch != 64))
            return fail(c, VGR_ERR_INVALID_ARG, "tuning line %d is malformed", lineno);
        v.ms = (float)ms;
        add[k] = v;
    }
    for (const auto &kv : add) c->tune_cache[kv.first] = kv.second;
    return VGR_OK;
}

}  // extern "C"

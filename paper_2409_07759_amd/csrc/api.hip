// Host side of libswgs.so: argument checks, plans and workspace layout, and
// the launch sequences of the render, backward, step, relocation, window
// step and mature calls declared in include/swgs.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>

#include "swgs_internal.h"

using namespace swgs;

namespace {

#define HIP_TRY(ctx, expr)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail((ctx), SWGS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

swgs_status fail(swgs_context *ctx, swgs_status st, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return st;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Scratch {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::map<const swgs_context *, Scratch> g_scratch;

hipError_t ctx_scratch(swgs_context *ctx, size_t bytes, void **out) {
    Scratch &s = g_scratch[ctx];
    if (s.bytes < bytes) {
        if (s.ptr) {
            hipError_t e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) return e;
            (void)hipFree(s.ptr);
            s.ptr = nullptr;
            s.bytes = 0;
        }
        hipError_t e = hipMalloc(&s.ptr, bytes);
        if (e != hipSuccess) return e;
        s.bytes = bytes;
    }
    *out = s.ptr;
    return hipSuccess;
}

// Scratch of swgs_mature_noalloc: a file-scope device array (each device
// that runs the library holds its own copy until the process ends).  Host
// code never uses the array's name as an address: its device address is
// looked up once per device, with that device current, when a context is
// created on it, and kept in g_noalloc_ptr.
constexpr size_t kNoAllocWords = size_t(4) << 20;               // 16 MiB
static __device__ __align__(256) uint32_t scratch[kNoAllocWords];
constexpr int kMaxDevices = 64;
void *g_noalloc_ptr[kMaxDevices] = {};
std::mutex g_noalloc_mu;

hipError_t noalloc_lookup(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (g_noalloc_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_noalloc_ptr[device] = ptr;
    return hipSuccess;
}

// words of mature's scratch for num_gs slots: flags, positions, the scan's
// per-chunk sums, the count
size_t mature_scratch_words(size_t n) { return 2 * (n + 1) + n / 4096 + 8; }

bool pool_ok(const swgs_pool *p, bool need_train, std::string &why) {
    if (!p) { why = "pool is NULL"; return false; }
    if (p->struct_size != sizeof(swgs_pool)) { why = "pool.struct_size mismatch"; return false; }
    if (p->sh_degree < 0 || p->sh_degree > kMaxShDegree) { why = "sh_degree must be 0..3"; return false; }
    if (p->n_slots < 1 || p->num_gs < 0 || p->num_gs > p->n_slots) { why = "need 0 <= num_gs <= n_slots, n_slots >= 1"; return false; }
    if (p->swin <= 0) { why = "swin must be > 0"; return false; }
    if (!p->params || !p->start || !p->expire) { why = "params/start/expire must not be NULL"; return false; }
    if (need_train && p->num_gs > 0 && (!p->grads || !p->adam_m || !p->adam_v)) {
        why = "grads/adam_m/adam_v must not be NULL for training";
        return false;
    }
    return true;
}

// Constant block uploaded at the head of each call: views, groups, group
// view list, record view bases.
void upload_consts(hipStream_t s, swgs_plan &p, uint8_t *ws) {
    (void)hipMemcpyAsync(ws + p.lay.off[WB_VIEWS], p.consts_host, p.consts_bytes, hipMemcpyHostToDevice, s);
}

swgs_status check_ws(swgs_context *ctx, const swgs_plan *p, const void *ws, size_t ws_bytes) {
    if (!ws) return fail(ctx, SWGS_ERR_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(ctx, SWGS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < p->lay.total)
        return fail(ctx, SWGS_ERR_WORKSPACE_TOO_SMALL,
                    "workspace has " + std::to_string(ws_bytes) + " bytes, needs " + std::to_string(p->lay.total));
    return SWGS_OK;
}

}  // namespace

void swgs::compute_layout(const LayoutDims &d, Layout &lay, size_t &consts_bytes) {
    const size_t G = d.G, V = d.V, R = d.R, T = d.T, P = d.P, cap = d.cap;
    const size_t S = d.S, NG = d.NG, nA = d.nA, n_list = d.n_list;
    const size_t nblk = (S + kGateChunk - 1) / kGateChunk;
    const size_t nbu = (nA + 2047) / 2048;
    size_t sz[WB_COUNT];
    std::memset(sz, 0, sizeof sz);
    // constant block first, contiguous
    sz[WB_VIEWS] = V * sizeof(ViewDev);
    sz[WB_GROUPS] = G * sizeof(GroupDev);
    sz[WB_GROUP_VIEWS] = V * 4;
    sz[WB_REC_VIEW_BASE] = (V + 1) * 4;
    sz[WB_ACTIVE_LIST] = (n_list + 1) * 4;
    sz[WB_ACTIVE_COUNT] = (G + 1) * 4;
    sz[WB_DEPTH_KEY] = R * 4;
    sz[WB_TILE_COUNT] = R * 4;
    sz[WB_RECT] = R * 8;
    sz[WB_RECT_SORTED] = R * 8;
    sz[WB_SPLAT] = R * kSplatFloats * 4;
    sz[WB_PAIR_KEY] = cap * 4;
    sz[WB_PAIR_VAL] = cap * 4;
    sz[WB_PAIR_COUNT] = 4 * 4;
    sz[WB_TILE_RANGE] = T * 8;
    sz[WB_T_FINAL] = P * 4;
    sz[WB_DLDC] = 3 * P * 4;
    sz[WB_REC_GRAD] = 9 * R * 4;
    sz[WB_GATE_BLK] = (G + 1) * nblk * 4;
    sz[WB_POS_OF] = G * NG * 4;
    sz[WB_PAIR_KEY_ALT] = cap * 4;
    sz[WB_PAIR_VAL_ALT] = cap * 4;
    sz[WB_REC_IDX] = R * 4;
    sz[WB_KEY_ALT] = R * 4;
    sz[WB_IDX_ALT] = R * 4;
    sz[WB_PAIR_OFFSET] = (R + 1) * 4;
    sz[WB_SORT_HIST] = (size_t)2048 * kSortBlocks * 4;
    sz[WB_SORT_TOTAL] = (std::max<size_t>(2048, R / 4096 + 2) + 8) * 4;
    sz[WB_LAST] = P * 4;
    sz[WB_LOSS_PART] = 2 * (T + 256) * 8;   // per-tile partials, then 256 chunk sums
    sz[WB_STATS] = 8 * 8;
    sz[WB_STEP] = sizeof(StepDev);
    sz[WB_RELOC_W] = (nA + 1 + nbu + 4) * 8;
    sz[WB_RELOC_FLAG] = 2 * (nA + 1) * 4;
    sz[WB_RELOC_CNT] = 2 * (nA + 1) * 4;
    sz[WB_RELOC_SRC] = (nA + 1) * 4;
    sz[WB_RELOC_DST] = (nA + 1) * 4;
    sz[WB_RELOC_SCAN] = (4 + nA / 4096 + 4) * 4;
    sz[WB_REG_PART] = 2 * ((nA + 255) / 256 + 1) * 8;
    sz[WB_COUNTERS] = 256 * 4 * 8;   // 256 slots x {fwd evals, bwd evals, blended, pad}
    sz[WB_CFLAGS] = R + 16;
    sz[WB_SSIM_PART] = 9 * P * 4;                     // dS/d(mu_x, E[x^2], E[xy]) per pixel and channel
    sz[WB_SSIM_SUM] = (3 * d.Tssim + 256) * 8;          // per (SSIM tile, channel), then 256 chunk sums
    sz[WB_IMAGE] = 3 * P * 4;                         // renders when the caller passes no image buffer
    sz[WB_PAIR_BASE] = R * 8;                         // each record's slot base and rect width (row scan -> backward)
    sz[WB_ROW_OFFSET] = (R + 1) * 4;                  // each record's first gradient row (row scan -> reduce)
    sz[WB_PAIR_MASK] = (cap + 3) / 4 * 4;             // each pair's support mask over the tile's waves (forward -> backward)
    sz[WB_PAIR_GRAD] = cap * 9 * 4 + 16;              // 9 gradient terms per (tile, record) pair, record
                                                      // order (+16: the reduce reads whole 16-byte vectors)
    if (d.forward_only) {
        // serving: no gating (the live lists are resident), no gradients,
        // no loss, no step
        for (int b : {WB_ACTIVE_LIST, WB_GATE_BLK, WB_POS_OF, WB_DLDC, WB_REC_GRAD, WB_LOSS_PART, WB_RELOC_W,
                      WB_RELOC_FLAG, WB_RELOC_CNT, WB_RELOC_SRC, WB_RELOC_DST, WB_RELOC_SCAN, WB_REG_PART,
                      WB_SSIM_PART, WB_SSIM_SUM, WB_IMAGE, WB_PAIR_BASE, WB_PAIR_GRAD, WB_PAIR_MASK,
                      WB_ROW_OFFSET})
            sz[b] = 0;
        if (d.own_lists) {
            // a standalone batch render gates into its workspace (no
            // optimisable slots: no window set, no pos_of)
            sz[WB_ACTIVE_LIST] = (n_list + 1) * 4;
            sz[WB_GATE_BLK] = (G + 1) * nblk * 4;
        }
    }
    // order: constant block, then the rest
    const int order_first[] = {WB_VIEWS, WB_GROUPS, WB_GROUP_VIEWS, WB_REC_VIEW_BASE};
    size_t off = 0;
    for (int b : order_first) {
        lay.off[b] = off;
        lay.size[b] = sz[b];
        off = align_up(off + sz[b], 16);
    }
    consts_bytes = off;
    off = align_up(off, 256);
    for (int b = 0; b < WB_COUNT; ++b) {
        if (b == WB_VIEWS || b == WB_GROUPS || b == WB_GROUP_VIEWS || b == WB_REC_VIEW_BASE) continue;
        lay.off[b] = off;
        lay.size[b] = sz[b];
        off = align_up(off + sz[b], 256);
    }
    lay.total = off;
}

namespace {

void build_layout(swgs_plan &p) {
    LayoutDims d;
    d.G = p.groups.size();
    d.V = p.views.size();
    d.R = (size_t)p.R;
    d.T = (size_t)p.T;
    d.P = (size_t)p.P;
    d.cap = (size_t)p.pair_cap;
    d.S = (size_t)p.pool.n_slots;
    d.NG = (size_t)p.pool.num_gs;
    d.nA = p.n_A;
    d.n_list = p.n_A;
    for (auto &g : p.groups) d.n_list += g.n_live;
    d.Tssim = (size_t)p.Tssim;
    d.forward_only = p.forward_only;
    d.own_lists = p.own_lists;
    compute_layout(d, p.lay, p.consts_bytes);
}


// kernel classes timed with events when a plan's timing is on
enum { TK_GATE = 0, TK_PREPROCESS, TK_SORT, TK_FWD, TK_BWD, TK_PREBWD, TK_ADAM, TK_RELOC, TK_SSIM, TK_N };

struct TimeScope {
    swgs_plan &p;
    hipStream_t s;
    int kind;
    bool on;
    TimeScope(swgs_plan &p_, hipStream_t s_, int k) : p(p_), s(s_), kind(k), on(p_.timing) {
        if (on) rec();
    }
    ~TimeScope() {
        if (on) rec();
    }
    void rec() {
        auto &v = p.ev[kind];
        if (p.ev_used[kind] == v.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
            v.push_back(e);
        }
        (void)hipEventRecord(v[p.ev_used[kind]++], s);
    }
};

int tile_bits(int64_t T) {
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) < T) ++b;
    return b;
}

unsigned long long *counters_of(swgs_plan &p, uint8_t *ws) {
    return p.counting ? wsp<unsigned long long>(ws, p, WB_COUNTERS) : nullptr;
}

// ------------------------------------------------------------ launch blocks
void seq_gate(hipStream_t s, swgs_plan &p, uint8_t *ws) {
    TimeScope t(p, s, TK_GATE);
    launch_gate(s, p, ws);
}

// forward of records [rec_lo, rec_hi) and tiles [tile_lo, tile_hi): one
// view (plain) or all views (batched)
// with ssim_follows the D-SSIM backward writes the whole of dL/dC (its L1
// term included), so the forward only takes the loss
void seq_forward(hipStream_t s, swgs_plan &p, uint8_t *ws, int view, float *images, const float *targets,
                 float l1_weight = 1.0f, bool ssim_follows = false) {
    uint32_t rec_lo = 0, rec_hi = (uint32_t)p.R, tile_lo = 0, tile_hi = (uint32_t)p.T;
    if (view >= 0) {
        rec_lo = p.vdev[view].rec_base;
        rec_hi = view + 1 < (int)p.views.size() ? p.vdev[view + 1].rec_base : (uint32_t)p.R;
        tile_lo = p.vdev[view].tile_base;
        tile_hi = view + 1 < (int)p.views.size() ? p.vdev[view + 1].tile_base : (uint32_t)p.T;
    }
    {
        TimeScope t(p, s, TK_PREPROCESS);
        launch_preprocess(s, p, ws, view, view);
    }
    {
        TimeScope t(p, s, TK_SORT);
        uint32_t *hist = wsp<uint32_t>(ws, p, WB_SORT_HIST), *tot = wsp<uint32_t>(ws, p, WB_SORT_TOTAL);
        // records by FP32 depth (ties keep record order), then the pairs
        // emitted in that order stably by tile: (tile, depth, record) order
        radix_sort_pairs(s, wsp<uint32_t>(ws, p, WB_DEPTH_KEY) + rec_lo, wsp<uint32_t>(ws, p, WB_REC_IDX) + rec_lo,
                         wsp<uint32_t>(ws, p, WB_KEY_ALT) + rec_lo, wsp<uint32_t>(ws, p, WB_IDX_ALT) + rec_lo, nullptr,
                         rec_hi - rec_lo, rec_hi - rec_lo, 32, hist, tot, wsp<uint2>(ws, p, WB_RECT),
                         wsp<uint2>(ws, p, WB_RECT_SORTED), wsp<uint32_t>(ws, p, WB_PAIR_OFFSET));
        launch_pair_offsets(s, p, ws, rec_lo, rec_hi);
        launch_emit_pairs(s, p, ws, rec_lo, rec_hi);
        launch_row_offsets(s, p, ws, rec_lo, rec_hi);
        uint32_t *pc = wsp<uint32_t>(ws, p, WB_PAIR_COUNT);
        radix_sort_pairs(s, wsp<uint32_t>(ws, p, WB_PAIR_KEY), wsp<uint32_t>(ws, p, WB_PAIR_VAL),
                         wsp<uint32_t>(ws, p, WB_PAIR_KEY_ALT), wsp<uint32_t>(ws, p, WB_PAIR_VAL_ALT), pc, 0,
                         (uint32_t)p.pair_cap, p.tile_key_bits, hist, tot);
        launch_tile_ranges(s, p, ws, tile_lo, tile_hi);
    }
    {
        TimeScope t(p, s, TK_FWD);
        launch_blend_forward(s, p, ws, images, targets, tile_lo, tile_hi, counters_of(p, ws), l1_weight,
                             !ssim_follows);
    }
}

// backward blend of one view (plain) or all views, then the record
// gradients of the same records from their per-pair terms (a view's pair
// slots are reused by the next view, so the reduce follows each backward)
void seq_backward_blend(hipStream_t s, swgs_plan &p, uint8_t *ws, int view, const float *dLdC) {
    uint32_t rec_lo = 0, rec_hi = (uint32_t)p.R, tile_lo = 0, tile_hi = (uint32_t)p.T;
    if (view >= 0) {
        rec_lo = p.vdev[view].rec_base;
        rec_hi = view + 1 < (int)p.views.size() ? p.vdev[view + 1].rec_base : (uint32_t)p.R;
        tile_lo = p.vdev[view].tile_base;
        tile_hi = view + 1 < (int)p.views.size() ? p.vdev[view + 1].tile_base : (uint32_t)p.T;
    }
    {
        TimeScope t(p, s, TK_BWD);
        launch_blend_backward(s, p, ws, dLdC, tile_lo, tile_hi, counters_of(p, ws));
    }
    TimeScope t(p, s, TK_PREBWD);
    launch_pair_grad_reduce(s, p, ws, rec_lo, rec_hi);
}

}  // namespace


std::string swgs::plan_geometry(swgs_plan &p, const swgs_view *views, int n_views, const std::vector<int32_t> &frames,
                                const std::vector<int> &vgroup, const std::vector<uint32_t> &live, uint32_t n_A) {
    const int G = (int)frames.size();
    p.views.assign(views, views + n_views);
    p.groups.clear();
    p.group_views.clear();
    // groups and the group-ordered view list
    p.groups.resize(G);
    uint32_t lb_acc = 0;
    for (int g = 0; g < G; ++g) {
        GroupDev &gd = p.groups[g];
        std::memset(&gd, 0, sizeof gd);
        gd.frame = frames[g];
        gd.n_live = live[g];
        gd.list_base = lb_acc;
        lb_acc += live[g];
    }
    p.n_A = n_A;
    p.list_A_base = lb_acc;
    for (int g = 0; g < G; ++g) {
        p.groups[g].view_first = (int32_t)p.group_views.size();
        for (int v = 0; v < n_views; ++v)
            if (vgroup[v] == g) p.group_views.push_back(v);
        p.groups[g].n_views = (int32_t)p.group_views.size() - p.groups[g].view_first;
    }
    // per-view geometry in caller order
    p.vdev.resize(n_views);
    uint64_t rec = 0, tiles = 0, tssim = 0;
    int64_t pix = 0;
    for (int v = 0; v < n_views; ++v) {
        const swgs_view &w = views[v];
        ViewDev &d = p.vdev[v];
        std::memset(&d, 0, sizeof d);
        std::memcpy(d.R, w.R, sizeof d.R);
        std::memcpy(d.t, w.t, sizeof d.t);
        d.fx = w.fx; d.fy = w.fy; d.cx = w.cx; d.cy = w.cy;
        for (int c = 0; c < 3; ++c) d.campos[c] = -(w.R[c] * w.t[0] + w.R[3 + c] * w.t[1] + w.R[6 + c] * w.t[2]);
        d.limx = 1.3 * (0.5 * w.width / w.fx);
        d.limy = 1.3 * (0.5 * w.height / w.fy);
        for (int c = 0; c < 3; ++c) d.bg[c] = w.bg[c];
        d.frame = w.frame;
        d.width = w.width;
        d.height = w.height;
        d.tiles_x = (w.width + p.tile_w - 1) / p.tile_w;
        d.tiles_y = (w.height + p.tile_h - 1) / p.tile_h;
        d.group = vgroup[v];
        d.rec_base = (uint32_t)rec;
        d.tile_base = (uint32_t)tiles;
        d.pix_base = pix;
        d.inv_norm = (float)(1.0 / ((double)n_views * 3.0 * (double)w.width * (double)w.height));
        d.ssim_tile_base = (uint32_t)tssim;
        tssim += ssim_tiles(w.width, w.height);
        rec += live[vgroup[v]];
        tiles += (uint64_t)d.tiles_x * d.tiles_y;
        pix += (int64_t)w.width * w.height;
    }
    if (rec >= 0xFFFFFFF0ull || tiles >= 0xFFFFFFF0ull) return "more than 2^32 records or tiles in one plan";
    // the work per tile follows the live Gaussians per pixel of a view: a
    // window whose views differ there is launched spread over the XCDs
    double dmin = 1e300, dmax = 0.0;
    for (int v = 0; v < n_views; ++v) {
        const double d = (double)live[vgroup[v]] / ((double)views[v].width * (double)views[v].height);
        dmin = std::min(dmin, d);
        dmax = std::max(dmax, d);
    }
    p.uneven = n_views > 1 && dmax > 1.25 * dmin;
    p.R = (int64_t)rec;
    p.T = (int64_t)tiles;
    p.Tssim = (int64_t)tssim;
    p.tile_key_bits = tile_bits(p.T);
    p.P = pix;
    build_layout(p);
    return std::string();
}

void swgs::fill_consts(swgs_plan &p) {
    uint8_t *h = static_cast<uint8_t *>(p.consts_host);
    std::memset(h, 0, p.consts_bytes);
    std::memcpy(h + p.lay.off[WB_VIEWS], p.vdev.data(), p.vdev.size() * sizeof(ViewDev));
    std::memcpy(h + p.lay.off[WB_GROUPS], p.groups.data(), p.groups.size() * sizeof(GroupDev));
    std::memcpy(h + p.lay.off[WB_GROUP_VIEWS], p.group_views.data(), p.group_views.size() * 4);
    std::vector<uint32_t> rvb(p.views.size() + 1);
    for (size_t v = 0; v < p.views.size(); ++v) rvb[v] = p.vdev[v].rec_base;
    rvb[p.views.size()] = (uint32_t)p.R;
    std::memcpy(h + p.lay.off[WB_REC_VIEW_BASE], rvb.data(), rvb.size() * 4);
}

void swgs::seq_forward_all(hipStream_t s, swgs_plan &p, uint8_t *ws, float *images, const float *targets) {
    seq_forward(s, p, ws, -1, images, targets);
}

std::string swgs::tile_opts(int tile_w, int tile_h, int lds_batch, int *tw, int *th, int *lb) {
    int w = tile_w, h = tile_h;
    if (w == 0 && h == 0) { w = 16; h = 16; }
    if (!((w == 16 && h == 16) || (w == 8 && h == 8) || (w == 32 && h == 8)))
        return "tile shape must be 8x8, 16x16 or 32x8";
    const int b = lds_batch == 0 ? w * h : lds_batch;
    if (!(b == 64 || b == 128 || b == 256)) return "lds_batch must be 64, 128 or 256";
    if (b == 64 && !(w == 8 && h == 8)) return "lds_batch 64 needs 8x8 tiles";
    *tw = w;
    *th = h;
    *lb = b;
    return std::string();
}

// ============================================================== ABI
extern "C" {

int swgs_version(void) { return SWGS_VERSION; }

void swgs_step_cfg_default(swgs_step_cfg *c) {
    if (!c) return;
    std::memset(c, 0, sizeof *c);
    c->struct_size = sizeof *c;
    c->lr_mean = 1.6e-4f;
    c->lr_scale = 5e-3f;
    c->lr_quat = 1e-3f;
    c->lr_logit = 5e-2f;
    c->lr_sh_dc = 2.5e-3f;
    c->lr_sh_rest = 1.25e-4f;
    c->beta1 = 0.9f;
    c->beta2 = 0.999f;
    c->eps = 1e-15f;
    c->noise_lr = 5e4f;
    c->noise_k = 100.0f;
    c->noise_t0 = 0.005f;
    c->lambda_opacity = 2e-2f;
    c->lambda_scale = 1e-2f;
    c->lambda_dssim = 0.2f;
    c->grad_scale_base = 0.0f;
    c->window_start = 0;
    c->relocate_period = 1;
    c->reloc_n_max = 32;
    c->mode = SWGS_MODE_BATCHED;
}

swgs_status swgs_context_create(int device, void *hip_stream, swgs_context **out) {
    if (!out) return SWGS_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SWGS_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return SWGS_ERR_HIP;
    // the allocation-free entry points' scratch address on this device
    if (noalloc_lookup(device) != hipSuccess) return SWGS_ERR_HIP;
    auto *c = new (std::nothrow) swgs_context;
    if (!c) return SWGS_ERR_HIP;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    *out = c;
    return SWGS_OK;
}

swgs_status swgs_context_set_stream(swgs_context *ctx, void *hip_stream) {
    if (!ctx) return SWGS_ERR_INVALID_ARG;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return SWGS_OK;
}

swgs_status swgs_context_destroy(swgs_context *ctx) {
    if (!ctx) return SWGS_ERR_INVALID_ARG;
    auto it = g_scratch.find(ctx);
    if (it != g_scratch.end()) {
        (void)hipStreamSynchronize(ctx->stream);
        if (it->second.ptr) (void)hipFree(it->second.ptr);
        g_scratch.erase(it);
    }
    delete ctx;
    return SWGS_OK;
}

const char *swgs_last_error(const swgs_context *ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

// A plan object for `views` on `pool` (checks, live counts per frame on the
// device -- synchronising --, geometry and layout).  forward_only plans
// with own_lists gate into their own workspace and keep no training
// buffers; their constant block lives in `host_consts` (pageable) instead of
// pinned memory.
static swgs_status make_plan(swgs_context *ctx, const swgs_pool *pool, const swgs_view *views, int32_t n_views,
                             const swgs_plan_opts *opts, bool forward_only, swgs_plan **out);

swgs_status swgs_plan_create(swgs_context *ctx, const swgs_pool *pool, const swgs_view *views, int32_t n_views,
                             const swgs_plan_opts *opts, swgs_plan **out, size_t *ws_bytes) {
    if (!ctx) return SWGS_ERR_INVALID_ARG;
    if (!out || !ws_bytes) return fail(ctx, SWGS_ERR_INVALID_ARG, "out/ws_bytes must not be NULL");
    *out = nullptr;
    swgs_plan *p = nullptr;
    const swgs_status st = make_plan(ctx, pool, views, n_views, opts, false, &p);
    if (st != SWGS_OK) return st;
    if (hipHostMalloc(&p->consts_host, p->consts_bytes) != hipSuccess) {
        delete p;
        return fail(ctx, SWGS_ERR_HIP, "pinned constant block alloc failed");
    }
    fill_consts(*p);
    *out = p;
    *ws_bytes = p->lay.total;
    return SWGS_OK;
}

static swgs_status make_plan(swgs_context *ctx, const swgs_pool *pool, const swgs_view *views, int32_t n_views,
                             const swgs_plan_opts *opts, bool forward_only, swgs_plan **out) {
    *out = nullptr;
    std::string why;
    if (!pool_ok(pool, false, why)) return fail(ctx, SWGS_ERR_INVALID_ARG, why);
    if (!views || n_views <= 0) return fail(ctx, SWGS_ERR_INVALID_ARG, "need at least one view");
    if (n_views > 65535) return fail(ctx, SWGS_ERR_UNSUPPORTED, "at most 65535 views per plan");
    if (!opts || opts->struct_size != sizeof(swgs_plan_opts)) return fail(ctx, SWGS_ERR_INVALID_ARG, "opts.struct_size mismatch");
    int tw = 16, th = 16, lb = 256;
    const std::string terr = tile_opts(opts->tile_w, opts->tile_h, opts->lds_batch, &tw, &th, &lb);
    if (!terr.empty()) return fail(ctx, SWGS_ERR_UNSUPPORTED, terr);
    if (opts->pair_capacity <= 0 || opts->pair_capacity > 0xFFFFFFF0LL)
        return fail(ctx, SWGS_ERR_INVALID_ARG, "pair_capacity must be in (0, 2^32 - 16)");
    for (int v = 0; v < n_views; ++v) {
        const swgs_view &w = views[v];
        if (w.width <= 0 || w.height <= 0 || w.width > 16384 * 8 || w.height > 16384 * 8 ||
            (int64_t)w.width * w.height > (int64_t)INT32_MAX)
            return fail(ctx, SWGS_ERR_INVALID_ARG, "view " + std::to_string(v) + ": bad size");
        if (!(w.fx > 0 && w.fy > 0)) return fail(ctx, SWGS_ERR_INVALID_ARG, "view " + std::to_string(v) + ": focal must be > 0");
    }
    auto *p = new (std::nothrow) swgs_plan;
    if (!p) return fail(ctx, SWGS_ERR_HIP, "out of host memory");
    p->pool = *pool;
    if (forward_only) {
        // every live slot is drawn; none is optimised
        p->pool.num_gs = 0;
        p->forward_only = true;
        p->own_lists = true;
    }
    p->sh_degree = pool->sh_degree;
    p->F = rows_for(pool->sh_degree);
    p->tile_w = tw;
    p->tile_h = th;
    p->lds_batch = lb;
    p->pair_cap = opts->pair_capacity;
    // distinct frames in order of appearance
    std::vector<int32_t> frames;
    std::vector<int> vgroup(n_views);
    for (int v = 0; v < n_views; ++v) {
        auto it = std::find(frames.begin(), frames.end(), views[v].frame);
        if (it == frames.end()) { vgroup[v] = (int)frames.size(); frames.push_back(views[v].frame); }
        else vgroup[v] = (int)(it - frames.begin());
    }
    const int G = (int)frames.size();
    // live counts per frame and |A| on the device (synchronising)
    void *scr = nullptr;
    if (ctx_scratch(ctx, 4 * (2 * G + 8), &scr) != hipSuccess) { delete p; return fail(ctx, SWGS_ERR_HIP, "scratch alloc failed"); }
    int32_t *d_frames = static_cast<int32_t *>(scr);
    uint32_t *d_counts = reinterpret_cast<uint32_t *>(d_frames + G + 2);
    std::vector<uint32_t> counts(G + 1, 0);
    if (hipMemcpyAsync(d_frames, frames.data(), 4 * G, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        hipMemsetAsync(d_counts, 0, 4 * (G + 1), ctx->stream) != hipSuccess) {
        delete p;
        return fail(ctx, SWGS_ERR_HIP, "count upload failed");
    }
    launch_count_live(ctx->stream, pool->start, pool->expire, pool->n_slots, p->pool.num_gs, d_frames, G, d_counts);
    if (hipMemcpyAsync(counts.data(), d_counts, 4 * (G + 1), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        delete p;
        return fail(ctx, SWGS_ERR_HIP, std::string("live count failed: ") + hipGetErrorString(hipGetLastError()));
    }
    std::vector<uint32_t> live(counts.begin(), counts.begin() + G);
    const std::string gerr = plan_geometry(*p, views, n_views, frames, vgroup, live, counts[G]);
    if (!gerr.empty()) {
        delete p;
        return fail(ctx, SWGS_ERR_UNSUPPORTED, gerr);
    }
    *out = p;
    return SWGS_OK;
}

// ------------------------------------------------------------ pool handles
struct swgs_pool_handle {
    swgs_pool desc{};
    int device = 0;
};

static bool device_ptr_on(const void *ptr, int device) {
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof a);
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();   // an unknown host pointer is an answer, not a sticky error
        return false;
    }
    return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == device;
}

swgs_status swgs_pool_bind(swgs_context *ctx, const swgs_pool *desc, swgs_pool_handle **out) {
    if (!ctx) return SWGS_ERR_INVALID_ARG;
    if (!out) return fail(ctx, SWGS_ERR_INVALID_ARG, "out must not be NULL");
    *out = nullptr;
    std::string why;
    if (!pool_ok(desc, false, why)) return fail(ctx, SWGS_ERR_INVALID_ARG, why);
    const struct { const void *p; const char *name; } ptrs[] = {
        {desc->params, "params"}, {desc->grads, "grads"}, {desc->adam_m, "adam_m"}, {desc->adam_v, "adam_v"},
        {desc->birth, "birth"}, {desc->start, "start"}, {desc->expire, "expire"}};
    for (const auto &q : ptrs)
        if (q.p && !device_ptr_on(q.p, ctx->device))
            return fail(ctx, SWGS_ERR_INVALID_ARG, std::string("pool.") + q.name + " is not device memory of device " +
                                                       std::to_string(ctx->device));
    auto *h = new (std::nothrow) swgs_pool_handle;
    if (!h) return fail(ctx, SWGS_ERR_HIP, "out of host memory");
    h->desc = *desc;
    h->device = ctx->device;
    *out = h;
    return SWGS_OK;
}

const swgs_pool *swgs_pool_desc(const swgs_pool_handle *h) { return h ? &h->desc : nullptr; }

swgs_status swgs_pool_release(swgs_pool_handle *h) {
    if (!h) return SWGS_ERR_INVALID_ARG;
    delete h;
    return SWGS_OK;
}

// ------------------------------------------------------------ batch render
static swgs_status batch_views(swgs_context *ctx, const swgs_request *reqs, int32_t n, std::vector<swgs_view> &views) {
    if (!reqs || n <= 0) return fail(ctx, SWGS_ERR_INVALID_ARG, "need at least one request");
    views.resize(n);
    for (int i = 0; i < n; ++i) views[i] = reqs[i].view;
    return SWGS_OK;
}

static size_t batch_ws_bytes(const swgs_plan &p) { return align_up(p.lay.total, 256) + align_up(12 * (size_t)p.P, 256); }

swgs_status swgs_query_workspace_batch(swgs_context *ctx, const swgs_pool *pool, const swgs_request *reqs, int32_t n,
                                       const swgs_plan_opts *opts, size_t *ws_bytes) {
    if (!ctx) return SWGS_ERR_INVALID_ARG;
    if (!ws_bytes) return fail(ctx, SWGS_ERR_INVALID_ARG, "ws_bytes must not be NULL");
    std::vector<swgs_view> views;
    swgs_status st = batch_views(ctx, reqs, n, views);
    if (st) return st;
    swgs_plan *p = nullptr;
    if ((st = make_plan(ctx, pool, views.data(), n, opts, true, &p))) return st;
    *ws_bytes = batch_ws_bytes(*p);
    delete p;
    return SWGS_OK;
}

swgs_status swgs_render_batch(swgs_context *ctx, const swgs_pool *pool, swgs_request *reqs, int32_t n,
                              const swgs_plan_opts *opts, void *workspace, size_t ws_bytes) {
    if (!ctx) return SWGS_ERR_INVALID_ARG;
    std::vector<swgs_view> views;
    swgs_status st = batch_views(ctx, reqs, n, views);
    if (st) return st;
    swgs_plan *p = nullptr;
    if ((st = make_plan(ctx, pool, views.data(), n, opts, true, &p))) return st;
    std::unique_ptr<swgs_plan> hold(p);
    if (!workspace) return fail(ctx, SWGS_ERR_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(ctx, SWGS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const size_t need = batch_ws_bytes(*p);
    if (ws_bytes < need)
        return fail(ctx, SWGS_ERR_WORKSPACE_TOO_SMALL,
                    "workspace has " + std::to_string(ws_bytes) + " bytes, needs " + std::to_string(need));
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    float *images = reinterpret_cast<float *>(ws + align_up(p->lay.total, 256));
    hipStream_t s = ctx->stream;
    // constant block from pageable memory: this call synchronises before it
    // returns, so the buffer outlives the transfer
    std::vector<uint8_t> consts(p->consts_bytes);
    p->consts_host = consts.data();
    fill_consts(*p);
    const hipError_t ce = hipMemcpyAsync(ws + p->lay.off[WB_VIEWS], consts.data(), p->consts_bytes,
                                         hipMemcpyHostToDevice, s);
    p->consts_host = nullptr;
    if (ce != hipSuccess) return fail(ctx, SWGS_ERR_HIP, std::string("constant upload: ") + hipGetErrorString(ce));
    launch_gate(s, *p, ws);
    seq_forward_all(s, *p, ws, images, nullptr);
    for (int v = 0; v < n; ++v) {
        if (!reqs[v].image) continue;
        const size_t m = 3 * (size_t)views[v].width * (size_t)views[v].height;
        HIP_TRY(ctx, hipMemcpyAsync(reqs[v].image, images + 3 * (size_t)p->vdev[v].pix_base, m * 4,
                                    hipMemcpyDeviceToDevice, s));
    }
    uint32_t pc[2] = {0, 0};
    HIP_TRY(ctx, hipMemcpyAsync(pc, wsp<uint32_t>(ws, *p, WB_PAIR_COUNT), 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const bool over = pc[1] != 0;
    for (int v = 0; v < n; ++v) {
        reqs[v].status = over ? SWGS_ERR_CAPACITY : SWGS_OK;
        reqs[v].batch = 0;
        reqs[v].ready = 0.0;
    }
    if (over)
        return fail(ctx, SWGS_ERR_CAPACITY, "batch needs " + std::to_string(pc[0]) + " pairs, capacity " +
                                                std::to_string(p->pair_cap));
    return SWGS_OK;
}

swgs_status swgs_plan_destroy(swgs_plan *p) {
    if (!p) return SWGS_ERR_INVALID_ARG;
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->consts_host) (void)hipHostFree(p->consts_host);
    for (int k = 0; k < TK_N; ++k)
        for (auto e : p->ev[k]) (void)hipEventDestroy(e);
    delete p;
    return SWGS_OK;
}

swgs_status swgs_plan_buffer(const swgs_plan *p, int32_t which, size_t *offset, size_t *bytes) {
    if (!p || !offset || !bytes) return SWGS_ERR_INVALID_ARG;
    static const int map[SWGS_BUF_COUNT_] = {WB_ACTIVE_LIST, WB_ACTIVE_COUNT, WB_REC_VIEW_BASE, WB_DEPTH_KEY,
                                             WB_TILE_COUNT, WB_RECT, WB_SPLAT, WB_PAIR_KEY, WB_PAIR_VAL,
                                             WB_PAIR_COUNT, WB_TILE_RANGE, WB_T_FINAL, WB_DLDC, WB_REC_GRAD,
                                             WB_REC_IDX};
    if (which < 0 || which >= SWGS_BUF_COUNT_) return SWGS_ERR_INVALID_ARG;
    *offset = p->lay.off[map[which]];
    *bytes = p->lay.size[map[which]];
    return SWGS_OK;
}

swgs_status swgs_plan_info(const swgs_plan *p, int64_t *n_groups, int64_t *n_records, int64_t *n_pixels,
                           int64_t *n_tiles) {
    if (!p) return SWGS_ERR_INVALID_ARG;
    if (n_groups) *n_groups = (int64_t)p->groups.size();
    if (n_records) *n_records = p->R;
    if (n_pixels) *n_pixels = p->P;
    if (n_tiles) *n_tiles = p->T;
    return SWGS_OK;
}

swgs_status swgs_plan_measure(swgs_context *ctx, swgs_plan *p, void *workspace, size_t ws_bytes, int64_t *n_pairs,
                              int64_t *n_records) {
    if (!ctx || !p) return SWGS_ERR_INVALID_ARG;
    swgs_status st = check_ws(ctx, p, workspace, ws_bytes);
    if (st) return st;
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    hipStream_t s = ctx->stream;
    upload_consts(s, *p, ws);
    launch_gate(s, *p, ws);
    launch_preprocess(s, *p, ws, -1, -1);
    uint32_t *tc = wsp<uint32_t>(ws, *p, WB_TILE_COUNT);
    uint32_t *tot = wsp<uint32_t>(ws, *p, WB_PAIR_COUNT) + 2;
    exclusive_scan_u32(s, tc, wsp<uint32_t>(ws, *p, WB_PAIR_OFFSET), (uint32_t)p->R, tot,
                       wsp<uint32_t>(ws, *p, WB_SORT_TOTAL));
    uint32_t k = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&k, tot, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (n_pairs) *n_pairs = k;
    if (n_records) *n_records = p->R;
    return SWGS_OK;
}

swgs_status swgs_render_forward(swgs_context *ctx, swgs_plan *p, void *workspace, size_t ws_bytes, float *images,
                                const float *targets, double *stats) {
    if (!ctx || !p) return SWGS_ERR_INVALID_ARG;
    swgs_status st = check_ws(ctx, p, workspace, ws_bytes);
    if (st) return st;
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    hipStream_t s = ctx->stream;
    upload_consts(s, *p, ws);
    launch_gate(s, *p, ws);
    seq_forward(s, *p, ws, -1, images, targets);
    double *sdev = wsp<double>(ws, *p, WB_STATS);
    launch_fill_f64(s, sdev, 0.0, 8);
    if (targets) launch_loss_reduce(s, *p, ws, nullptr, false);
    if (stats) launch_stats_out(s, sdev, wsp<uint32_t>(ws, *p, WB_PAIR_COUNT), nullptr, stats);
    HIP_TRY(ctx, hipGetLastError());
    return SWGS_OK;
}

swgs_status swgs_render_backward(swgs_context *ctx, swgs_plan *p, void *workspace, size_t ws_bytes,
                                 const float *dL_dimages, int32_t add_regulariser, const swgs_step_cfg *cfg) {
    if (!ctx || !p) return SWGS_ERR_INVALID_ARG;
    swgs_status st = check_ws(ctx, p, workspace, ws_bytes);
    if (st) return st;
    std::string why;
    if (!p->pool.grads && p->pool.num_gs > 0) return fail(ctx, SWGS_ERR_INVALID_ARG, "pool.grads is NULL");
    if (add_regulariser && (!cfg || cfg->struct_size != sizeof(swgs_step_cfg)))
        return fail(ctx, SWGS_ERR_INVALID_ARG, "cfg required (struct_size) when add_regulariser != 0");
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    hipStream_t s = ctx->stream;
    upload_consts(s, *p, ws);
    const float *g = dL_dimages ? dL_dimages : wsp<float>(ws, *p, WB_DLDC);
    seq_backward_blend(s, *p, ws, -1, g);
    launch_preprocess_backward(s, *p, ws, add_regulariser, cfg ? cfg->lambda_opacity : 0.f,
                               cfg ? cfg->lambda_scale : 0.f);
    HIP_TRY(ctx, hipGetLastError());
    return SWGS_OK;
}

static swgs_status check_cfg(swgs_context *ctx, const swgs_step_cfg *cfg) {
    if (!cfg || cfg->struct_size != sizeof(swgs_step_cfg)) return fail(ctx, SWGS_ERR_INVALID_ARG, "cfg.struct_size mismatch");
    if (cfg->reloc_n_max < 1) return fail(ctx, SWGS_ERR_INVALID_ARG, "reloc_n_max must be >= 1");
    if (cfg->relocate_period < 0) return fail(ctx, SWGS_ERR_INVALID_ARG, "relocate_period must be >= 0");
    if (!(cfg->beta1 >= 0 && cfg->beta1 < 1 && cfg->beta2 >= 0 && cfg->beta2 < 1))
        return fail(ctx, SWGS_ERR_INVALID_ARG, "betas must be in [0, 1)");
    if (!(cfg->lambda_dssim >= 0 && cfg->lambda_dssim <= 1))
        return fail(ctx, SWGS_ERR_INVALID_ARG, "lambda_dssim must be in [0, 1]");
    return SWGS_OK;
}

swgs_status swgs_step(swgs_context *ctx, swgs_plan *p, void *workspace, size_t ws_bytes, const swgs_step_cfg *cfg,
                      int64_t adam_t, uint64_t step, uint64_t seed, const float *eta) {
    if (!ctx || !p) return SWGS_ERR_INVALID_ARG;
    swgs_status st = check_ws(ctx, p, workspace, ws_bytes);
    if (st) return st;
    if ((st = check_cfg(ctx, cfg))) return st;
    std::string why;
    if (!pool_ok(&p->pool, true, why)) return fail(ctx, SWGS_ERR_INVALID_ARG, why);
    if (adam_t < 1) return fail(ctx, SWGS_ERR_INVALID_ARG, "adam_t must be >= 1");
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    hipStream_t s = ctx->stream;
    upload_consts(s, *p, ws);
    launch_gate(s, *p, ws);
    launch_set_step(s, reinterpret_cast<uint8_t *>(wsp<StepDev>(ws, *p, WB_STEP)), adam_t, step, seed);
    launch_adam_sgld(s, *p, ws, *cfg, eta);
    HIP_TRY(ctx, hipGetLastError());
    return SWGS_OK;
}

swgs_status swgs_relocate(swgs_context *ctx, swgs_plan *p, void *workspace, size_t ws_bytes, const swgs_step_cfg *cfg,
                          uint64_t step, uint64_t seed, int32_t *dst, int32_t *src, int32_t *count) {
    if (!ctx || !p) return SWGS_ERR_INVALID_ARG;
    swgs_status st = check_ws(ctx, p, workspace, ws_bytes);
    if (st) return st;
    if ((st = check_cfg(ctx, cfg))) return st;
    std::string why;
    if (!pool_ok(&p->pool, true, why)) return fail(ctx, SWGS_ERR_INVALID_ARG, why);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    hipStream_t s = ctx->stream;
    upload_consts(s, *p, ws);
    launch_gate(s, *p, ws);
    launch_set_step(s, reinterpret_cast<uint8_t *>(wsp<StepDev>(ws, *p, WB_STEP)), 1, step, seed);
    swgs_step_cfg c = *cfg;
    if (c.relocate_period == 0) c.relocate_period = 1;   // standalone call: always relocate
    launch_relocate(s, *p, ws, c, dst, src, count);
    HIP_TRY(ctx, hipGetLastError());
    return SWGS_OK;
}

// one batched step, launched in order on stream s (also the captured body)
static void seq_step_tail(hipStream_t s, swgs_plan &p, uint8_t *ws, const swgs_step_cfg &cfg) {
    {
        TimeScope t(p, s, TK_PREBWD);
        launch_preprocess_backward(s, p, ws, 1, cfg.lambda_opacity, cfg.lambda_scale);
    }
    {
        TimeScope t(p, s, TK_ADAM);
        launch_adam_sgld(s, p, ws, cfg, nullptr);
    }
    if (cfg.relocate_period > 0) {
        TimeScope t(p, s, TK_RELOC);
        launch_relocate(s, p, ws, cfg, nullptr, nullptr, nullptr);
    }
}

static void seq_ssim(hipStream_t s, swgs_plan &p, uint8_t *ws, int v_lo, int v_hi, const float *images,
                     const float *targets, float lambda) {
    TimeScope t(p, s, TK_SSIM);
    launch_ssim(s, p, ws, v_lo, v_hi, images, targets, lambda, 1.0f - lambda);
}

static void seq_window_batched(hipStream_t s, swgs_plan &p, uint8_t *ws, const swgs_step_cfg &cfg,
                               const float *targets, float *images) {
    seq_gate(s, p, ws);
    seq_forward(s, p, ws, -1, images, targets, 1.0f - cfg.lambda_dssim, cfg.lambda_dssim > 0.0f);
    launch_loss_reduce(s, p, ws, &cfg, true);
    if (cfg.lambda_dssim > 0.0f) {
        seq_ssim(s, p, ws, 0, (int)p.views.size(), images, targets, cfg.lambda_dssim);
        launch_ssim_reduce(s, p, ws, cfg.lambda_dssim);
    }
    seq_backward_blend(s, p, ws, -1, wsp<float>(ws, p, WB_DLDC));
    seq_step_tail(s, p, ws, cfg);
}

swgs_status swgs_window_step(swgs_context *ctx, swgs_plan *p, void *workspace, size_t ws_bytes,
                             const swgs_step_cfg *cfg, const float *targets, float *images, int64_t adam_t,
                             uint64_t step, uint64_t seed, double *stats) {
    if (!ctx || !p) return SWGS_ERR_INVALID_ARG;
    swgs_status st = check_ws(ctx, p, workspace, ws_bytes);
    if (st) return st;
    if ((st = check_cfg(ctx, cfg))) return st;
    std::string why;
    if (!pool_ok(&p->pool, true, why)) return fail(ctx, SWGS_ERR_INVALID_ARG, why);
    if (!targets) return fail(ctx, SWGS_ERR_INVALID_ARG, "targets must not be NULL");
    if (adam_t < 1) return fail(ctx, SWGS_ERR_INVALID_ARG, "adam_t must be >= 1");
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    hipStream_t s = ctx->stream;
    double *sdev = wsp<double>(ws, *p, WB_STATS);
    // the D-SSIM term needs the rendered images: without a caller buffer
    // they go to the workspace
    if (!images && cfg->lambda_dssim > 0.0f) images = wsp<float>(ws, *p, WB_IMAGE);
    upload_consts(s, *p, ws);

    if (cfg->mode == SWGS_MODE_GRAPH) {
        if (!s) return fail(ctx, SWGS_ERR_INVALID_ARG, "graph mode needs a non-default stream");
        const bool same = p->graph_exec && p->graph_ws == workspace && p->graph_targets == targets &&
                          p->graph_images == images && std::memcmp(&p->graph_cfg, cfg, sizeof *cfg) == 0;
        if (!same) {
            if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
            if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
            const bool was_timing = p->timing, was_counting = p->counting;
            p->timing = p->counting = false;   // no event records or counters inside a graph
            hipError_t ce = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (ce != hipSuccess) { p->timing = was_timing; p->counting = was_counting; return fail(ctx, SWGS_ERR_HIP, std::string("begin capture: ") + hipGetErrorString(ce)); }
            launch_fill_f64(s, sdev, 0.0, 8);
            seq_window_batched(s, *p, ws, *cfg, targets, images);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(s, &g);
            p->timing = was_timing;
            p->counting = was_counting;
            if (e != hipSuccess) return fail(ctx, SWGS_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            p->graph = g;
            HIP_TRY(ctx, hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0));
            p->graph_ws = workspace;
            p->graph_targets = targets;
            p->graph_images = images;
            p->graph_cfg = *cfg;
        }
        // the graph reads Adam's t, the step and the seed from the device:
        // set them from this call's arguments outside the graph, so every
        // replay takes exactly the numbers it is given
        launch_set_step(s, reinterpret_cast<uint8_t *>(wsp<StepDev>(ws, *p, WB_STEP)), adam_t, step, seed);
        HIP_TRY(ctx, hipGraphLaunch(p->graph_exec, s));
    } else if (cfg->mode == SWGS_MODE_BATCHED) {
        launch_set_step(s, reinterpret_cast<uint8_t *>(wsp<StepDev>(ws, *p, WB_STEP)), adam_t, step, seed);
        launch_fill_f64(s, sdev, 0.0, 8);
        seq_window_batched(s, *p, ws, *cfg, targets, images);
    } else {
        // plain: one launch sequence per view, reading each view's pair
        // count back to the host the way a per-frame renderer sizes its
        // buffers, then one backward preprocess and one step
        launch_set_step(s, reinterpret_cast<uint8_t *>(wsp<StepDev>(ws, *p, WB_STEP)), adam_t, step, seed);
        launch_fill_f64(s, sdev, 0.0, 8);
        seq_gate(s, *p, ws);
        uint32_t *pc = wsp<uint32_t>(ws, *p, WB_PAIR_COUNT);
        uint64_t k_total = 0;
        for (int v = 0; v < (int)p->views.size(); ++v) {
            seq_forward(s, *p, ws, v, images, targets, 1.0f - cfg->lambda_dssim, cfg->lambda_dssim > 0.0f);
            if (cfg->lambda_dssim > 0.0f) seq_ssim(s, *p, ws, v, v + 1, images, targets, cfg->lambda_dssim);
            uint32_t k = 0;
            HIP_TRY(ctx, hipMemcpyAsync(&k, pc, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(ctx, hipStreamSynchronize(s));
            if (k > (uint64_t)p->pair_cap) return fail(ctx, SWGS_ERR_CAPACITY, "pair capacity exceeded in view " + std::to_string(v));
            k_total += k;
            seq_backward_blend(s, *p, ws, v, wsp<float>(ws, *p, WB_DLDC));
        }
        // the step's pair count: the sum over the views (each view's count
        // replaced the previous one on the device)
        launch_fill_u32(s, pc, (uint32_t)std::min<uint64_t>(k_total, 0xFFFFFFFFull), 1);
        launch_loss_reduce(s, *p, ws, cfg, true);
        if (cfg->lambda_dssim > 0.0f) launch_ssim_reduce(s, *p, ws, cfg->lambda_dssim);
        seq_step_tail(s, *p, ws, *cfg);
    }
    if (stats)
        launch_stats_out(s, sdev, wsp<uint32_t>(ws, *p, WB_PAIR_COUNT),
                         wsp<uint32_t>(ws, *p, WB_ACTIVE_COUNT) + p->groups.size(), stats);
    HIP_TRY(ctx, hipGetLastError());
    return SWGS_OK;
}

swgs_status swgs_plan_set_timing(swgs_context *ctx, swgs_plan *p, void *workspace, size_t ws_bytes, int32_t flags) {
    if (!ctx || !p) return SWGS_ERR_INVALID_ARG;
    if (flags & ~(SWGS_TIMING_EVENTS | SWGS_TIMING_COUNT)) return fail(ctx, SWGS_ERR_INVALID_ARG, "unknown timing flags");
    swgs_status st = check_ws(ctx, p, workspace, ws_bytes);
    if (st) return st;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    p->timing = (flags & SWGS_TIMING_EVENTS) != 0;
    p->counting = (flags & SWGS_TIMING_COUNT) != 0;
    for (int k = 0; k < TK_N; ++k) p->ev_used[k] = 0;
    launch_fill_u32(ctx->stream, reinterpret_cast<uint32_t *>(wsp<unsigned long long>(static_cast<uint8_t *>(workspace), *p, WB_COUNTERS)), 0, 2 * 1024);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return SWGS_OK;
}

swgs_status swgs_plan_timing(swgs_context *ctx, swgs_plan *p, void *workspace, size_t ws_bytes, double *ms,
                             int64_t *launches, uint64_t *evals) {
    if (!ctx || !p || !ms || !launches) return SWGS_ERR_INVALID_ARG;
    swgs_status st = check_ws(ctx, p, workspace, ws_bytes);
    if (st) return st;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < TK_N; ++k) {
        double tot = 0.0;
        const size_t n = p->ev_used[k] / 2;
        for (size_t i = 0; i < n; ++i) {
            float m = 0.0f;
            HIP_TRY(ctx, hipEventElapsedTime(&m, p->ev[k][2 * i], p->ev[k][2 * i + 1]));
            tot += m;
        }
        ms[k] = tot;
        launches[k] = (int64_t)n;
        p->ev_used[k] = 0;
    }
    if (evals) {
        std::vector<uint64_t> c(256 * 4);
        HIP_TRY(ctx, hipMemcpy(c.data(), wsp<unsigned long long>(static_cast<uint8_t *>(workspace), *p, WB_COUNTERS),
                               c.size() * 8, hipMemcpyDeviceToHost));
        evals[0] = evals[1] = evals[2] = 0;
        for (int i = 0; i < 256; ++i)
            for (int k = 0; k < 3; ++k) evals[k] += c[4 * i + k];
    }
    launch_fill_u32(ctx->stream, reinterpret_cast<uint32_t *>(wsp<unsigned long long>(static_cast<uint8_t *>(workspace), *p, WB_COUNTERS)), 0, 2 * 1024);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return SWGS_OK;
}

size_t swgs_record_bytes(int64_t count, int32_t sh_degree) {
    if (count < 0 || sh_degree < 0 || sh_degree > 3) return 0;
    return 32 + (size_t)count * (16 + 4 * (size_t)rows_for(sh_degree));
}

swgs_status swgs_mature(swgs_context *ctx, const swgs_pool *pool, int32_t st, void *record, size_t capacity,
                        int64_t *count_out, size_t *bytes_out) {
    if (!ctx) return SWGS_ERR_INVALID_ARG;
    std::string why;
    if (!pool_ok(pool, false, why)) return fail(ctx, SWGS_ERR_INVALID_ARG, why);
    if (pool->n_slots < 2 * pool->num_gs) return fail(ctx, SWGS_ERR_INVALID_ARG, "mature needs n_slots >= 2 num_gs");
    if (!record) return fail(ctx, SWGS_ERR_INVALID_ARG, "record is NULL");
    const int n = pool->num_gs;
    void *scr = nullptr;
    const size_t words = mature_scratch_words((size_t)n);
    HIP_TRY(ctx, ctx_scratch(ctx, words * 4, &scr));
    uint32_t *sc = static_cast<uint32_t *>(scr);
    uint32_t *d_count = sc + words - 2;
    // the count comes first (from start[] on the host): the record must be
    // known to fit before anything is written
    hipStream_t s = ctx->stream;
    const int F = rows_for(pool->sh_degree);
    swgs_pool q = *pool;
    uint32_t cnt = 0;
    {
        std::vector<int32_t> hs(n);
        HIP_TRY(ctx, hipMemcpyAsync(hs.data(), pool->start, 4 * (size_t)n, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        for (int i = 0; i < n; ++i) cnt += hs[i] < st ? 1u : 0u;
    }
    const size_t need = swgs_record_bytes(cnt, pool->sh_degree);
    if (capacity < need) return fail(ctx, SWGS_ERR_INVALID_ARG, "record capacity " + std::to_string(capacity) + " < " + std::to_string(need));
    launch_mature(s, q, F, st, static_cast<uint8_t *>(record), sc, d_count);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (count_out) *count_out = cnt;
    if (bytes_out) *bytes_out = need;
    return SWGS_OK;
}

swgs_status swgs_mature_noalloc(swgs_context *ctx, const swgs_pool *pool, int32_t st, void *record,
                                size_t capacity, int64_t *count_out, size_t *bytes_out) {
    if (!ctx) return SWGS_ERR_INVALID_ARG;
    std::string why;
    if (!pool_ok(pool, false, why)) return fail(ctx, SWGS_ERR_INVALID_ARG, why);
    if (pool->n_slots < 2 * pool->num_gs) return fail(ctx, SWGS_ERR_INVALID_ARG, "mature needs n_slots >= 2 num_gs");
    if (!record) return fail(ctx, SWGS_ERR_INVALID_ARG, "record is NULL");
    const int n = pool->num_gs;
    const size_t words = mature_scratch_words((size_t)n);
    if (words > kNoAllocWords)
        return fail(ctx, SWGS_ERR_CAPACITY, "num_gs " + std::to_string(n) + " needs " + std::to_string(4 * words) +
                                                " bytes of scratch; the allocation-free call holds " +
                                                std::to_string(4 * kNoAllocWords) + " (num_gs <= " +
                                                std::to_string(swgs_mature_noalloc_max_gs()) + ")");
    uint32_t *sc = static_cast<uint32_t *>(ctx->device >= 0 && ctx->device < kMaxDevices ? g_noalloc_ptr[ctx->device] : nullptr);
    if (!sc) return fail(ctx, SWGS_ERR_HIP, "no scratch address for this device");
    uint32_t *flag = sc;
    uint32_t *pos = sc + n + 1;
    uint32_t *d_count = sc + words - 2;
    hipStream_t s = ctx->stream;
    const int F = rows_for(pool->sh_degree);
    // the count first, on the device (flags and their scan; every word these
    // kernels read is written earlier in the same call): the record must be
    // known to fit before anything is written
    launch_mature_count(s, *pool, st, flag, pos, d_count);
    uint32_t cnt = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&cnt, d_count, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const size_t need = swgs_record_bytes(cnt, pool->sh_degree);
    if (capacity < need) return fail(ctx, SWGS_ERR_INVALID_ARG, "record capacity " + std::to_string(capacity) + " < " + std::to_string(need));
    launch_mature_pack(s, *pool, F, st, static_cast<uint8_t *>(record), flag, pos, d_count);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (count_out) *count_out = cnt;
    if (bytes_out) *bytes_out = need;
    return SWGS_OK;
}

int64_t swgs_mature_noalloc_max_gs(void) {
    // largest n with 2 (n + 1) + n / 4096 + 8 <= kNoAllocWords
    int64_t lo = 0, hi = (int64_t)kNoAllocWords;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (mature_scratch_words((size_t)mid) <= kNoAllocWords) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// version-2 (compact) records: header int32[16], see swgs_encode_update
static swgs_status apply_update_v2(swgs_context *ctx, const swgs_pool *pool, const void *record, size_t record_bytes,
                                   int64_t slot_base, int64_t *count_out) {
    hipStream_t s = ctx->stream;
    if (record_bytes < 64) return fail(ctx, SWGS_ERR_INVALID_ARG, "record shorter than its 64-byte header");
    int32_t h[16];
    HIP_TRY(ctx, hipMemcpyAsync(h, record, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (h[3] < 0 || h[4] < 0 || h[4] > h[3]) return fail(ctx, SWGS_ERR_INVALID_ARG, "bad entry counts in the record");
    if (h[5] != SWGS_ENC_FP32 && h[5] != SWGS_ENC_Q) return fail(ctx, SWGS_ERR_INVALID_ARG, "unknown record encoding");
    if (h[7] & ~3) return fail(ctx, SWGS_ERR_INVALID_ARG, "unknown record flags");
    if (!(h[7] & 2) && h[4] != h[3]) return fail(ctx, SWGS_ERR_INVALID_ARG, "entries dropped without a keep mask");
    size_t need = 0;
    decode_layout(h, &need);
    if (record_bytes < need) return fail(ctx, SWGS_ERR_INVALID_ARG, "record_bytes smaller than the record's entries");
    const uint32_t n = (uint32_t)h[3];
    if (slot_base >= 0 && slot_base + (int64_t)n > (int64_t)pool->n_slots)
        return fail(ctx, SWGS_ERR_INVALID_ARG, "slot_base + count exceeds n_slots");
    const uint32_t words = (n + 31) / 32;
    void *scr = nullptr;
    HIP_TRY(ctx, ctx_scratch(ctx, 4 * ((size_t)words + words / 4096 + 64), &scr));
    uint32_t *sc = static_cast<uint32_t *>(scr);
    uint32_t *bad = sc;
    launch_fill_u32(s, bad, 0, 1);
    launch_decode(s, *pool, rows_for(pool->sh_degree), static_cast<const uint8_t *>(record), h, slot_base, sc + 8, bad);
    uint32_t nbad = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&nbad, bad, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (count_out) *count_out = n;
    if (nbad) return fail(ctx, SWGS_ERR_INVALID_ARG, std::to_string(nbad) + " record entries name slots outside the pool");
    return SWGS_OK;
}

swgs_status swgs_encode_update(swgs_context *ctx, const void *record, size_t record_bytes, int32_t enc, int64_t keep,
                               void *out, size_t capacity, size_t *bytes_out) {
    if (!ctx) return SWGS_ERR_INVALID_ARG;
    if (!record || record_bytes < 32) return fail(ctx, SWGS_ERR_INVALID_ARG, "record is NULL or shorter than its header");
    if (enc != SWGS_ENC_FP32 && enc != SWGS_ENC_Q) return fail(ctx, SWGS_ERR_INVALID_ARG, "unknown encoding");
    hipStream_t s = ctx->stream;
    int32_t h[8];
    HIP_TRY(ctx, hipMemcpyAsync(h, record, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (h[0] != 0x53475753 || h[1] != 1) return fail(ctx, SWGS_ERR_INVALID_ARG, "not a version-1 update record");
    if (h[3] < 0) return fail(ctx, SWGS_ERR_INVALID_ARG, "negative entry count in the record");
    if (h[4] < 0 || h[4] > 3 || h[5] != rows_for(h[4])) return fail(ctx, SWGS_ERR_INVALID_ARG, "bad SH degree / row count");
    const uint32_t n = (uint32_t)h[3];
    if (record_bytes < swgs_record_bytes(n, h[4])) return fail(ctx, SWGS_ERR_INVALID_ARG, "record_bytes smaller than the record's entries");
    const uint32_t kept = keep < 0 || keep >= (int64_t)n ? n : (uint32_t)keep;
    void *scr = nullptr;
    HIP_TRY(ctx, ctx_scratch(ctx, 4 * encode_scratch_words(n), &scr));
    uint32_t *sc = static_cast<uint32_t *>(scr);
    const uint8_t *src = static_cast<const uint8_t *>(record);
    launch_encode_uniform(s, src, n, sc);
    uint32_t nonuniform = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&nonuniform, sc, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const bool uniform = nonuniform == 0;
    const size_t need = encoded_bytes(n, kept, enc, uniform, kept < n);
    if (bytes_out) *bytes_out = need;
    if (!out) return SWGS_OK;   // size query
    if (capacity < need) return fail(ctx, SWGS_ERR_INVALID_ARG, "capacity " + std::to_string(capacity) + " < " + std::to_string(need));
    int32_t head[16] = {0x53475753, 2, h[2], (int32_t)n, (int32_t)kept, enc, h[6], (uniform ? 0 : 1) | (kept < n ? 2 : 0),
                        0, 0, 0, 0, h[4], 0, 0, 0};
    if (uniform && n) {
        int32_t first[4];   // slot, birth, start, expire of entry 0
        for (int i = 0; i < 4; ++i)
            HIP_TRY(ctx, hipMemcpyAsync(&first[i], src + 32 + 4 * (size_t)n * i, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        for (int i = 0; i < 4; ++i) head[8 + i] = first[i];
    }
    launch_encode(s, src, n, h[5], enc, kept, uniform, head, static_cast<uint8_t *>(out), sc + 8);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(s));   // the header is copied from this frame
    return SWGS_OK;
}

swgs_status swgs_apply_update(swgs_context *ctx, const swgs_pool *pool, const void *record, size_t record_bytes,
                              int64_t slot_base, int64_t *count_out) {
    if (!ctx) return SWGS_ERR_INVALID_ARG;
    std::string why;
    if (!pool_ok(pool, false, why)) return fail(ctx, SWGS_ERR_INVALID_ARG, why);
    if (!record || record_bytes < 32) return fail(ctx, SWGS_ERR_INVALID_ARG, "record is NULL or shorter than its header");
    hipStream_t s = ctx->stream;
    int32_t h[8];
    HIP_TRY(ctx, hipMemcpyAsync(h, record, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (h[0] == 0x53475753 && h[1] == 2) return apply_update_v2(ctx, pool, record, record_bytes, slot_base, count_out);
    if (h[0] != 0x53475753 || h[1] != 1) return fail(ctx, SWGS_ERR_INVALID_ARG, "not a version-1 or version-2 update record");
    if (h[3] < 0) return fail(ctx, SWGS_ERR_INVALID_ARG, "negative entry count in the record");
    if (h[4] != pool->sh_degree || h[5] != rows_for(pool->sh_degree))
        return fail(ctx, SWGS_ERR_INVALID_ARG, "record SH degree " + std::to_string(h[4]) + " differs from the pool's");
    const uint32_t n = (uint32_t)h[3];
    if (record_bytes < swgs_record_bytes(n, pool->sh_degree))
        return fail(ctx, SWGS_ERR_INVALID_ARG, "record_bytes smaller than the record's entries");
    if (slot_base >= 0 && slot_base + (int64_t)n > (int64_t)pool->n_slots)
        return fail(ctx, SWGS_ERR_INVALID_ARG, "slot_base + count exceeds n_slots");
    void *scr = nullptr;
    HIP_TRY(ctx, ctx_scratch(ctx, 256, &scr));
    uint32_t *bad = static_cast<uint32_t *>(scr);
    launch_fill_u32(s, bad, 0, 1);
    launch_apply_update(s, *pool, rows_for(pool->sh_degree), static_cast<const uint8_t *>(record), n, slot_base, bad);
    uint32_t nbad = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&nbad, bad, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (count_out) *count_out = n;
    if (nbad) return fail(ctx, SWGS_ERR_INVALID_ARG, std::to_string(nbad) + " record entries name slots outside the pool");
    return SWGS_OK;
}

}  // extern "C"

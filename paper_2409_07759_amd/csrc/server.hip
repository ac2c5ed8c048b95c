// Render server of libswgs.so (declared in include/swgs.h): serving side of
// Sec. 4.3 with every per-frame update resident.  Host runtime only; the
// device work is the forward launch sequence of the plans (preprocess, depth
// sort, binning, tile sort, blend) on a batch of mixed-resolution views.
//
//  - Live lists: built once per frame at creation, held at the head of the
//    caller's arena; a batch's groups point into them, so batches run no
//    gating.
//  - Memory budget: the rest of the arena, handed out first-fit in 256-byte
//    granules with coalescing on release.
//  - Admission: FIFO; requests join the batch of a free lane while the exact
//    workspace of the batch (layout of the plan it becomes, plus its images)
//    fits the largest free block.
//  - Lanes: one stream, one completion event and one pinned staging buffer
//    each; a lane's batch is launched in one submission and retired when its
//    event has completed.  Pair overflow (capacity from an estimate) is
//    detected from the pair count read back with the batch and the batch is
//    rendered again with the exact count.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <numeric>
#include <thread>

#include "swgs_internal.h"

using namespace swgs;

namespace {

using Clock = std::chrono::steady_clock;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing; offsets and sizes are
// multiples of 256 bytes.
class Budget {
  public:
    void reset(size_t size) {
        free_.clear();
        size_ = size & ~(size_t)255;
        if (size_) free_[0] = size_;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align256(std::max<size_t>(bytes, 256));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, o = it->first + bytes;
            free_.erase(it);
            if (rest) free_[o] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(std::max<size_t>(bytes, 256));
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t m = 0;
        for (auto &f : free_) m = std::max(m, f.second);
        return m;
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    void reset_peak() { peak_ = used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

enum LaneState { LANE_IDLE = 0, LANE_RUNNING, LANE_REDO };

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint8_t *pinned = nullptr;       // constant block, then 16 bytes of pair-count readback
    size_t pinned_bytes = 0;
    swgs_plan plan;
    std::vector<swgs_request *> reqs;
    size_t off = 0, bytes = 0;       // the batch's block in the budget
    size_t img_off = 0;              // its image buffer, inside the block
    int64_t batch = -1;
    LaneState state = LANE_IDLE;
    uint32_t *readback() { return reinterpret_cast<uint32_t *>(pinned + pinned_bytes - 16); }
};

// Dimensions of a candidate batch.
struct BatchDims {
    size_t V = 0, G = 0, R = 0, T = 0, P = 0;
};

}  // namespace

struct swgs_server {
    swgs_context *ctx = nullptr;
    swgs_pool pool{};
    swgs_server_opts o{};
    int tile_w = 16, tile_h = 16, lds_batch = 256;
    uint8_t *arena = nullptr;
    size_t arena_bytes = 0, resident = 0;
    uint32_t *lists = nullptr;
    std::vector<uint32_t> live, list_base;   // per frame
    Budget budget;
    std::vector<std::unique_ptr<Lane>> lanes;
    std::deque<swgs_request *> queue;
    double ratio = 4.0;                      // pairs-per-record estimate (largest seen x 1.15)
    Clock::time_point origin;
    int64_t next_batch = 0, pending = 0, batched_reqs = 0;
    swgs_serve_stats st{};
    double first_arrival = 0.0, last_ready = 0.0;
    bool any_ready = false, any_arrival = false;

    double now() const { return std::chrono::duration<double>(Clock::now() - origin).count(); }
};

namespace {

swgs_status sfail(swgs_server *s, swgs_status code, const std::string &msg) {
    if (s && s->ctx) s->ctx->err = msg;
    return code;
}

size_t tiles_of(const swgs_server *s, const swgs_view &w) {
    return (size_t)((w.width + s->tile_w - 1) / s->tile_w) * (size_t)((w.height + s->tile_h - 1) / s->tile_h);
}

size_t cap_for(const swgs_server *s, size_t R) {
    const double c = std::ceil(s->ratio * (double)R);
    return std::max<size_t>(1024, (size_t)std::min(c, 4.0e9));
}

// bytes of the block a batch needs: its workspace plus its images
size_t batch_bytes(const swgs_server *s, const BatchDims &d, size_t cap, size_t *img_off) {
    LayoutDims ld;
    ld.V = d.V;
    ld.G = d.G;
    ld.R = d.R;
    ld.T = d.T;
    ld.P = d.P;
    ld.cap = cap;
    ld.S = (size_t)s->pool.n_slots;
    ld.forward_only = true;
    Layout lay;
    size_t cb = 0;
    compute_layout(ld, lay, cb);
    const size_t ws = align256(lay.total);
    if (img_off) *img_off = ws;
    return ws + align256(3 * d.P * 4);
}

void finish_request(swgs_server *s, swgs_request *r, int32_t status, double t) {
    r->status = status;
    r->ready = t;
    --s->pending;
    if (status == SWGS_OK) {
        ++s->st.completed;
        if (!s->any_ready || t > s->last_ready) s->last_ready = t;
        s->any_ready = true;
    } else {
        ++s->st.failed;
    }
}

void fail_lane(swgs_server *s, Lane &L, int32_t status) {
    const double t = s->now();
    for (auto *r : L.reqs) finish_request(s, r, status, t);
    L.reqs.clear();
    L.state = LANE_IDLE;
}

// Build the lane's plan for its requests with pair capacity cap, take its
// block from the budget (must fit) and launch it.  Returns a HIP error
// string or "".
std::string launch_lane(swgs_server *s, Lane &L, size_t cap) {
    swgs_plan &p = L.plan;
    const int V = (int)L.reqs.size();
    std::vector<swgs_view> views(V);
    std::vector<int32_t> frames;
    std::vector<int> vgroup(V);
    for (int v = 0; v < V; ++v) {
        views[v] = L.reqs[v]->view;
        auto it = std::find(frames.begin(), frames.end(), views[v].frame);
        if (it == frames.end()) {
            vgroup[v] = (int)frames.size();
            frames.push_back(views[v].frame);
        } else {
            vgroup[v] = (int)(it - frames.begin());
        }
    }
    std::vector<uint32_t> live(frames.size());
    for (size_t g = 0; g < frames.size(); ++g) live[g] = s->live[frames[g]];
    p.pool = s->pool;
    p.sh_degree = s->pool.sh_degree;
    p.F = rows_for(s->pool.sh_degree);
    p.tile_w = s->tile_w;
    p.tile_h = s->tile_h;
    p.lds_batch = s->lds_batch;
    p.pair_cap = (int64_t)cap;
    p.forward_only = true;
    p.timing = false;
    p.counting = false;
    std::string err = plan_geometry(p, views.data(), V, frames, vgroup, live, 0);
    if (!err.empty()) return err;
    for (size_t g = 0; g < frames.size(); ++g) p.groups[g].list_base = s->list_base[frames[g]];
    p.ext[WB_ACTIVE_LIST] = reinterpret_cast<uint8_t *>(s->lists);
    if (p.consts_bytes + 16 > L.pinned_bytes) return "constant block larger than the lane's staging buffer";
    p.consts_host = L.pinned;
    fill_consts(p);
    p.consts_host = nullptr;   // owned by the lane, never freed through the plan

    BatchDims d;
    d.V = (size_t)V;
    d.G = frames.size();
    d.R = (size_t)p.R;
    d.T = (size_t)p.T;
    d.P = (size_t)p.P;
    size_t img_off = 0;
    const size_t bytes = batch_bytes(s, d, cap, &img_off);
    if (align256(p.lay.total) != img_off) return "internal: batch layout mismatch";
    size_t off = 0;
    if (!s->budget.alloc(bytes, &off)) return "internal: batch block does not fit";
    L.off = off;
    L.bytes = bytes;
    L.img_off = img_off;
    uint8_t *ws = s->arena + s->resident + off;
    float *images = reinterpret_cast<float *>(ws + img_off);
    hipStream_t st = L.stream;
    (void)hipMemcpyAsync(ws + p.lay.off[WB_VIEWS], L.pinned, p.consts_bytes, hipMemcpyHostToDevice, st);
    seq_forward_all(st, p, ws, images, nullptr);
    for (int v = 0; v < V; ++v) {
        swgs_request *r = L.reqs[v];
        if (!r->image) continue;
        const size_t n = 3 * (size_t)views[v].width * (size_t)views[v].height;
        (void)hipMemcpyAsync(r->image, images + 3 * (size_t)p.vdev[v].pix_base, n * 4, hipMemcpyDeviceToDevice, st);
    }
    (void)hipMemcpyAsync(L.readback(), wsp<uint32_t>(ws, p, WB_PAIR_COUNT), 8, hipMemcpyDeviceToHost, st);
    (void)hipEventRecord(L.done, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        s->budget.release(L.off, L.bytes);
        return std::string("launch: ") + hipGetErrorString(e);
    }
    L.state = LANE_RUNNING;
    return std::string();
}

bool any_running(const swgs_server *s) {
    for (auto &L : s->lanes)
        if (L->state == LANE_RUNNING) return true;
    return false;
}

// The lane's batch was too small for its pairs: try to relaunch with the
// exact count.
swgs_status redo_lane(swgs_server *s, Lane &L) {
    const uint32_t K = L.readback()[0];
    BatchDims d;
    d.V = L.plan.views.size();
    d.G = L.plan.groups.size();
    d.R = (size_t)L.plan.R;
    d.T = (size_t)L.plan.T;
    d.P = (size_t)L.plan.P;
    const size_t cap = std::max<size_t>(K, 1);
    const size_t need = batch_bytes(s, d, cap, nullptr);
    if (need > s->budget.largest()) {
        if (!any_running(s)) {
            s->ctx->err = "a batch's exact pair buffers do not fit the memory budget";
            fail_lane(s, L, SWGS_ERR_CAPACITY);
            return SWGS_OK;
        }
        L.state = LANE_REDO;
        return SWGS_OK;
    }
    std::string e = launch_lane(s, L, cap);
    if (!e.empty()) {
        s->ctx->err = e;
        fail_lane(s, L, SWGS_ERR_HIP);
        return SWGS_ERR_HIP;
    }
    return SWGS_OK;
}

// Retire a lane whose event completed.
swgs_status retire_lane(swgs_server *s, Lane &L) {
    const uint32_t K = L.readback()[0], overflow = L.readback()[1];
    s->budget.release(L.off, L.bytes);
    const double R = (double)L.plan.R;
    if (overflow) {
        ++s->st.redone;
        if (R > 0) s->ratio = std::max(s->ratio, 1.15 * (double)K / R);
        return redo_lane(s, L);
    }
    if (R > 0) s->ratio = std::max(s->ratio, 1.15 * (double)K / R);
    const double t = s->now();
    for (auto *r : L.reqs) {
        r->batch = (int32_t)L.batch;
        finish_request(s, r, SWGS_OK, t);
    }
    L.reqs.clear();
    L.state = LANE_IDLE;
    return SWGS_OK;
}

// Take requests from the head of the queue into lane L while they fit.
swgs_status admit(swgs_server *s, Lane &L) {
    while (!s->queue.empty()) {
        const size_t avail = s->budget.largest();
        BatchDims d;
        std::vector<int32_t> frames;
        std::vector<swgs_request *> take;
        for (auto *r : s->queue) {
            if ((int)take.size() >= s->o.max_batch) break;
            const swgs_view &w = r->view;
            const size_t px = (size_t)w.width * (size_t)w.height;
            if (s->o.max_batch_pixels > 0 && !take.empty() && d.P + px > (size_t)s->o.max_batch_pixels) break;
            BatchDims e = d;
            const bool newf = std::find(frames.begin(), frames.end(), w.frame) == frames.end();
            e.V += 1;
            e.G += newf ? 1 : 0;
            e.R += s->live[w.frame];
            e.T += tiles_of(s, w);
            e.P += px;
            if (e.R >= 0xFFFFFFF0ull || e.T >= 0xFFFFFFF0ull) break;
            if (batch_bytes(s, e, cap_for(s, e.R), nullptr) > avail) break;
            d = e;
            if (newf) frames.push_back(w.frame);
            take.push_back(r);
        }
        if (take.empty()) {
            // the head does not fit now; if nothing in flight can free
            // memory it never will
            if (any_running(s)) return SWGS_OK;
            for (auto &M : s->lanes)
                if (M->state == LANE_REDO) return SWGS_OK;
            swgs_request *r = s->queue.front();
            s->queue.pop_front();
            s->ctx->err = "request does not fit the memory budget";
            finish_request(s, r, SWGS_ERR_WORKSPACE_TOO_SMALL, s->now());
            continue;
        }
        for (size_t i = 0; i < take.size(); ++i) s->queue.pop_front();
        L.reqs = std::move(take);
        L.batch = s->next_batch++;
        ++s->st.batches;
        s->batched_reqs += (int64_t)L.reqs.size();
        std::string e = launch_lane(s, L, cap_for(s, d.R));
        if (!e.empty()) {
            s->ctx->err = e;
            fail_lane(s, L, SWGS_ERR_HIP);
            return SWGS_ERR_HIP;
        }
        return SWGS_OK;
    }
    return SWGS_OK;
}

swgs_status progress_once(swgs_server *s) {
    swgs_status rc = SWGS_OK;
    for (auto &L : s->lanes) {
        if (L->state != LANE_RUNNING) continue;
        hipError_t q = hipEventQuery(L->done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
            s->budget.release(L->off, L->bytes);
            s->ctx->err = std::string("batch failed: ") + hipGetErrorString(q);
            fail_lane(s, *L, SWGS_ERR_HIP);
            rc = SWGS_ERR_HIP;
            continue;
        }
        swgs_status r = retire_lane(s, *L);
        if (r) rc = r;
    }
    for (auto &L : s->lanes) {
        if (L->state != LANE_REDO) continue;
        swgs_status r = redo_lane(s, *L);
        if (r) rc = r;
    }
    for (auto &L : s->lanes) {
        if (L->state != LANE_IDLE || s->queue.empty()) continue;
        swgs_status r = admit(s, *L);
        if (r) rc = r;
    }
    return rc;
}

bool view_ok(const swgs_server *s, const swgs_view &w) {
    return w.frame >= 0 && w.frame < s->o.n_frames && w.width > 0 && w.height > 0 && w.width <= 16384 * 8 &&
           w.height <= 16384 * 8 && (int64_t)w.width * w.height <= (int64_t)INT32_MAX && w.fx > 0 && w.fy > 0;
}

void enqueue(swgs_server *s, swgs_request *r) {
    if (!s->any_arrival || r->arrival < s->first_arrival) s->first_arrival = r->arrival;
    s->any_arrival = true;
    r->status = -1;
    r->ready = 0.0;
    r->batch = -1;
    ++s->pending;
    if (!view_ok(s, r->view)) {
        finish_request(s, r, SWGS_ERR_INVALID_ARG, s->now());
        return;
    }
    s->queue.push_back(r);
}

void reset_stats(swgs_server *s) {
    std::memset(&s->st, 0, sizeof s->st);
    s->st.struct_size = sizeof s->st;
    s->batched_reqs = 0;
    s->any_ready = s->any_arrival = false;
    s->first_arrival = s->last_ready = 0.0;
    s->budget.reset_peak();
}

void fill_stats(const swgs_server *s, swgs_serve_stats *out) {
    *out = s->st;
    out->struct_size = sizeof *out;
    out->wall_s = s->any_ready ? s->last_ready - s->first_arrival : 0.0;
    out->mean_batch = s->st.batches ? (double)s->batched_reqs / (double)s->st.batches : 0.0;
    out->peak_bytes = s->budget.peak();
    out->budget_bytes = s->budget.size();
    out->resident_bytes = s->resident;
}

}  // namespace

extern "C" {

swgs_status swgs_server_create(swgs_context *ctx, const swgs_pool *pool, const swgs_server_opts *opts, void *arena,
                               size_t arena_bytes, swgs_server **out) {
    if (!ctx) return SWGS_ERR_INVALID_ARG;
    auto bad = [&](const std::string &m) {
        ctx->err = m;
        return SWGS_ERR_INVALID_ARG;
    };
    if (!out) return bad("out is NULL");
    *out = nullptr;
    if (!pool || pool->struct_size != sizeof(swgs_pool)) return bad("pool.struct_size mismatch");
    if (pool->sh_degree < 0 || pool->sh_degree > kMaxShDegree) return bad("sh_degree must be 0..3");
    if (pool->n_slots < 1) return bad("n_slots must be >= 1");
    if (!pool->params || !pool->start || !pool->expire) return bad("params/start/expire must not be NULL");
    if (!opts || opts->struct_size != sizeof(swgs_server_opts)) return bad("opts.struct_size mismatch");
    if (opts->n_frames < 1) return bad("n_frames must be >= 1");
    if (opts->lanes < 1 || opts->lanes > 4) return bad("lanes must be 1..4");
    if (opts->max_batch < 1 || opts->max_batch > 1024) return bad("max_batch must be 1..1024");
    if (opts->max_batch_pixels < 0) return bad("max_batch_pixels must be >= 0");
    int tw = 16, th = 16, lb = 256;
    std::string why = tile_opts(opts->tile_w, opts->tile_h, opts->lds_batch, &tw, &th, &lb);
    if (!why.empty()) {
        ctx->err = why;
        return SWGS_ERR_UNSUPPORTED;
    }
    if (!arena || reinterpret_cast<uintptr_t>(arena) % 256) return bad("arena must be non-NULL and 256-byte aligned");

    auto s = std::unique_ptr<swgs_server>(new (std::nothrow) swgs_server);
    if (!s) {
        ctx->err = "out of host memory";
        return SWGS_ERR_HIP;
    }
    s->ctx = ctx;
    s->pool = *pool;
    s->o = *opts;
    s->tile_w = tw;
    s->tile_h = th;
    s->lds_batch = lb;
    s->arena = static_cast<uint8_t *>(arena);
    s->arena_bytes = arena_bytes;
    if (opts->pair_ratio > 0) s->ratio = opts->pair_ratio;

    // live counts and lists per frame, using the arena's tail as scratch
    const int F = opts->n_frames;
    const size_t words = frame_lists_scratch_words(pool->n_slots, F);
    const size_t scratch = align256(4 * (size_t)F) + align256(sizeof(GroupDev) * (size_t)F) + align256(4 * words) +
                           align256(4 * ((size_t)F + 2));
    if (arena_bytes < scratch + 256) return bad("arena too small for the live-list set-up");
    uint8_t *tail = s->arena + ((arena_bytes - scratch) & ~(size_t)255);
    int32_t *d_frames = reinterpret_cast<int32_t *>(tail);
    GroupDev *d_groups = reinterpret_cast<GroupDev *>(tail + align256(4 * (size_t)F));
    uint32_t *d_blk = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(d_groups) + align256(sizeof(GroupDev) * (size_t)F));
    uint32_t *d_counts = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(d_blk) + align256(4 * words));
    hipStream_t st = ctx->stream;
    std::vector<int32_t> frames(F);
    std::iota(frames.begin(), frames.end(), 0);
    std::vector<uint32_t> counts(F + 1, 0);
    auto hip_fail = [&](hipError_t e, const char *what) {
        ctx->err = std::string(what) + ": " + hipGetErrorString(e);
        return SWGS_ERR_HIP;
    };
    hipError_t e;
    if ((e = hipMemcpyAsync(d_frames, frames.data(), 4 * (size_t)F, hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail(e, "frame upload");
    launch_fill_u32(st, d_counts, 0, (size_t)F + 1);
    launch_count_live(st, pool->start, pool->expire, pool->n_slots, 0, d_frames, F, d_counts);
    if ((e = hipMemcpyAsync(counts.data(), d_counts, 4 * ((size_t)F + 1), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(e, "count read-back");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "live count");
    s->live.assign(counts.begin(), counts.begin() + F);
    s->list_base.resize(F);
    size_t total = 0;
    for (int f = 0; f < F; ++f) {
        s->list_base[f] = (uint32_t)total;
        total += s->live[f];
        if (total >= 0xFFFFFFF0ull) {
            ctx->err = "more than 2^32 live-list entries";
            return SWGS_ERR_UNSUPPORTED;
        }
    }
    s->resident = align256(4 * (total + 1));
    if (s->resident + scratch > arena_bytes) return bad("arena too small for the per-frame live lists");
    s->lists = reinterpret_cast<uint32_t *>(s->arena);
    std::vector<GroupDev> groups(F);
    for (int f = 0; f < F; ++f) {
        std::memset(&groups[f], 0, sizeof(GroupDev));
        groups[f].frame = f;
        groups[f].n_views = 0;
        groups[f].list_base = s->list_base[f];
        groups[f].n_live = s->live[f];
    }
    if ((e = hipMemcpyAsync(d_groups, groups.data(), sizeof(GroupDev) * (size_t)F, hipMemcpyHostToDevice, st)) !=
        hipSuccess)
        return hip_fail(e, "group upload");
    launch_frame_lists(st, pool->start, pool->expire, pool->n_slots, d_groups, F, d_blk, d_counts, s->lists);
    std::vector<uint32_t> check(F + 1, 0);
    if ((e = hipMemcpyAsync(check.data(), d_counts, 4 * ((size_t)F + 1), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(e, "list check read-back");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "live lists");
    for (int f = 0; f < F; ++f)
        if (check[f] != s->live[f]) {
            ctx->err = "lifespans changed while the server was built";
            return SWGS_ERR_INVALID_ARG;
        }
    s->budget.reset(arena_bytes - s->resident);

    // lanes: stream, event, pinned staging sized for max_batch views
    LayoutDims ld;
    ld.V = ld.G = (size_t)opts->max_batch;
    ld.forward_only = true;
    Layout lay;
    size_t consts = 0;
    compute_layout(ld, lay, consts);
    for (int l = 0; l < opts->lanes; ++l) {
        auto L = std::unique_ptr<Lane>(new (std::nothrow) Lane);
        if (!L) {
            ctx->err = "out of host memory";
            return SWGS_ERR_HIP;
        }
        L->pinned_bytes = align256(consts + 16);
        if ((e = hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&L->done, hipEventDisableTiming)) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void **>(&L->pinned), L->pinned_bytes)) != hipSuccess) {
            s->lanes.push_back(std::move(L));
            swgs_server_destroy(s.release());
            ctx->err = std::string("lane set-up: ") + hipGetErrorString(e);
            return SWGS_ERR_HIP;
        }
        std::memset(L->pinned, 0, L->pinned_bytes);
        s->lanes.push_back(std::move(L));
    }
    s->origin = Clock::now();
    reset_stats(s.get());
    *out = s.release();
    return SWGS_OK;
}

swgs_status swgs_server_destroy(swgs_server *s) {
    if (!s) return SWGS_ERR_INVALID_ARG;
    for (auto &L : s->lanes) {
        if (L->stream) (void)hipStreamSynchronize(L->stream);
        if (L->done) (void)hipEventDestroy(L->done);
        if (L->stream) (void)hipStreamDestroy(L->stream);
        if (L->pinned) (void)hipHostFree(L->pinned);
        L->plan.consts_host = nullptr;
    }
    delete s;
    return SWGS_OK;
}

swgs_status swgs_server_submit(swgs_server *s, swgs_request *reqs, int32_t n) {
    if (!s) return SWGS_ERR_INVALID_ARG;
    if (n < 0 || (n > 0 && !reqs)) return sfail(s, SWGS_ERR_INVALID_ARG, "reqs is NULL or n < 0");
    const double t = s->now();
    for (int32_t i = 0; i < n; ++i) {
        reqs[i].arrival = t;
        enqueue(s, &reqs[i]);
    }
    return SWGS_OK;
}

swgs_status swgs_server_progress(swgs_server *s, int32_t wait, int64_t *pending) {
    if (!s) return SWGS_ERR_INVALID_ARG;
    swgs_status rc = SWGS_OK;
    const int64_t before = s->pending;
    for (;;) {
        swgs_status r = progress_once(s);
        if (r) rc = r;
        if (!wait || s->pending == 0 || s->pending < before || rc) break;
        std::this_thread::yield();
    }
    if (pending) *pending = s->pending;
    return rc;
}

swgs_status swgs_server_run(swgs_server *s, swgs_request *reqs, int32_t n, int32_t realtime,
                            swgs_serve_stats *stats) {
    if (!s) return SWGS_ERR_INVALID_ARG;
    if (n < 0 || (n > 0 && !reqs)) return sfail(s, SWGS_ERR_INVALID_ARG, "reqs is NULL or n < 0");
    if (s->pending) return sfail(s, SWGS_ERR_INVALID_ARG, "requests from swgs_server_submit are still pending");
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    if (realtime) {
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return reqs[a].arrival < reqs[b].arrival; });
    } else {
        for (int32_t i = 0; i < n; ++i) reqs[i].arrival = 0.0;
    }
    reset_stats(s);
    s->origin = Clock::now();
    swgs_status rc = SWGS_OK;
    int32_t i = 0;
    for (;;) {
        const double t = s->now();
        while (i < n && (!realtime || reqs[order[i]].arrival <= t)) enqueue(s, &reqs[order[i++]]);
        swgs_status r = progress_once(s);
        if (r && !rc) rc = r;
        if (i == n && s->pending == 0) break;
        if (r == SWGS_ERR_HIP) {
            // a failed batch leaves the device in an unknown state: fail the rest
            while (i < n) enqueue(s, &reqs[order[i++]]);
            const double tf = s->now();
            while (!s->queue.empty()) {
                finish_request(s, s->queue.front(), SWGS_ERR_HIP, tf);
                s->queue.pop_front();
            }
            for (auto &L : s->lanes)
                if (L->state != LANE_IDLE) {
                    if (L->stream) (void)hipStreamSynchronize(L->stream);
                    if (L->state == LANE_RUNNING) s->budget.release(L->off, L->bytes);
                    fail_lane(s, *L, SWGS_ERR_HIP);
                }
            break;
        }
    }
    if (stats) fill_stats(s, stats);
    return rc;
}

swgs_status swgs_server_stats(const swgs_server *s, swgs_serve_stats *stats) {
    if (!s || !stats) return SWGS_ERR_INVALID_ARG;
    fill_stats(s, stats);
    return SWGS_OK;
}

}  // extern "C"

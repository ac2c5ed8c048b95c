// Client-side playback of the update stream (Algorithm 2, Sec. 4.3).
//
// The client keeps a buffer of num_gs slots; every update record carries one
// slice (the genesis record, all slots) and is due at the birth frame of its
// Gaussians.  push() is Algorithm 2's stream read: the record goes into a
// pinned host staging slot and starts its host-to-device copy on the
// player's own copy stream, so the transfer overlaps whatever the context
// stream is rendering.  advance(frame) is one tick of the update thread: each
// queued record due at `frame` (or earlier) is decoded into the buffer on the
// context stream, after its copy, without a host synchronisation; renders
// issued afterwards on the context stream see the new slice.  Slot ranges are
// checked on the host at push time, from the record itself.
#include <cstring>
#include <deque>
#include <string>
#include <vector>

#include "swgs_internal.h"

struct swgs_player {
    swgs_context *ctx = nullptr;
    swgs_pool pool{};
    int depth = 0;
    size_t slot_bytes = 0;
    uint8_t *host_ring = nullptr;   // pinned
    uint8_t *dev_ring = nullptr;
    uint32_t *scratch = nullptr;    // decode scratch (mask ranks) + bad-slot counter
    hipStream_t copy = nullptr;
    std::vector<hipEvent_t> copied, applied;
    std::vector<int> state;         // 0 free, 1 queued, 2 applied (free once `applied` completes)
    struct Event {
        int32_t target;
        int slot;
        size_t bytes;
        int32_t head[16];
        int version;
    };
    std::deque<Event> queue;
    int64_t n_applied = 0;
};

using namespace swgs;

namespace {

swgs_status pfail(swgs_context *ctx, swgs_status st, const std::string &why) {
    if (ctx) ctx->err = why;
    return st;
}

// A ring slot for the next record: free, or applied and finished.
int take_slot(swgs_player *p) {
    for (int i = 0; i < p->depth; ++i)
        if (p->state[i] == 0) return i;
    for (int i = 0; i < p->depth; ++i)
        if (p->state[i] == 2 && hipEventSynchronize(p->applied[i]) == hipSuccess) {
            p->state[i] = 0;
            return i;
        }
    return -1;
}

void release(swgs_player *p) {
    if (!p) return;
    if (p->copy) (void)hipStreamSynchronize(p->copy);
    if (p->ctx) (void)hipStreamSynchronize(p->ctx->stream);
    for (auto e : p->copied) (void)hipEventDestroy(e);
    for (auto e : p->applied) (void)hipEventDestroy(e);
    if (p->copy) (void)hipStreamDestroy(p->copy);
    if (p->host_ring) (void)hipHostFree(p->host_ring);
    if (p->dev_ring) (void)hipFree(p->dev_ring);
    if (p->scratch) (void)hipFree(p->scratch);
    delete p;
}

}  // namespace

swgs_status swgs_player_create(swgs_context *ctx, const swgs_pool *buffer, const swgs_player_opts *opts,
                               swgs_player **out) {
    if (!ctx || !out) return SWGS_ERR_INVALID_ARG;
    *out = nullptr;
    if (!buffer || !buffer->params || !buffer->start || !buffer->expire || buffer->n_slots <= 0)
        return pfail(ctx, SWGS_ERR_INVALID_ARG, "buffer needs params, start and expire");
    if (buffer->sh_degree < 0 || buffer->sh_degree > 3) return pfail(ctx, SWGS_ERR_INVALID_ARG, "SH degree must be 0..3");
    if (!opts || opts->struct_size != sizeof(swgs_player_opts)) return pfail(ctx, SWGS_ERR_INVALID_ARG, "opts.struct_size mismatch");
    if (opts->queue_depth < 1 || opts->queue_depth > 64) return pfail(ctx, SWGS_ERR_INVALID_ARG, "queue_depth must be 1..64");
    if (opts->max_record_bytes < 64) return pfail(ctx, SWGS_ERR_INVALID_ARG, "max_record_bytes must be >= 64");
    auto *p = new swgs_player;
    p->ctx = ctx;
    p->pool = *buffer;
    p->depth = opts->queue_depth;
    p->slot_bytes = (opts->max_record_bytes + 255) / 256 * 256;
    const size_t words = p->slot_bytes / 32 + p->slot_bytes / 32 / 4096 + 64;
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&p->host_ring), p->slot_bytes * p->depth, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&p->dev_ring), p->slot_bytes * p->depth);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&p->scratch), 4 * words);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking);
    p->copied.assign(p->depth, nullptr);
    p->applied.assign(p->depth, nullptr);
    p->state.assign(p->depth, 0);
    for (int i = 0; i < p->depth && e == hipSuccess; ++i) {
        e = hipEventCreateWithFlags(&p->copied[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->applied[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        release(p);
        return pfail(ctx, SWGS_ERR_HIP, std::string("player allocation: ") + hipGetErrorString(e));
    }
    *out = p;
    return SWGS_OK;
}

swgs_status swgs_player_push(swgs_player *p, const void *record, size_t bytes) {
    if (!p) return SWGS_ERR_INVALID_ARG;
    swgs_context *ctx = p->ctx;
    if (!record || bytes < 32) return pfail(ctx, SWGS_ERR_INVALID_ARG, "record is NULL or shorter than a header");
    if (bytes > p->slot_bytes) return pfail(ctx, SWGS_ERR_INVALID_ARG, "record larger than max_record_bytes");
    const uint8_t *rec = static_cast<const uint8_t *>(record);
    swgs_player::Event ev{};
    std::memcpy(ev.head, rec, bytes >= 64 ? 64 : 32);
    if (ev.head[0] != 0x53475753 || (ev.head[1] != 1 && ev.head[1] != 2))
        return pfail(ctx, SWGS_ERR_INVALID_ARG, "not an update record");
    ev.version = ev.head[1];
    const int64_t n = ev.head[3];
    if (n < 0) return pfail(ctx, SWGS_ERR_INVALID_ARG, "negative entry count");
    const int64_t S = p->pool.n_slots;
    if (ev.version == 1) {
        if (ev.head[4] != p->pool.sh_degree) return pfail(ctx, SWGS_ERR_INVALID_ARG, "record SH degree differs from the buffer's");
        if (bytes < swgs_record_bytes(n, ev.head[4])) return pfail(ctx, SWGS_ERR_INVALID_ARG, "record shorter than its entries");
        const uint32_t *slot = reinterpret_cast<const uint32_t *>(rec + 32);
        for (int64_t k = 0; k < n; ++k)
            if ((int64_t)slot[k] >= S) return pfail(ctx, SWGS_ERR_INVALID_ARG, "record slot outside the buffer");
        ev.target = n ? reinterpret_cast<const int32_t *>(rec + 32 + 4 * n)[0] : 0;
    } else {
        if (bytes < 64) return pfail(ctx, SWGS_ERR_INVALID_ARG, "record shorter than its header");
        if (ev.head[4] < 0 || ev.head[4] > n || (ev.head[7] & ~3) || (!(ev.head[7] & 2) && ev.head[4] != n) ||
            (ev.head[5] != SWGS_ENC_FP32 && ev.head[5] != SWGS_ENC_Q))
            return pfail(ctx, SWGS_ERR_INVALID_ARG, "bad compact record header");
        size_t need = 0;
        decode_layout(ev.head, &need);
        if (bytes < need) return pfail(ctx, SWGS_ERR_INVALID_ARG, "record shorter than its entries");
        if (ev.head[7] & 1) {
            const uint32_t *slot = reinterpret_cast<const uint32_t *>(rec + 64);
            for (int64_t k = 0; k < n; ++k)
                if ((int64_t)slot[k] >= S) return pfail(ctx, SWGS_ERR_INVALID_ARG, "record slot outside the buffer");
            ev.target = n ? reinterpret_cast<const int32_t *>(rec + 64 + ((4 * n + 15) / 16 * 16))[0] : 0;
        } else {
            if (n && (ev.head[8] < 0 || ev.head[8] + n > S)) return pfail(ctx, SWGS_ERR_INVALID_ARG, "record slots outside the buffer");
            ev.target = ev.head[9];
        }
    }
    const int slot = take_slot(p);
    if (slot < 0) return pfail(ctx, SWGS_ERR_CAPACITY, "update queue full: advance to apply queued records first");
    ev.slot = slot;
    ev.bytes = bytes;
    std::memcpy(p->host_ring + slot * p->slot_bytes, rec, bytes);
    hipError_t e = hipMemcpyAsync(p->dev_ring + slot * p->slot_bytes, p->host_ring + slot * p->slot_bytes, bytes,
                                  hipMemcpyHostToDevice, p->copy);
    if (e == hipSuccess) e = hipEventRecord(p->copied[slot], p->copy);
    if (e != hipSuccess) return pfail(ctx, SWGS_ERR_HIP, std::string("push: ") + hipGetErrorString(e));
    p->state[slot] = 1;
    p->queue.push_back(ev);
    return SWGS_OK;
}

swgs_status swgs_player_advance(swgs_player *p, int32_t frame, int32_t *applied) {
    if (!p) return SWGS_ERR_INVALID_ARG;
    swgs_context *ctx = p->ctx;
    hipStream_t s = ctx->stream;
    const int F = 11 + 3 * (p->pool.sh_degree + 1) * (p->pool.sh_degree + 1);
    int32_t cnt = 0;
    for (auto it = p->queue.begin(); it != p->queue.end();) {
        if (it->target > frame) {
            ++it;
            continue;
        }
        const uint8_t *rec = p->dev_ring + it->slot * p->slot_bytes;
        hipError_t e = hipStreamWaitEvent(s, p->copied[it->slot], 0);
        if (e != hipSuccess) return pfail(ctx, SWGS_ERR_HIP, std::string("advance: ") + hipGetErrorString(e));
        uint32_t *bad = p->scratch;   // slots were checked at push: the count is not read
        if (it->version == 1)
            launch_apply_update(s, p->pool, F, rec, (uint32_t)it->head[3], -1, bad);
        else
            launch_decode(s, p->pool, F, rec, it->head, -1, p->scratch + 8, bad);
        e = hipEventRecord(p->applied[it->slot], s);
        if (e != hipSuccess) return pfail(ctx, SWGS_ERR_HIP, std::string("advance: ") + hipGetErrorString(e));
        p->state[it->slot] = 2;
        ++cnt;
        it = p->queue.erase(it);
    }
    p->n_applied += cnt;
    if (applied) *applied = cnt;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return pfail(ctx, SWGS_ERR_HIP, std::string("advance: ") + hipGetErrorString(e));
    return SWGS_OK;
}

swgs_status swgs_player_queued(const swgs_player *p, int32_t *queued, int64_t *applied_total) {
    if (!p) return SWGS_ERR_INVALID_ARG;
    if (queued) *queued = (int32_t)p->queue.size();
    if (applied_total) *applied_total = p->n_applied;
    return SWGS_OK;
}

void swgs_player_destroy(swgs_player *p) { release(p); }

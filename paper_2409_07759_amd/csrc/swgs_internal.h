// Internal declarations shared by the translation units of libswgs.so.
// Nothing here is part of the public ABI (include/swgs.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/swgs.h"

namespace swgs {

// ----------------------------------------------------------------- limits
constexpr int kMaxShDegree = 3;
constexpr int kMaxRows = 11 + 3 * 16;      // F at SH degree 3
constexpr int kGateChunk = 2048;           // slots per gating block
constexpr int kSortBlocks = 1024;          // fixed grid of the radix-sort passes
constexpr int kSplatFloats = 12;           // floats per splat record
constexpr int kXcds = 8;                   // accelerator complex dies (one L2 each)

inline int rows_for(int sh_degree) { return 11 + 3 * (sh_degree + 1) * (sh_degree + 1); }

// Workgroups of a launch are dealt to the XCDs round-robin (workgroup b runs
// on XCD b mod 8), and each XCD has its own L2.  This bijection of [0, n)
// hands XCD x the contiguous range of work items [x q + min(x, r), ...),
// q = n / 8, r = n mod 8, so neighbouring tiles, which share records or
// halo rows, meet in the same L2.
__host__ __device__ inline uint32_t xcd_order(uint32_t b, uint32_t n) {
    const uint32_t x = b % kXcds, i = b / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + i;
}

// A launch over many views whose work per tile differs between views (an
// uneven window: frames with few and with many live Gaussians) would leave
// the XCDs holding the densest views' eighths busy after the others are
// done.  xcd_spread maps a position p of xcd_order's order to a work item
// so that the full chunks of kSpreadChunk consecutive items are visited in
// the order k -> (k s) mod m (m full chunks, s coprime to m, about m / 8):
// each XCD's contiguous positions then cover chunks spread over the whole
// range, and neighbouring items stay together inside a chunk.  s = 0: p
// itself.
constexpr uint32_t kSpreadChunk = 1024;
__host__ __device__ inline uint32_t xcd_spread(uint32_t p, uint32_t n, uint32_t s) {
    const uint32_t m = n / kSpreadChunk, k = p / kSpreadChunk;
    if (s == 0 || k >= m) return p;
    return (uint32_t)(((uint64_t)k * s) % m) * kSpreadChunk + p % kSpreadChunk;
}
// the multiplier xcd_spread uses for n items (0 when there are fewer than
// two full chunks per XCD)
inline uint32_t spread_multiplier(uint32_t n) {
    const uint32_t m = n / kSpreadChunk;
    if (m < 2 * kXcds) return 0;
    auto gcd = [](uint32_t a, uint32_t b) { while (b) { const uint32_t t = a % b; a = b; b = t; } return a; };
    uint32_t s = m / kXcds + 1;
    while (gcd(s, m) != 1) ++s;
    return s;
}

// A view as the kernels see it: camera in FP64 plus its place in the plan.
struct ViewDev {
    double R[9];
    double t[3];
    double fx, fy, cx, cy;
    double campos[3];          // camera centre in world coordinates
    double limx, limy;         // 1.3 * tan(half FoV) per axis
    float bg[3];
    int32_t frame;
    int32_t width, height;
    int32_t tiles_x, tiles_y;
    int32_t group;             // distinct-frame group
    uint32_t rec_base;         // first record of this view
    uint32_t tile_base;        // first global tile id of this view
    int64_t pix_base;          // first pixel of this view in the image buffers
    float inv_norm;            // 1 / (V * 3 * H * W): L1 gradient scale
    uint32_t ssim_tile_base;   // first 16x16 SSIM tile of this view
};

struct GroupDev {
    int32_t frame;
    int32_t n_views;
    int32_t view_first;        // index into the plan's group-ordered view list
    uint32_t list_base;        // first entry of this group's live list
    uint32_t n_live;           // live slots (known at plan time)
    uint32_t pad;
};

// Byte offsets of every workspace buffer.
struct Layout {
    size_t off[64];
    size_t size[64];
    size_t total = 0;
};

// What a workspace layout depends on: views, distinct frames, records,
// tiles, pixels, pair capacity, pool slots, optimisable slots, window set,
// live-list entries.
struct LayoutDims {
    size_t V = 0, G = 0, R = 0, T = 0, P = 0, cap = 0, S = 0, NG = 0, nA = 0, n_list = 0, Tssim = 0;
    bool forward_only = false;
    bool own_lists = false;    // forward only, but gating into the workspace
};

enum WsBuf {
    WB_ACTIVE_LIST = 0, WB_ACTIVE_COUNT, WB_REC_VIEW_BASE, WB_DEPTH_KEY, WB_TILE_COUNT,
    WB_RECT, WB_SPLAT, WB_PAIR_KEY, WB_PAIR_VAL, WB_PAIR_COUNT, WB_TILE_RANGE, WB_T_FINAL,
    WB_DLDC, WB_REC_GRAD,
    // internal
    WB_GATE_BLK, WB_POS_OF, WB_REC_IDX, WB_KEY_ALT, WB_IDX_ALT, WB_PAIR_KEY_ALT, WB_PAIR_VAL_ALT,
    WB_PAIR_OFFSET, WB_SORT_HIST, WB_SORT_TOTAL, WB_LAST, WB_LOSS_PART, WB_STATS, WB_STEP,
    WB_VIEWS, WB_GROUPS, WB_GROUP_VIEWS,
    WB_RELOC_W, WB_RELOC_FLAG, WB_RELOC_SRC, WB_RELOC_DST, WB_RELOC_CNT, WB_RELOC_SCAN, WB_REG_PART, WB_COUNTERS, WB_CFLAGS,
    WB_SSIM_PART, WB_SSIM_SUM, WB_IMAGE, WB_PAIR_BASE, WB_PAIR_GRAD, WB_RECT_SORTED, WB_PAIR_MASK,
    WB_ROW_OFFSET, WB_COUNT
};

}  // namespace swgs

struct swgs_context {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
};

struct swgs_plan {
    swgs_pool pool{};
    int sh_degree = 0;
    int F = 0;
    int tile_w = 16, tile_h = 16;
    int lds_batch = 256;
    int64_t pair_cap = 0;
    std::vector<swgs_view> views;                 // caller order
    std::vector<swgs::ViewDev> vdev;              // caller order
    std::vector<swgs::GroupDev> groups;           // distinct frames
    std::vector<int32_t> group_views;             // view indices ordered by group
    bool uneven = false;                          // views' live Gaussians per pixel differ by more than 25%
    uint32_t n_A = 0;                             // |A|
    uint32_t list_A_base = 0;
    int64_t R = 0, P = 0, T = 0, Tssim = 0;   // records, pixels, tiles, SSIM tiles
    int tile_key_bits = 1;
    int loss_blocks = 0;
    swgs::Layout lay;
    // graph mode
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    void *graph_ws = nullptr;
    const void *graph_targets = nullptr;
    void *graph_images = nullptr;
    swgs_step_cfg graph_cfg{};
    void *consts_host = nullptr;                  // pinned copy of the constant block
    size_t consts_bytes = 0;
    // forward-only plans (serving) carry no training buffers
    bool forward_only = false;
    // a forward-only plan that gates into its own workspace (a standalone
    // batch render) instead of reading resident lists
    bool own_lists = false;
    // buffers that live outside the workspace (absolute device pointers; a
    // null entry means "at lay.off[] in the workspace")
    uint8_t *ext[swgs::WB_COUNT] = {};
    // event timing of kernel classes and blend pair counters (off unless
    // enabled; never inside a graph)
    bool timing = false;
    bool counting = false;
    std::vector<hipEvent_t> ev[9];
    size_t ev_used[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
};

namespace swgs {

// ----------------------------------------------------------- launchers
// Gating / compaction (kernels_gate.hip)
void launch_gate(hipStream_t s, const swgs_plan &p, uint8_t *ws);
void launch_count_live(hipStream_t s, const int32_t *start, const int32_t *expire, int n_slots,
                       int num_gs, const int32_t *frames, int n_frames, uint32_t *out_counts);

// Preprocess and binning (kernels_preprocess.hip)
void launch_preprocess(hipStream_t s, const swgs_plan &p, uint8_t *ws, int view_lo, int view_hi);
void launch_pair_offsets(hipStream_t s, const swgs_plan &p, uint8_t *ws, uint32_t rec_lo, uint32_t rec_hi);
void launch_emit_pairs(hipStream_t s, const swgs_plan &p, uint8_t *ws, uint32_t rec_lo, uint32_t rec_hi);
// gradient-row layout of records [rec_lo, rec_hi) for the backward: each
// record's first row (record order) and slot base
void launch_row_offsets(hipStream_t s, const swgs_plan &p, uint8_t *ws, uint32_t rec_lo, uint32_t rec_hi);
void launch_tile_ranges(hipStream_t s, const swgs_plan &p, uint8_t *ws, uint32_t tile_lo, uint32_t tile_hi);

// Radix sort (kernels_sort.hip): stable LSD sort of (key, val) uint32 pairs,
// n given on the device (*d_n, clamped to cap) over bits [0, bits), in
// radix_passes(bits) passes of at most 8 bits.  The input is read from
// (keys_alt, vals_alt) when radix_input_in_alt(bits) (an odd pass count),
// else from (keys, vals); on return the sorted data is in (keys, vals) and
// the other pair holds scratch.  32-bit keys take 4 passes (input in keys).
// With gather_rect (tile rectangles packed as in the binning: x0 | y0 << 16,
// x1 | y1 << 16), the last pass also writes, for every sorted position i,
// rect_out[i] = gather_rect[vals[i]] and count_out[i] = its tile count.
int radix_passes(int bits);
bool radix_input_in_alt(int bits);
void radix_sort_pairs(hipStream_t s, uint32_t *keys, uint32_t *vals, uint32_t *keys_alt,
                      uint32_t *vals_alt, const uint32_t *d_n, uint32_t n_fixed, uint32_t cap,
                      int bits, uint32_t *hist, uint32_t *totals, const uint2 *gather_rect = nullptr,
                      uint2 *rect_out = nullptr, uint32_t *count_out = nullptr);
// exclusive scan (in may equal out); *total_out = sum
void exclusive_scan_u32(hipStream_t s, const uint32_t *in, uint32_t *out, uint32_t n,
                        uint32_t *total_out, uint32_t *scratch);
// exclusive scan of tile counts into first rows, also writing, per element,
// (first row - y0 w - x0, w) of its tile rect (packed as in the binning) to
// slot_base (w = the rect's width, at least 1)
void exclusive_scan_rows(hipStream_t s, const uint32_t *count, const uint2 *rect, uint32_t n, uint32_t *first,
                         uint2 *slot_base, uint32_t *scratch);

// Blend (kernels_blend.hip)
// counters (nullable): [0] pixel x list entries evaluated by the forward,
// [1] by the backward
// l1_weight scales the fused L1 term and its gradient (1 - lambda_dssim);
// without write_dldc only the loss is taken (the D-SSIM backward writes dL/dC)
void launch_blend_forward(hipStream_t s, const swgs_plan &p, uint8_t *ws, float *images,
                          const float *targets, uint32_t tile_lo, uint32_t tile_hi,
                          unsigned long long *counters, float l1_weight, bool write_dldc = true);
void launch_blend_backward(hipStream_t s, const swgs_plan &p, uint8_t *ws, const float *dLdC,
                           uint32_t tile_lo, uint32_t tile_hi, unsigned long long *counters);
// Compact update record (kernels_codec.hip)
size_t encoded_bytes(uint32_t n, uint32_t m, int enc, bool uniform, bool masked);
size_t encode_scratch_words(uint32_t n);
void launch_encode_uniform(hipStream_t s, const uint8_t *src, uint32_t n, uint32_t *flag);
void launch_encode(hipStream_t s, const uint8_t *src, uint32_t n, int F, int enc, uint32_t keep, bool uniform,
                   const int32_t header[16], uint8_t *out, uint32_t *scratch);
bool decode_layout(const int32_t h[16], size_t *need);
void launch_decode(hipStream_t s, const swgs_pool &pool, int F, const uint8_t *rec, const int32_t h[16],
                   int64_t slot_base, uint32_t *scratch, uint32_t *bad);

// record gradients [R][9] of records [rec_lo, rec_hi): the per-pair gradient
// rows the backward blend left (a record's rows consecutive, records in
// record order), summed in row order
void launch_pair_grad_reduce(hipStream_t s, const swgs_plan &p, uint8_t *ws, uint32_t rec_lo, uint32_t rec_hi);
void launch_loss_reduce(hipStream_t s, const swgs_plan &p, uint8_t *ws, const swgs_step_cfg *cfg,
                        bool with_reg);

// D-SSIM term (kernels_ssim.hip): SSIM of views [view_lo, view_hi); dL/dC of
// those views is written whole: the L1 term (weight l1_weight) plus the
// D-SSIM term; then the weighted SSIM sums are added to stats[0]
size_t ssim_tiles(int width, int height);
void launch_ssim(hipStream_t s, const swgs_plan &p, uint8_t *ws, int view_lo, int view_hi, const float *images,
                 const float *targets, float lambda, float l1_weight);
void launch_ssim_reduce(hipStream_t s, const swgs_plan &p, uint8_t *ws, float lambda);

// Backward preprocess, step, relocation, mature (kernels_step.hip)
void launch_preprocess_backward(hipStream_t s, const swgs_plan &p, uint8_t *ws, int add_reg,
                                float lambda_o, float lambda_s);
void launch_adam_sgld(hipStream_t s, const swgs_plan &p, uint8_t *ws, const swgs_step_cfg &cfg,
                      const float *eta);
void launch_relocate(hipStream_t s, const swgs_plan &p, uint8_t *ws, const swgs_step_cfg &cfg,
                     int32_t *dst_out, int32_t *src_out, int32_t *count_out);
void launch_set_step(hipStream_t s, uint8_t *ws_step, int64_t adam_t, uint64_t step, uint64_t seed);
void launch_fill_u32(hipStream_t s, uint32_t *p, uint32_t v, size_t n);
void launch_fill_f32(hipStream_t s, float *p, float v, size_t n);
void launch_fill_f64(hipStream_t s, double *p, double v, size_t n);

// stats[0..7] -> out, with out[4] = pairs, out[6] = overflow, out[7] = |A| (if nA)
void launch_stats_out(hipStream_t s, const double *stats, const uint32_t *pair_count, const uint32_t *nA,
                      double *out);

// Mature (kernels_step.hip)
void launch_mature(hipStream_t s, const swgs_pool &pool, int F, int st, uint8_t *record,
                   uint32_t *scratch, uint32_t *d_count);
void launch_mature_count(hipStream_t s, const swgs_pool &pool, int st, uint32_t *flag, uint32_t *pos,
                         uint32_t *d_count);
void launch_mature_pack(hipStream_t s, const swgs_pool &pool, int F, int st, uint8_t *record, const uint32_t *flag,
                        const uint32_t *pos, const uint32_t *d_count);

// Device step parameters (kept in the workspace so a captured graph reads
// them; each call sets them from its arguments before the replay).
struct StepDev {
    int64_t adam_t;
    uint64_t step;
    uint64_t seed;
    uint64_t pad;
};

template <typename T>
inline T *wsp(uint8_t *ws, const swgs_plan &p, int which) {
    return reinterpret_cast<T *>(p.ext[which] ? p.ext[which] : ws + p.lay.off[which]);
}

// Plan geometry shared by swgs_plan_create and the server: groups of
// distinct frames (live counts given per group), per-view records, tiles
// and pixels, the workspace layout and the pinned constant block.  Returns
// an empty string or the reason for failure.
std::string plan_geometry(swgs_plan &p, const swgs_view *views, int n_views, const std::vector<int32_t> &frames,
                          const std::vector<int> &vgroup, const std::vector<uint32_t> &live, uint32_t n_A);
// Checks a tile shape / LDS batch request (0,0 and 0 pick the defaults) and
// returns the effective values; "" or the reason it is not supported.
std::string tile_opts(int tile_w, int tile_h, int lds_batch, int *tw, int *th, int *lb);
// Workspace layout for the given dimensions (offsets, sizes, total) and the
// size of its leading constant block.
void compute_layout(const LayoutDims &d, Layout &lay, size_t &consts_bytes);
// Copy of the constant block (views, groups, group view list, record view
// bases) into p.consts_host (consts_bytes, allocated by the caller).
void fill_consts(swgs_plan &p);
// Forward of every view of a plan in one launch sequence (gating not
// included): preprocess, depth sort, pair offsets, emit, pair sort, tile
// ranges, blend.
void seq_forward_all(hipStream_t s, swgs_plan &p, uint8_t *ws, float *images, const float *targets);

// Per-frame live lists of a resident pool (serving): for groups[g] (device,
// frame and list_base set) the live slots in ascending order are written at
// lists[list_base...]; blk is scratch of (n_groups + 1) * ceil(n_slots /
// kGateChunk) uint32, totals of n_groups + 1.
void launch_frame_lists(hipStream_t s, const int32_t *start, const int32_t *expire, int n_slots,
                        const GroupDev *groups, int n_groups, uint32_t *blk, uint32_t *totals, uint32_t *lists);
inline size_t frame_lists_scratch_words(int n_slots, int n_groups) {
    return (size_t)(n_groups + 1) * (size_t)((n_slots + kGateChunk - 1) / kGateChunk) + (size_t)n_groups + 8;
}

// Scatter of a mature record into a pool (Algorithm 2's slice replacement
// when slot_base < 0, else append at slot_base + k).
void launch_apply_update(hipStream_t s, const swgs_pool &pool, int F, const uint8_t *record, uint32_t count,
                         int64_t slot_base, uint32_t *bad_slots);

}  // namespace swgs

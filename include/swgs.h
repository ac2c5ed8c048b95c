/*
 * swgs.h -- C ABI of libswgs.so, the MI355X (gfx950) hot path of SwinGS,
 * "Sliding Window Gaussian Splatting for Volumetric Video Streaming with
 * Arbitrary Length" (arXiv 2409.07759).
 *
 * The library trains and renders a pool of 3D Gaussians whose members carry
 * integer lifespans [start, expire) (Sec. 4.2): a window of (frame, camera)
 * views is rendered with the lifespan gate applied per frame (Algorithm 1's
 * two filters), differentiated (Algorithm 1's backward), stepped with Adam,
 * adaptive mean-gradient scaling (Sec. 4.5.1) and SGLD noise (Algorithm 1's
 * noise line), its dead members relocated (Sec. 3.2), and, when the window
 * advances, its oldest slice matured and emitted as a per-frame update
 * (Algorithm 1's mature, Eq. 4).
 *
 * Conventions shared by every call:
 *  - Memory: every buffer is caller-owned.  "device" pointers are HIP device
 *    memory on the context's device (PyTorch allocates them); "host" pointers
 *    are ordinary host memory.  The library owns only its opaque handles.
 *  - Streams: every call is asynchronous on the context's stream unless its
 *    comment says it synchronises.
 *  - Errors: every call returns swgs_status; nothing throws or aborts across
 *    the ABI.  The message of the last failure is swgs_last_error(ctx).
 *    Invalid arguments are detected on the host before anything is launched.
 *  - Layouts: parameters are "planar rows": a float array [F][n_slots] with
 *    F = 11 + 3 (d+1)^2 and rows 0-2 mean, 3-5 log-scale, 6-9 quaternion
 *    (w, x, y, z), 10 opacity logit, 11 + 3k + ch spherical-harmonic
 *    coefficient k of colour channel ch.  Images of a plan are concatenated
 *    view after view, each planar [3][height][width] float; pixel (x, y) has
 *    its centre at (x + 0.5, y + 0.5).
 *  - A context is used by one host thread at a time; contexts are independent.
 */
#ifndef SWGS_H
#define SWGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWGS_VERSION 1

typedef enum {
    SWGS_OK = 0,
    SWGS_ERR_INVALID_ARG = 1,          /* bad pointer, size or option */
    SWGS_ERR_UNSUPPORTED = 2,          /* e.g. SH degree > 3, tile shape */
    SWGS_ERR_WORKSPACE_TOO_SMALL = 3,  /* caller's workspace is smaller than required */
    SWGS_ERR_CAPACITY = 4,             /* tile-pair capacity exceeded (found at a sync) */
    SWGS_ERR_HIP = 5                   /* a HIP runtime call failed */
} swgs_status;

typedef struct swgs_context swgs_context;
typedef struct swgs_plan swgs_plan;

/* Library version (SWGS_VERSION). */
int swgs_version(void);

/* Bind device `device` and the caller's HIP stream (hipStream_t, may be
 * NULL for the default stream; PyTorch: torch.cuda.current_stream().cuda_stream).
 * *out receives a new context. */
swgs_status swgs_context_create(int device, void *hip_stream, swgs_context **out);
swgs_status swgs_context_set_stream(swgs_context *ctx, void *hip_stream);
swgs_status swgs_context_destroy(swgs_context *ctx);
/* Message of the last failure on ctx ("" if none); valid until the next call. */
const char *swgs_last_error(const swgs_context *ctx);

/* ------------------------------------------------------------------ pool
 * A pool of Gaussian slots (Algorithm 1's global gs and matured).  Slots
 * [0, num_gs) are optimisable; slots [num_gs, n_slots) are frozen: they are
 * rendered but never receive gradients, steps or relocation (Sec. 4.2).
 * A training pool has n_slots = 2 num_gs (slot i's matured snapshot lives at
 * num_gs + i); a serving pool may set num_gs = 0.
 * All pointers are device memory, caller-owned; the library keeps copies of
 * the pointers only.  grads/adam_m/adam_v may be NULL for forward-only use. */
typedef struct {
    size_t struct_size;        /* sizeof(swgs_pool) */
    int32_t num_gs;            /* optimisable slots */
    int32_t n_slots;           /* total slots */
    int32_t swin;              /* window length (maximum lifespan) */
    int32_t sh_degree;         /* 0..3 */
    float *params;             /* device [F][n_slots] */
    float *grads;              /* device [F][num_gs] */
    float *adam_m;             /* device [F][num_gs] */
    float *adam_v;             /* device [F][num_gs] */
    int32_t *birth;            /* device [n_slots] */
    int32_t *start;            /* device [n_slots] */
    int32_t *expire;           /* device [n_slots] */
} swgs_pool;

/* One (frame, camera) view (Algorithm 1 samples these from the window).
 * R, t map world to camera (x right, y down, z forward), row-major.
 * The camera is kept in double precision: the integer decisions derived from
 * it (culling, tile ranges, depth keys) are taken in FP64. */
typedef struct {
    int32_t frame;             /* frame index for the lifespan gate */
    int32_t width, height;     /* pixels, >= 1 */
    int32_t reserved;
    double R[9];
    double t[3];
    double fx, fy, cx, cy;     /* pinhole intrinsics in pixels */
    float bg[3];               /* background colour */
    float reserved2;
} swgs_view;

enum { SWGS_MODE_PLAIN = 0, SWGS_MODE_BATCHED = 1, SWGS_MODE_GRAPH = 2 };

typedef struct {
    size_t struct_size;        /* sizeof(swgs_plan_opts) */
    int32_t tile_w, tile_h;    /* 8x8, 16x16 or 32x8 (0,0 = 16x16) */
    int32_t lds_batch;         /* Gaussians staged in LDS per batch: 64/128/256 (0 = tile pixels) */
    int32_t reserved;
    int64_t pair_capacity;     /* (view, tile, Gaussian) pairs held by the workspace (> 0) */
} swgs_plan_opts;

/* Create a plan for rendering/training `views` (host array, copied) on
 * `pool` (copied).  Synchronises: counts the live slots of every distinct
 * frame on the device (lifespans must not change while the plan is in use;
 * mature() invalidates plans whose frames it touches).  *ws_bytes receives
 * the workspace size every call on this plan needs. */
swgs_status swgs_plan_create(swgs_context *ctx, const swgs_pool *pool,
                             const swgs_view *views, int32_t n_views,
                             const swgs_plan_opts *opts, swgs_plan **out,
                             size_t *ws_bytes);
swgs_status swgs_plan_destroy(swgs_plan *plan);

/* Run gating, preprocess and the pair count only, then synchronise and
 * return the number of (view, tile, Gaussian) pairs and of records. */
swgs_status swgs_plan_measure(swgs_context *ctx, swgs_plan *plan, void *workspace,
                              size_t ws_bytes, int64_t *n_pairs, int64_t *n_records);

/* Workspace sub-buffers, for inspection by tests (offset and size in bytes
 * inside the workspace).  Buffers: */
enum {
    SWGS_BUF_ACTIVE_LIST = 0,  /* uint32 slot ids per distinct frame, then the window set A */
    SWGS_BUF_ACTIVE_COUNT,     /* uint32 [n_groups + 1] live counts (last: |A|) */
    SWGS_BUF_RECORD_VIEW_BASE, /* uint32 [n_views + 1] first record of each view */
    SWGS_BUF_DEPTH_KEY,        /* uint32 [R] FP32 camera-z bits of the records, sorted ascending after a
                                  forward (culled records carry 0xFFFFFFFF and sort last) */
    SWGS_BUF_TILE_COUNT,       /* uint32 [R] tiles covered by each record */
    SWGS_BUF_RECT,             /* uint32 [R][2]: x0 | y0 << 16, x1 | y1 << 16 (tiles, half-open) */
    SWGS_BUF_SPLAT,            /* float [R][12]: floor(u), floor(v), 0.5-(u-floor(u)), 0.5-(v-floor(v)),
                                  -log2(e) A/2, -log2(e) B, -log2(e) C/2 (conic [[A,B],[B,C]]), opacity,
                                  r, g, b, FP32 depth */
    SWGS_BUF_PAIR_KEY,         /* uint32 [cap] global tile id of each sorted pair */
    SWGS_BUF_PAIR_VAL,         /* uint32 [cap] record of each sorted pair */
    SWGS_BUF_PAIR_COUNT,       /* uint32 [2]: pairs emitted, overflow flag */
    SWGS_BUF_TILE_RANGE,       /* uint32 [n_tiles][2] first, last pair of each tile */
    SWGS_BUF_T_FINAL,          /* float [P] final transmittance per pixel */
    SWGS_BUF_DLDC,             /* float [3P] dL/dimage (fused L1 gradient) */
    SWGS_BUF_RECORD_GRAD,      /* float [9][R] d/d(u, v, A, B, C, o, r, g, b) */
    SWGS_BUF_DEPTH_ORDER,      /* uint32 [R] records in ascending (depth, record) order after a forward */
    SWGS_BUF_COUNT_
};
swgs_status swgs_plan_buffer(const swgs_plan *plan, int32_t which, size_t *offset, size_t *bytes);

/* Plan geometry: n_groups distinct frames, R records, P pixels, n_tiles. */
swgs_status swgs_plan_info(const swgs_plan *plan, int64_t *n_groups, int64_t *n_records,
                           int64_t *n_pixels, int64_t *n_tiles);

/* ----------------------------------------------------------- render path
 * Forward render of every view (Eqs. 1-3 with the lifespan gate): writes
 * `images` (device float [3 P], concatenated planar views).  When `targets`
 * (device, same layout) is not NULL, also computes the L1 image loss and its
 * gradient dL/dimage = sign(C - GT) / (V * 3 * H_v * W_v) into the workspace
 * (SWGS_BUF_DLDC), and, when `stats` (device double[8]) is not NULL, writes
 * stats[0] = sum_v mean|C - GT| / V, stats[1] = mean (C - GT)^2 over all
 * pixels and channels, stats[4] = pairs, stats[6] = overflow flag. */
swgs_status swgs_render_forward(swgs_context *ctx, swgs_plan *plan, void *workspace,
                                size_t ws_bytes, float *images, const float *targets,
                                double *stats);

/* Backward of the last forward on this plan and workspace (Algorithm 1's
 * backward): given dL/dimage (device float [3 P], or NULL to use the fused
 * L1 gradient of the forward), writes dL/dparams of the optimisable slots
 * that are live in a frame of the plan into pool->grads (other slots'
 * gradients are not written).  Frozen slots receive nothing.
 * When add_regulariser != 0 the gradient of
 * lambda_o mean_A sigmoid(logit) + lambda_s mean_A sum_j exp(s_j) is added,
 * with the weights of `cfg` (may be NULL only when add_regulariser == 0). */
typedef struct swgs_step_cfg swgs_step_cfg;
swgs_status swgs_render_backward(swgs_context *ctx, swgs_plan *plan, void *workspace,
                                 size_t ws_bytes, const float *dL_dimages,
                                 int32_t add_regulariser, const swgs_step_cfg *cfg);

/* ------------------------------------------------------------- step
 * Optimiser hyper-parameters (Sec. 8.1 gives lambda_o, lambda_s, noise_lr;
 * the rest are readings of the 3DGS / 3DGS-MCMC defaults). */
struct swgs_step_cfg {
    size_t struct_size;        /* sizeof(swgs_step_cfg) */
    float lr_mean, lr_scale, lr_quat, lr_logit, lr_sh_dc, lr_sh_rest;
    float beta1, beta2, eps;
    float noise_lr, noise_k, noise_t0;     /* SGLD: noise_lr lr_mean sigmoid(-k (o - t0)) Sigma eta */
    float lambda_opacity, lambda_scale;    /* regulariser weights */
    float grad_scale_base;                 /* adaptive mean-gradient scaling base (0 = off) */
    int32_t window_start;                  /* st of the window [st, st + swin) */
    int32_t relocate_period;               /* relocate when step % period == 0 (0 = never) */
    int32_t reloc_n_max;                   /* cap on copies per source (>= 1) */
    int32_t mode;                          /* SWGS_MODE_* for swgs_window_step */
    int32_t reserved;
};

/* Fill *cfg with the defaults (Sec. 8.1 values and the readings). */
void swgs_step_cfg_default(swgs_step_cfg *cfg);

/* Adam (bias-correction step adam_t >= 1) with adaptive mean-gradient
 * scaling, then SGLD noise on the means, over A = optimisable slots live in
 * a frame of the plan, reading pool->grads.  Noise uses Philox4x32-10 keyed
 * by `seed` with counter (slot, step).  When eta (device float [3][num_gs])
 * is not NULL it replaces the generated normals. */
swgs_status swgs_step(swgs_context *ctx, swgs_plan *plan, void *workspace, size_t ws_bytes,
                      const swgs_step_cfg *cfg, int64_t adam_t, uint64_t step, uint64_t seed,
                      const float *eta);

/* Relocation of dead Gaussians in A (Sec. 3.2): see DESIGN for the exact
 * sampler.  dst, src: device int32 [num_gs]; count: device int32 [1]; pairs
 * (dst[j], src[j]), j < *count, in ascending dst order. */
swgs_status swgs_relocate(swgs_context *ctx, swgs_plan *plan, void *workspace, size_t ws_bytes,
                          const swgs_step_cfg *cfg, uint64_t step, uint64_t seed,
                          int32_t *dst, int32_t *src, int32_t *count);

/* One window step (Algorithm 1's inner iteration over all views of the
 * window at once): forward with the fused L1 gradient against `targets`,
 * backward with the regulariser, Adam + scaling + SGLD, and relocation when
 * step % relocate_period == 0.  cfg->mode selects the launch structure:
 * PLAIN = one launch sequence per view (the per-frame baseline), BATCHED =
 * one launch per kernel over all views, GRAPH = the batched sequence
 * captured once into a hipGraph and replayed (step numbers advance on the
 * device; the first call with a plan captures).  `images` may be NULL.
 * stats (device double[8]): [0] L1 term, [1] MSE, [2] regulariser,
 * [3] total loss, [4] pairs, [5] dead slots relocated, [6] overflow flag,
 * [7] |A|. */
swgs_status swgs_window_step(swgs_context *ctx, swgs_plan *plan, void *workspace, size_t ws_bytes,
                             const swgs_step_cfg *cfg, const float *targets, float *images,
                             int64_t adam_t, uint64_t step, uint64_t seed, double *stats);

/* ------------------------------------------------------------- timing
 * Measurement support.  When timing is on, every launch of a kernel class
 * made by the eager modes (not inside a captured graph) is bracketed by HIP
 * events recorded on the context stream, and the blend kernels count the
 * (pixel, list entry) pairs they evaluate.  swgs_plan_set_timing
 * synchronises, resets the records and switches timing on (on != 0) or off.
 * swgs_plan_timing synchronises, returns per class the summed kernel time
 * (ms[8], host) and the number of bracketed launches (launches[8], host),
 * and, if evals (host uint64[3]) is not NULL, the (pixel, list entry) pairs
 * evaluated by the forward [0] and the backward [1] blend and the pairs the
 * forward blended [2] (the backward differentiates exactly those); then
 * resets.  Classes: 0 gating,
 * 1 preprocess, 2 depth sort + pair emission + tile sort + ranges,
 * 3 forward blend, 4 backward blend, 5 backward preprocess, 6 Adam + SGLD,
 * 7 relocation. */
swgs_status swgs_plan_set_timing(swgs_context *ctx, swgs_plan *plan, void *workspace, size_t ws_bytes,
                                 int32_t on);
swgs_status swgs_plan_timing(swgs_context *ctx, swgs_plan *plan, void *workspace, size_t ws_bytes,
                             double *ms, int64_t *launches, uint64_t *evals);

/* ------------------------------------------------------------- mature
 * Algorithm 1's mature(st) on a training pool: optimisable slots with
 * start < st are copied to their frozen slot (num_gs + i) with their
 * lifespan, emitted into `record` (device memory, capacity bytes), and
 * re-armed to [expire, expire + swin) with birth = start = old expire.
 * Record layout (little endian): header int32[8] = {0x53475753 ('SWGS'),
 * version 1, st, count, sh_degree, F, swin, 0}; then uint32 slot[count];
 * int32 birth[count], start[count], expire[count]; float params[F][count].
 * Synchronises (the count is needed); *count_out (host) receives it and
 * *bytes_out (host) the record size. */
swgs_status swgs_mature(swgs_context *ctx, const swgs_pool *pool, int32_t st,
                        void *record, size_t capacity, int64_t *count_out, size_t *bytes_out);

/* Bytes of a mature record for `count` Gaussians of SH degree d. */
size_t swgs_record_bytes(int64_t count, int32_t sh_degree);

#ifdef __cplusplus
}
#endif
#endif /* SWGS_H */

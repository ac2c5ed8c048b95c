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
    int32_t width, height;     /* pixels, 1..131072 each, width * height < 2^31 */
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

/* Bind a pool once (Algorithm 1's global gs and matured, Sec. 4.2): the
 * descriptor is checked (struct_size, counts, SH degree) and every non-NULL
 * pointer must be device memory of the context's device
 * (SWGS_ERR_INVALID_ARG names the first that is not).  The handle keeps a
 * copy of the descriptor -- the library never frees the caller's buffers --
 * and swgs_pool_desc returns it (valid until release) for every call that
 * takes a const swgs_pool *. */
typedef struct swgs_pool_handle swgs_pool_handle;
swgs_status swgs_pool_bind(swgs_context *ctx, const swgs_pool *desc, swgs_pool_handle **out);
const swgs_pool *swgs_pool_desc(const swgs_pool_handle *h);
swgs_status swgs_pool_release(swgs_pool_handle *h);

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
    SWGS_BUF_RECORD_GRAD,      /* float [R][9] d/d(u, v, A, B, C, o, r, g, b), each the sum of
                                  the record's per-tile terms in tile row-major order */
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
 * pixels and channels, stats[4] = pairs, stats[6] = flags as for
 * swgs_window_step (1: pair overflow, 2: stale plan). */
swgs_status swgs_render_forward(swgs_context *ctx, swgs_plan *plan, void *workspace,
                                size_t ws_bytes, float *images, const float *targets,
                                double *stats);

/* Backward of the last forward on this plan and workspace (Algorithm 1's
 * backward): given dL/dimage (device float [3 P], or NULL to use the fused
 * L1 gradient of the forward), writes dL/dparams of the optimisable slots
 * that are live in a frame of the plan into pool->grads (other slots'
 * gradients are not written).  Frozen slots receive nothing.  After a
 * forward whose pairs overflowed the capacity (stats flag 1) the image
 * term contributes zero gradients.
 * When add_regulariser != 0 the gradient of
 * lambda_o mean_A sigmoid(logit) + lambda_s mean_A sum_j exp(s_j) is added,
 * with the weights of `cfg` (may be NULL only when add_regulariser == 0). */
typedef struct swgs_step_cfg swgs_step_cfg;
swgs_status swgs_render_backward(swgs_context *ctx, swgs_plan *plan, void *workspace,
                                 size_t ws_bytes, const float *dL_dimages,
                                 int32_t add_regulariser, const swgs_step_cfg *cfg);

/* ------------------------------------------------------------- step
 * Optimiser and loss hyper-parameters (Sec. 8.1 gives lambda_o, lambda_s,
 * noise_lr; the loss follows 3DGS-MCMC's practice, Sec. 4.4; the rest are
 * readings of the 3DGS / 3DGS-MCMC defaults). */
struct swgs_step_cfg {
    size_t struct_size;        /* sizeof(swgs_step_cfg) */
    float lr_mean, lr_scale, lr_quat, lr_logit, lr_sh_dc, lr_sh_rest;
    float beta1, beta2, eps;
    float noise_lr, noise_k, noise_t0;     /* SGLD: noise_lr lr_mean sigmoid(-k (o - t0)) Sigma eta */
    float lambda_opacity, lambda_scale;    /* regulariser weights */
    float lambda_dssim;                    /* image term (1 - l) L1 + l (1 - SSIM), in [0, 1] (default 0.2) */
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
 * the D-SSIM term and its gradient when cfg->lambda_dssim > 0 (SSIM of Wang
 * et al. 2004: 11x11 Gaussian window, sigma 1.5, zero padding,
 * C1 = 0.01^2, C2 = 0.03^2, averaged over pixels and channels), backward
 * with the regulariser, Adam + scaling + SGLD, and relocation when
 * step % relocate_period == 0.  cfg->mode selects the launch structure:
 * PLAIN = one launch sequence per view (the per-frame baseline), BATCHED =
 * one launch per kernel over all views, GRAPH = the batched sequence
 * captured once into a hipGraph and replayed (the first call with a plan,
 * or with a different workspace, targets, images or cfg, captures; adam_t,
 * step and seed are taken from every call's arguments).  `images` may be NULL (the
 * renders then stay in the workspace).
 * stats (device double[8]): [0] image term
 * (1/V) sum_v [(1 - l) mean|C - GT| + l (1 - SSIM_v)], [1] MSE, [2] regulariser,
 * [3] total loss, [4] pairs, [5] dead slots relocated, [6] flags: bit 0
 * (value 1) the pair capacity overflowed (BATCHED and GRAPH modes: the
 * step's image term then contributes zero gradients; PLAIN mode fails with
 * SWGS_ERR_CAPACITY), bit 1 (value 2) a frame's live
 * count differs from the count at plan creation (the lifespans changed, e.g.
 * by mature() or apply_update(): the plan's lists are stale and the step's
 * results are not valid; make a new plan), [7] |A|. */
swgs_status swgs_window_step(swgs_context *ctx, swgs_plan *plan, void *workspace, size_t ws_bytes,
                             const swgs_step_cfg *cfg, const float *targets, float *images,
                             int64_t adam_t, uint64_t step, uint64_t seed, double *stats);

/* ------------------------------------------------------------- timing
 * Measurement support for the eager modes (nothing is recorded inside a
 * captured graph).  swgs_plan_set_timing synchronises, resets the records
 * and sets `flags`: SWGS_TIMING_EVENTS brackets every launch of a kernel
 * class with HIP events on the context stream; SWGS_TIMING_COUNT makes the
 * blend kernels count the (pixel, list entry) pairs they evaluate (the
 * forward then runs its counting build, a few instructions per entry
 * slower, so time and count in separate runs); 0 switches both off; other
 * bits are rejected.  swgs_plan_timing synchronises, returns per class the
 * summed kernel time (ms[9], host) and the number of bracketed launches
 * (launches[9], host), and, if evals (host uint64[3]) is not NULL, the
 * (pixel, list entry) pairs evaluated by the forward [0] and the backward
 * [1] blend and the pairs the forward blended [2] (the backward
 * differentiates exactly those); then resets.  Classes: 0 gating,
 * 1 preprocess, 2 depth sort + pair emission + tile sort + ranges,
 * 3 forward blend, 4 backward blend, 5 record-gradient reduce + backward
 * preprocess, 6 Adam + SGLD,
 * 7 relocation, 8 D-SSIM (forward and gradient). */
enum { SWGS_TIMING_EVENTS = 1, SWGS_TIMING_COUNT = 2 };
swgs_status swgs_plan_set_timing(swgs_context *ctx, swgs_plan *plan, void *workspace, size_t ws_bytes,
                                 int32_t flags);
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

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): swgs_mature without
 * any allocation.  Arguments, record layout, pool changes and errors are
 * those of swgs_mature, and so are the results, bit for bit.  Its scratch
 * (flags, positions, scan sums, count: about 8 bytes per optimisable slot)
 * is a 16 MiB array that the library holds on each device it runs on until
 * the process ends, so num_gs must not exceed swgs_mature_noalloc_max_gs()
 * (2,096,891); a larger pool fails with SWGS_ERR_CAPACITY before anything is
 * launched.  All calls on one device share that array: calls that overlap
 * on one device (two host threads, or two contexts on different streams)
 * race.  Synchronises (once to read the count, once at the end). */
swgs_status swgs_mature_noalloc(swgs_context *ctx, const swgs_pool *pool, int32_t st,
                                void *record, size_t capacity, int64_t *count_out, size_t *bytes_out);
/* Largest num_gs swgs_mature_noalloc accepts. */
int64_t swgs_mature_noalloc_max_gs(void);

/* Bytes of a mature record for `count` Gaussians of SH degree d. */
size_t swgs_record_bytes(int64_t count, int32_t sh_degree);

/* ------------------------------------------------------------- codec
 * The compact per-frame update (Sec. 5.2 Eq. 4, Sec. 5.6.2 and Table 6,
 * Sec. 5.5): re-encode a mature record (`record`, device, version 1) into a
 * version-2 record in `out` (device, capacity bytes) carrying per Gaussian
 * only its mean, log-scale, rotation, opacity and SH DC term -- the higher
 * SH bands are not streamed -- either in FP32 (enc SWGS_ENC_FP32, 56 bytes)
 * or at Table 6's precisions (SWGS_ENC_Q: FP16 mean and log-scale saturated
 * to +-65504, round to nearest even; 8-bit rotation code
 * rint(c 127.5 + 127.5) of each component c of q/|q| in IEEE FP32 with the
 * zero quaternion sent as the identity; 8-bit opacity code round(sigma 255)
 * decided on the logit against the thresholds fl32(logit((k - 1/2)/255)),
 * k = 1..255; SH DC in FP32: 29 bytes).  keep in [0, count) keeps the keep
 * entries of largest opacity logit (ties to the lower entry) and marks the
 * others empty (Sec. 5.5's tail-drop); keep < 0 keeps all.
 * Layout (little endian): int32 header[16] = {magic 'SWGS', 2, st, count,
 * kept, enc, swin, flags, slot0, birth0, start0, expire0, source SH degree,
 * 0, 0, 0}; then, each array at a 16-byte boundary: [flags & 1] uint32
 * slot[count], int32 birth[count], start[count], expire[count] (present
 * unless every entry shares one lifespan and the slots are slot0 + k);
 * [flags & 2] uint32 keep mask[ceil(count/32)] (bit k & 31 of word k >> 5);
 * the kept entries' attributes in entry order, planar: mean[3][kept],
 * scale[3][kept], quat[4][kept], opacity[kept], dc[3][kept].
 * out == NULL: only *bytes_out (host) receives the size.  Synchronises. */
enum { SWGS_ENC_FP32 = 1, SWGS_ENC_Q = 2 };
swgs_status swgs_encode_update(swgs_context *ctx, const void *record, size_t record_bytes, int32_t enc,
                               int64_t keep, void *out, size_t capacity, size_t *bytes_out);

/* ------------------------------------------------------------- update
 * Algorithm 2's client-side update (Sec. 4.3): write the entries of a mature
 * record (device memory, record_bytes bytes, the layout swgs_mature writes,
 * or the compact layout of swgs_encode_update) into `pool`.  A compact
 * record writes the five streamed attributes, zeroes the pool's higher SH
 * rows, and gives entries the tail-drop removed the empty lifespan
 * [birth, birth) (never drawn; parameters untouched).  slot_base < 0: entry k goes to slot record.slot[k], the slot
 * it was emitted from (Algorithm 2 replaces slice birth mod swin of the
 * client buffer, which is that slot range); slot_base >= 0: entry k goes to
 * slot slot_base + k (appending the update to a pool that keeps every frame
 * resident).  Parameters, start and expire, and birth if pool->birth is not
 * NULL, are overwritten.  Synchronises twice: to read and check the header
 * (magic, version, SH degree of a full record, size) and, after the scatter, to check
 * that every entry's slot lies inside the pool (SWGS_ERR_INVALID_ARG names
 * how many did not; those entries are skipped, the others written).
 * *count_out (host, nullable) receives the entry count. */
swgs_status swgs_apply_update(swgs_context *ctx, const swgs_pool *pool, const void *record,
                              size_t record_bytes, int64_t slot_base, int64_t *count_out);

/* ------------------------------------------------------------ trainer
 * The paper's training loop over one window (Algorithm 1's train_swin):
 * each iteration samples one (frame, camera) view of the window, renders
 * it, and runs loss, backward, Adam + SGLD on the Gaussians live in its
 * frame and relocation every cfg->relocate_period iterations (Sec. 4.4,
 * Sec. 3.2).  swgs_trainer_create makes one single-view plan per entry of
 * `views` (host array; opts as for swgs_plan_create, pair_capacity large
 * enough for every view) sharing one workspace; the pool's lifespans must
 * not change while the trainer lives (destroy it before mature()).
 * swgs_trainer_run runs `iterations` iterations numbered iter0, iter0 + 1,
 * ...: iteration i uses view swgs_trainer_view(seed, i, n_views), Adam
 * bias-correction step t = i + 1, and i as the step keying the SGLD noise,
 * the relocation draw and the relocation cadence (i % relocate_period == 0);
 * targets (host array of n_views device pointers) hold each view's ground
 * truth [3][H][W].  cfg->mode is ignored (each iteration is one batched
 * window step).  stats (device, nullable) receives 8 doubles per
 * iteration, as swgs_window_step reports them; views_out (host, nullable)
 * the view of each iteration.  Nothing synchronises.
 * swgs_trainer_view: floor(x0 n_views / 2^32) with x0 the first word of
 * Philox4x32-10 at counter (i_lo, i_hi, 0, 0x504D4153) keyed by the seed.
 * swgs_schedule_expire: Algorithm 1's schedule_expire after the genesis
 * window -- optimisable block k of num_gs/swin slots expires at frame k
 * (k >= 1), block 0 at swin -- so one slice matures per frame. */
typedef struct swgs_trainer swgs_trainer;
swgs_status swgs_trainer_create(swgs_context *ctx, const swgs_pool *pool, const swgs_view *views, int32_t n_views,
                                const swgs_plan_opts *opts, swgs_trainer **out);
swgs_status swgs_trainer_run(swgs_trainer *trainer, const swgs_step_cfg *cfg, const float *const *targets,
                             int64_t iterations, int64_t iter0, uint64_t seed, double *stats, int32_t *views_out);
void swgs_trainer_destroy(swgs_trainer *trainer);
int32_t swgs_trainer_view(uint64_t seed, int64_t iteration, int32_t n_views);
swgs_status swgs_schedule_expire(swgs_context *ctx, const swgs_pool *pool);

/* ------------------------------------------------------------- player
 * Client-side playback of the update stream (Algorithm 2, Sec. 4.3).  The
 * caller owns `buffer` (num_gs slots, parameters at the buffer's SH degree,
 * start/expire, optional birth).  swgs_player_push is the stream read: it
 * checks the record (version 1 or 2, host memory, `bytes` bytes) and that
 * its slots lie in the buffer, copies it into a pinned staging slot and
 * starts its host-to-device transfer on the player's own copy stream
 * (default priority), so the transfer overlaps rendering on the context
 * stream; the record is due at the birth frame of its first entry.  It
 * fails with SWGS_ERR_CAPACITY when queue_depth records are queued and not
 * yet applied (advance first), and waits for an applied record's decode to
 * finish before reusing its staging slot.  swgs_player_advance(frame) is one
 * tick of the update thread: every queued record due at `frame` or earlier
 * is decoded into the buffer on the context stream after its transfer, in
 * push order, without a host synchronisation (*applied, host, nullable,
 * receives how many); renders issued later on the context stream see the
 * new slices.  A record pushed after its frame was ticked is applied at the
 * next tick (the paper's loop matches the frame exactly and would skip it).
 * swgs_player_queued reports the records waiting and the total applied.
 * swgs_player_destroy synchronises both streams and frees the staging. */
typedef struct swgs_player swgs_player;
typedef struct {
    int32_t struct_size;       /* sizeof(swgs_player_opts) */
    int32_t queue_depth;       /* records in flight: 1..64 */
    int64_t max_record_bytes;  /* largest record pushed (>= 64) */
} swgs_player_opts;
swgs_status swgs_player_create(swgs_context *ctx, const swgs_pool *buffer, const swgs_player_opts *opts,
                               swgs_player **out);
swgs_status swgs_player_push(swgs_player *player, const void *record, size_t bytes);
swgs_status swgs_player_advance(swgs_player *player, int32_t frame, int32_t *applied);
swgs_status swgs_player_queued(const swgs_player *player, int32_t *queued, int64_t *applied_total);
void swgs_player_destroy(swgs_player *player);

/* ------------------------------------------------------------ serving
 * A render server over a resident pool.  Sec. 4.3's client keeps the
 * sliding pool on the device and renders, for a requested frame, the slots
 * live at that frame; here every per-frame update of a clip stays resident
 * (apply them with slot_base >= 0), so any frame can be served.
 *
 * Requests (frame, camera, resolution) wait in a FIFO queue.  Whenever one
 * of `lanes` streams is free, requests are taken from the head of the queue
 * into one batch while the batch's exact workspace fits the largest free
 * block of the memory budget, and max_batch / max_batch_pixels allow
 * (admission by memory; a request that cannot fit even an empty budget
 * fails with SWGS_ERR_WORKSPACE_TOO_SMALL).  Batches of mixed resolutions
 * and frames render forward only in one launch sequence (preprocess, depth
 * sort, binning, tile sort, blend); batches on different lanes overlap on
 * the device, and requests that arrive meanwhile queue for the next free
 * lane.  Live lists per frame are built once at creation, so a batch runs no
 * gating.  The pair capacity of a batch is estimated from the largest
 * pairs-per-record ratio seen so far; a batch whose pairs overflowed is
 * rendered again with the exact count (stats.redone).  An image never
 * depends on the batch it was rendered in: it equals the image of the same
 * request rendered alone, bit for bit. */
typedef struct swgs_server swgs_server;

typedef struct {
    size_t struct_size;        /* sizeof(swgs_server_opts) */
    int32_t n_frames;          /* frames 0 .. n_frames-1 may be requested (>= 1) */
    int32_t lanes;             /* batches in flight, one stream each: 1..4 */
    int32_t max_batch;         /* requests per batch: 1..1024 */
    int32_t tile_w, tile_h;    /* as swgs_plan_opts (0,0 = 16x16) */
    int32_t lds_batch;         /* as swgs_plan_opts (0 = tile pixels) */
    int64_t max_batch_pixels;  /* pixels per batch (0: no limit; a single larger request still runs alone) */
    double pair_ratio;         /* initial pairs-per-record estimate (<= 0: 4) */
} swgs_server_opts;

typedef struct {
    swgs_view view;            /* frame, resolution, camera, background */
    float *image;              /* device [3][height][width] output, or NULL: rendered, then dropped */
    double arrival;            /* seconds on the server clock (see swgs_server_submit / _run) */
    double ready;              /* out: seconds on the server clock when the image was complete */
    int32_t status;            /* out: -1 while pending, then SWGS_OK or the reason it failed */
    int32_t batch;             /* out: id of the batch that rendered it (-1 if none) */
} swgs_request;

typedef struct {
    size_t struct_size;        /* sizeof(swgs_serve_stats) */
    int64_t completed;         /* requests with status SWGS_OK */
    int64_t failed;            /* requests with any other final status */
    int64_t batches;           /* batches launched (redone ones counted once) */
    int64_t redone;            /* batches rendered again after a pair overflow */
    double wall_s;             /* first arrival to last ready, seconds */
    double mean_batch;         /* requests per batch */
    size_t peak_bytes;         /* high-water mark of the budget in use */
    size_t budget_bytes;       /* memory budget for batches (arena minus resident lists) */
    size_t resident_bytes;     /* per-frame live lists kept for the server's lifetime */
} swgs_serve_stats;

/* Algorithm 2's render (Sec. 4.3) of one batch of requests of mixed frames
 * and resolutions on `pool`, without a server: the slots live at each
 * request's frame (optimisable and frozen alike) are rendered forward in one
 * launch sequence (gating, preprocess, depth sort, binning, tile sort,
 * blend) into each request's `image` (device [3][height][width]; NULL:
 * rendered, then dropped), each image bit-identical to the same request in
 * any other batch.  opts as for swgs_plan_create (pair_capacity is the
 * batch's pair capacity).  swgs_query_workspace_batch returns the workspace
 * bytes the batch needs (device memory, 256-byte aligned, caller-owned;
 * it counts the live slots of each frame on the device and synchronises).
 * swgs_render_batch synchronises, sets each request's status (SWGS_OK, or
 * SWGS_ERR_CAPACITY when the pairs exceeded the capacity: the call then
 * fails with the needed count in its message), batch 0 and ready 0. */
swgs_status swgs_query_workspace_batch(swgs_context *ctx, const swgs_pool *pool, const swgs_request *reqs,
                                       int32_t n, const swgs_plan_opts *opts, size_t *ws_bytes);
swgs_status swgs_render_batch(swgs_context *ctx, const swgs_pool *pool, swgs_request *reqs, int32_t n,
                              const swgs_plan_opts *opts, void *workspace, size_t ws_bytes);

/* Create a server on `pool` (copied; only params, start, expire are used).
 * `arena` (device, 256-byte aligned, arena_bytes, caller-owned) is carved
 * up by the server: the per-frame live lists at its head for the server's
 * lifetime, the rest as the memory budget of the batches in flight.
 * Synchronises on the context stream (counts and builds the live lists);
 * the pool must not change while the server exists. */
swgs_status swgs_server_create(swgs_context *ctx, const swgs_pool *pool, const swgs_server_opts *opts,
                               void *arena, size_t arena_bytes, swgs_server **out);
/* Waits for the batches in flight, then releases the server's streams,
 * events and pinned buffers (not the arena). */
swgs_status swgs_server_destroy(swgs_server *srv);
/* Queue n requests (host array).  Each struct must stay valid until its
 * status is final: the server writes ready, status and batch into it.
 * arrival is set to the current server-clock time.  Requests with a bad
 * frame, size or focal length fail at once (SWGS_ERR_INVALID_ARG in their
 * status); the call itself fails only on bad arguments. */
swgs_status swgs_server_submit(swgs_server *srv, swgs_request *reqs, int32_t n);
/* Drive the scheduler once: retire finished batches (setting ready/status),
 * then launch batches on free lanes.  wait != 0: keep driving until at
 * least one request became final or none is pending.  *pending (host,
 * nullable) receives the number of requests not yet final. */
swgs_status swgs_server_progress(swgs_server *srv, int32_t wait, int64_t *pending);
/* Replay a request trace and return when every request is final.  The
 * server clock restarts at 0 at the call.  realtime != 0: request i is
 * queued once reqs[i].arrival seconds have passed (arrival values are kept);
 * realtime == 0: all are queued at once with arrival 0.  Requests are queued
 * in ascending arrival order (ties in array order).  *stats (host, nullable)
 * receives the run's statistics. */
swgs_status swgs_server_run(swgs_server *srv, swgs_request *reqs, int32_t n, int32_t realtime,
                            swgs_serve_stats *stats);
/* Statistics since the server (or its last swgs_server_run) started. */
swgs_status swgs_server_stats(const swgs_server *srv, swgs_serve_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* SWGS_H */

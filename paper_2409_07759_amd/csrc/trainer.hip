// The paper's training loop (Algorithm 1, train_swin): each iteration
// samples one (frame, camera) of the window, renders it, takes the loss and
// its gradient, and applies Adam + SGLD to the Gaussians live in that frame,
// relocating dead ones every relocate_period iterations.
//
// A trainer holds one single-view plan per (frame, camera) of the window,
// all sharing one workspace; an iteration is the window step of its
// sampled view's plan (the batched sequence), with the global iteration as
// Adam's bias-correction step t (= iteration + 1) and as the step that
// keys the SGLD noise, the relocation draw and the relocation cadence.
// The view of iteration i is floor(x0 n_views / 2^32) for x0 the first
// word of Philox4x32-10 at counter (i_lo, i_hi, 0, 'SAMP') with the 64-bit
// seed as key.  Schedule helper: Algorithm 1's schedule_expire.
#include <string>
#include <vector>

#include "swgs_internal.h"

struct swgs_trainer {
    swgs_context *ctx = nullptr;
    swgs_pool pool{};
    std::vector<swgs_plan *> plans;
    uint8_t *ws = nullptr;
    size_t ws_bytes = 0;
};

using namespace swgs;

namespace {

constexpr int kBlock = 256;

swgs_status tfail(swgs_context *ctx, swgs_status st, const std::string &why) {
    if (ctx) ctx->err = why;
    return st;
}

// Philox4x32-10 (Salmon et al., SC'11), host side
void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0, h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
        const uint32_t n0 = h1 ^ c[1] ^ k0, n2 = h0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = l1;
        c[2] = n2;
        c[3] = l0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__global__ void __launch_bounds__(kBlock)
k_schedule_expire(int32_t *__restrict__ expire, int num_gs, int swin) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int S = num_gs / swin;
    if (i >= swin * S || S == 0) return;
    const int k = i / S;
    expire[i] = k == 0 ? swin : k;
}

void release(swgs_trainer *t) {
    if (!t) return;
    if (t->ctx) (void)hipStreamSynchronize(t->ctx->stream);
    for (auto *p : t->plans) (void)swgs_plan_destroy(p);
    if (t->ws) (void)hipFree(t->ws);
    delete t;
}

}  // namespace

int32_t swgs_trainer_view(uint64_t seed, int64_t iteration, int32_t n_views) {
    if (n_views <= 0) return -1;
    uint32_t c[4] = {(uint32_t)iteration, (uint32_t)((uint64_t)iteration >> 32), 0u, 0x504D4153u};
    philox_host(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return (int32_t)(((uint64_t)c[0] * (uint64_t)n_views) >> 32);
}

swgs_status swgs_schedule_expire(swgs_context *ctx, const swgs_pool *pool) {
    if (!ctx || !pool || !pool->expire) return SWGS_ERR_INVALID_ARG;
    if (pool->swin < 1 || pool->num_gs < 0) return tfail(ctx, SWGS_ERR_INVALID_ARG, "swin must be >= 1");
    if (pool->num_gs == 0) return SWGS_OK;
    hipLaunchKernelGGL(k_schedule_expire, dim3((pool->num_gs + kBlock - 1) / kBlock), dim3(kBlock), 0, ctx->stream,
                       pool->expire, pool->num_gs, pool->swin);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return tfail(ctx, SWGS_ERR_HIP, hipGetErrorString(e));
    return SWGS_OK;
}

swgs_status swgs_trainer_create(swgs_context *ctx, const swgs_pool *pool, const swgs_view *views, int32_t n_views,
                                const swgs_plan_opts *opts, swgs_trainer **out) {
    if (!ctx || !out) return SWGS_ERR_INVALID_ARG;
    *out = nullptr;
    if (!pool || !views || n_views < 1) return tfail(ctx, SWGS_ERR_INVALID_ARG, "pool and at least one view required");
    auto *t = new swgs_trainer;
    t->ctx = ctx;
    t->pool = *pool;
    size_t need = 0;
    for (int v = 0; v < n_views; ++v) {
        swgs_plan *p = nullptr;
        size_t bytes = 0;
        const swgs_status st = swgs_plan_create(ctx, pool, &views[v], 1, opts, &p, &bytes);
        if (st != SWGS_OK) {
            release(t);
            return st;
        }
        t->plans.push_back(p);
        need = need > bytes ? need : bytes;
    }
    const hipError_t e = hipMalloc(reinterpret_cast<void **>(&t->ws), need);
    if (e != hipSuccess) {
        release(t);
        return tfail(ctx, SWGS_ERR_HIP, std::string("trainer workspace: ") + hipGetErrorString(e));
    }
    t->ws_bytes = need;
    *out = t;
    return SWGS_OK;
}

swgs_status swgs_trainer_run(swgs_trainer *t, const swgs_step_cfg *cfg, const float *const *targets,
                             int64_t iterations, int64_t iter0, uint64_t seed, double *stats, int32_t *views_out) {
    if (!t) return SWGS_ERR_INVALID_ARG;
    swgs_context *ctx = t->ctx;
    if (!cfg || cfg->struct_size != sizeof(swgs_step_cfg)) return tfail(ctx, SWGS_ERR_INVALID_ARG, "cfg.struct_size mismatch");
    if (!targets) return tfail(ctx, SWGS_ERR_INVALID_ARG, "targets must not be NULL");
    if (iterations < 0 || iter0 < 0) return tfail(ctx, SWGS_ERR_INVALID_ARG, "iterations and iter0 must be >= 0");
    const int n = (int)t->plans.size();
    for (int v = 0; v < n; ++v)
        if (!targets[v]) return tfail(ctx, SWGS_ERR_INVALID_ARG, "target of view " + std::to_string(v) + " is NULL");
    swgs_step_cfg c = *cfg;
    c.mode = SWGS_MODE_BATCHED;   // t and the step differ per iteration: set on every call
    for (int64_t i = 0; i < iterations; ++i) {
        const int64_t it = iter0 + i;
        const int v = swgs_trainer_view(seed, it, n);
        if (views_out) views_out[i] = v;
        const swgs_status st = swgs_window_step(ctx, t->plans[v], t->ws, t->ws_bytes, &c, targets[v], nullptr, it + 1,
                                                (uint64_t)it, seed, stats ? stats + 8 * i : nullptr);
        if (st != SWGS_OK) return st;
    }
    return SWGS_OK;
}

void swgs_trainer_destroy(swgs_trainer *t) { release(t); }

// Tile blend, forward (Eq. 3) and its adjoint (Algorithm 1's backward).
//
// One workgroup per (view, tile); one lane per pixel.  The tile's sorted
// list of splats is staged through LDS in batches; every lane walks the
// batch front to back:
//     alpha = min(0.99, o exp(-Q/2)),  skip alpha < 1/255,
//     stop before T (1 - alpha) < 1e-4,  C += c alpha T,  T *= 1 - alpha.
// The record stores the conic pre-scaled by -log2(e)/2 so exp(-Q/2) is one
// v_exp_f32, and the screen position split into an integer part and
// 0.5 - fraction so the pixel offset keeps ~1e-7 px of precision.
//
// The backward walks the same list back to front from each pixel's last
// contributor, recovering the transmittance in front of each splat by
// T <- T / (1 - alpha) (nothing per pair is stored), and keeping the colour
// behind the splat U and the product of (1 - alpha) behind it, so that
//     dC/dalpha_k = T_k (c_k - U_k - prod_k bg).
// Per-splat gradients are summed over the wave with DPP row/bcast adds,
// accumulated per batch in LDS across the waves of the tile, and flushed
// with one global float atomic per component per (tile, splat).
#include "swgs_internal.h"

namespace swgs {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

// alpha of a staged splat at a pixel; identical instruction sequence in the
// forward and the backward so both take the same skip/stop decisions.
#pragma clang fp contract(off)
struct Px {
    float dx, dy, g, og;  // offsets, 2^p2 (= exp(-Q/2)), o * g
};
__device__ __forceinline__ Px eval_splat(float fx, float fy, const float4 a, const float4 b) {
    Px r;
    r.dx = (fx - a.x) + a.z;
    r.dy = (fy - a.y) + a.w;
    // p2 = A' dx^2 + B' dx dy + C' dy^2 (A', B', C' = -log2(e) (A/2, B, C/2))
    const float t = fmaf(b.y, r.dy, b.x * r.dx);
    const float p2 = fmaf(b.z * r.dy, r.dy, t * r.dx);
    r.g = __builtin_amdgcn_exp2f(p2);
    r.og = b.w * r.g;
    return r;
}
#pragma clang fp contract(fast)

// full-wave sum with DPP; the result is valid in lane 63
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, false));
}
__device__ __forceinline__ float wave_sum_to_63(float x) {
    x += dpp_f<0xB1, 0xf>(x);   // quad_perm [1,0,3,2]
    x += dpp_f<0x4E, 0xf>(x);   // quad_perm [2,3,0,1]
    x += dpp_f<0x124, 0xf>(x);  // row_ror:4
    x += dpp_f<0x128, 0xf>(x);  // row_ror:8   -> every lane holds its row sum
    x += dpp_f<0x142, 0xa>(x);  // row_bcast:15 into rows 1, 3
    x += dpp_f<0x143, 0xc>(x);  // row_bcast:31 into rows 2, 3
    return x;
}

// view owning a global tile id: last view whose tile_base <= tile
__device__ __forceinline__ int view_of_tile(const ViewDev *views, int n_views, uint32_t tile) {
    int a = 0, b = n_views;
    while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (views[m].tile_base <= tile) a = m; else b = m;
    }
    return a;
}

template <int TW, int TH, int BATCH>
__global__ void __launch_bounds__(TW *TH)
k_blend_fwd(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ pair_val,
            const float4 *__restrict__ splat, const ViewDev *__restrict__ views,
            int n_views, uint32_t tile_lo, float *__restrict__ images,
            float *__restrict__ T_final, uint32_t *__restrict__ last_out,
            const float *__restrict__ targets, float *__restrict__ dLdC, double *__restrict__ loss_part,
            unsigned long long *__restrict__ counters) {
    constexpr int NT = TW * TH;
    __shared__ float4 sa[BATCH], sb[BATCH], sc[BATCH];
    __shared__ float red[2][NT / 64];
    __shared__ unsigned long long cnt_evals;
    const uint32_t tile = tile_lo + blockIdx.x;
    const ViewDev &V = views[view_of_tile(views, n_views, tile)];
    const uint32_t lt = tile - V.tile_base;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int x = tx * TW + (threadIdx.x % TW), y = ty * TH + (threadIdx.x / TW);
    const bool inside = x < V.width && y < V.height;
    const float fx = (float)x, fy = (float)y;
    const uint2 rg = ranges[tile];
    const uint32_t n = rg.y - rg.x;

    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    uint32_t last = 0;
    uint32_t stop_at = inside ? n : 0;   // list entries this pixel evaluates
    bool done = !inside;
    for (uint32_t b0 = 0; b0 < n; b0 += BATCH) {
        if (__syncthreads_and(done)) break;
        for (int k = threadIdx.x; k < BATCH; k += NT) {
            if (b0 + k < n) {
                const uint32_t r = pair_val[rg.x + b0 + k];
                sa[k] = splat[3 * (size_t)r];
                sb[k] = splat[3 * (size_t)r + 1];
                sc[k] = splat[3 * (size_t)r + 2];
            }
        }
        __syncthreads();
        const int m = (int)min((uint32_t)BATCH, n - b0);
        if (!done) {
            for (int k = 0; k < m; ++k) {
                const Px e = eval_splat(fx, fy, sa[k], sb[k]);
                const float alpha = fminf(0.99f, e.og);
                if (alpha < (1.0f / 255.0f)) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < 1e-4f) { done = true; stop_at = b0 + (uint32_t)k + 1; break; }
                const float w = alpha * T;
                const float4 c = sc[k];
                c0 = fmaf(c.x, w, c0);
                c1 = fmaf(c.y, w, c1);
                c2 = fmaf(c.z, w, c2);
                T = Tn;
                last = b0 + (uint32_t)k + 1;
            }
        }
    }
    float l1 = 0.0f, sq = 0.0f;
    if (inside) {
        const size_t HW = (size_t)V.width * V.height;
        const size_t pix = (size_t)V.pix_base + (size_t)y * V.width + x;
        const size_t o3 = 3 * (size_t)V.pix_base + (size_t)y * V.width + x;
        const float o0 = c0 + T * V.bg[0], o1 = c1 + T * V.bg[1], o2 = c2 + T * V.bg[2];
        if (images) {
            images[o3] = o0;
            images[o3 + HW] = o1;
            images[o3 + 2 * HW] = o2;
        }
        T_final[pix] = T;
        last_out[pix] = last;
        if (targets) {
            const float d0 = o0 - targets[o3], d1 = o1 - targets[o3 + HW], d2 = o2 - targets[o3 + 2 * HW];
            const float s = V.inv_norm;
            dLdC[o3] = d0 > 0.0f ? s : (d0 < 0.0f ? -s : 0.0f);
            dLdC[o3 + HW] = d1 > 0.0f ? s : (d1 < 0.0f ? -s : 0.0f);
            dLdC[o3 + 2 * HW] = d2 > 0.0f ? s : (d2 < 0.0f ? -s : 0.0f);
            l1 = (fabsf(d0) + fabsf(d1) + fabsf(d2)) * s;
            sq = d0 * d0 + d1 * d1 + d2 * d2;
        }
    }
    if (counters) {
        if (threadIdx.x == 0) cnt_evals = 0;
        __syncthreads();
        atomicAdd(&cnt_evals, (unsigned long long)stop_at);
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(counters, cnt_evals);
    }
    if (targets) {
        for (int o = 32; o > 0; o >>= 1) {
            l1 += __shfl_xor(l1, o, 64);
            sq += __shfl_xor(sq, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            red[0][threadIdx.x >> 6] = l1;
            red[1][threadIdx.x >> 6] = sq;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < NT / 64; ++w) { a += red[0][w]; b += red[1][w]; }
            loss_part[2 * (size_t)blockIdx.x] = a;
            loss_part[2 * (size_t)blockIdx.x + 1] = b;
        }
    }
}

template <int TW, int TH, int BATCH>
__global__ void __launch_bounds__(TW *TH)
k_blend_bwd(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ pair_val,
            const float4 *__restrict__ splat, const ViewDev *__restrict__ views,
            int n_views, uint32_t tile_lo, const float *__restrict__ T_final,
            const uint32_t *__restrict__ last_in, const float *__restrict__ dLdC,
            float *__restrict__ rec_grad, size_t R, unsigned long long *__restrict__ counters) {
    constexpr int NT = TW * TH;
    __shared__ float4 sa[BATCH], sb[BATCH], sc[BATCH];
    __shared__ uint32_t srec[BATCH];
    __shared__ float acc[9][BATCH];
    __shared__ uint32_t smax;
    const uint32_t tile = tile_lo + blockIdx.x;
    const ViewDev &V = views[view_of_tile(views, n_views, tile)];
    const uint32_t lt = tile - V.tile_base;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int x = tx * TW + (threadIdx.x % TW), y = ty * TH + (threadIdx.x / TW);
    const bool inside = x < V.width && y < V.height;
    const float fx = (float)x, fy = (float)y;
    const uint2 rg = ranges[tile];

    float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
    uint32_t lst = 0;
    if (inside) {
        const size_t HW = (size_t)V.width * V.height;
        const size_t pix = (size_t)V.pix_base + (size_t)y * V.width + x;
        const size_t o3 = 3 * (size_t)V.pix_base + (size_t)y * V.width + x;
        T = T_final[pix];
        lst = last_in[pix];
        g0 = dLdC[o3];
        g1 = dLdC[o3 + HW];
        g2 = dLdC[o3 + 2 * HW];
    }
    if (threadIdx.x == 0) smax = 0;
    for (int k = threadIdx.x; k < BATCH; k += NT)
        for (int c = 0; c < 9; ++c) acc[c][k] = 0.0f;
    __syncthreads();
    atomicMax(&smax, lst);
    __syncthreads();
    const uint32_t nmax = smax;
    if (counters) {
        // pixel x list entries this tile's backward evaluates (timing runs only)
        __shared__ unsigned long long cnt_evals;
        if (threadIdx.x == 0) cnt_evals = 0;
        __syncthreads();
        atomicAdd(&cnt_evals, (unsigned long long)lst);
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(counters + 1, cnt_evals);
    }
    const float bg0 = V.bg[0], bg1 = V.bg[1], bg2 = V.bg[2];
    float U0 = 0.0f, U1 = 0.0f, U2 = 0.0f, Rr = 1.0f;
    const int lane = threadIdx.x & 63;

    for (uint32_t b_end = nmax; b_end > 0;) {
        const uint32_t b_start = b_end > (uint32_t)BATCH ? b_end - BATCH : 0;
        const int m = (int)(b_end - b_start);
        for (int k = threadIdx.x; k < m; k += NT) {
            const uint32_t r = pair_val[rg.x + b_start + k];
            srec[k] = r;
            sa[k] = splat[3 * (size_t)r];
            sb[k] = splat[3 * (size_t)r + 1];
            sc[k] = splat[3 * (size_t)r + 2];
        }
        __syncthreads();
        for (int k = m - 1; k >= 0; --k) {
            const uint32_t idx = b_start + (uint32_t)k;
            float v0 = 0, v1 = 0, v2 = 0, v3 = 0, v4 = 0, v5 = 0, v6 = 0, v7 = 0, v8 = 0;
            bool contrib = false;
            if (idx < lst) {
                const Px e = eval_splat(fx, fy, sa[k], sb[k]);
                const float alpha = fminf(0.99f, e.og);
                if (alpha >= (1.0f / 255.0f)) {
                    contrib = true;
                    const float om = 1.0f - alpha;
                    T = T / om;                        // transmittance in front of k
                    const float4 c = sc[k];
                    const float da = T * (g0 * (c.x - U0 - Rr * bg0) + g1 * (c.y - U1 - Rr * bg1) +
                                          g2 * (c.z - U2 - Rr * bg2));
                    const float w = alpha * T;
                    v0 = g0 * w;
                    v1 = g1 * w;
                    v2 = g2 * w;
                    U0 = fmaf(c.x, alpha, om * U0);
                    U1 = fmaf(c.y, alpha, om * U1);
                    U2 = fmaf(c.z, alpha, om * U2);
                    Rr *= om;
                    if (e.og < 0.99f) {
                        // alpha = o g, g = exp(-Q/2): dQ = -alpha/2 dalpha
                        const float dQ = -0.5f * e.og * da;
                        v3 = e.g * da;
                        v4 = dQ * e.dx * e.dx;
                        v5 = dQ * e.dx * e.dy;
                        v6 = dQ * e.dy * e.dy;
                        v7 = dQ * e.dx;
                        v8 = dQ * e.dy;
                    }
                }
            }
            if (__ballot(contrib) != 0) {
                v0 = wave_sum_to_63(v0);
                v1 = wave_sum_to_63(v1);
                v2 = wave_sum_to_63(v2);
                v3 = wave_sum_to_63(v3);
                v4 = wave_sum_to_63(v4);
                v5 = wave_sum_to_63(v5);
                v6 = wave_sum_to_63(v6);
                v7 = wave_sum_to_63(v7);
                v8 = wave_sum_to_63(v8);
                if (lane == 63) {
                    if (NT == 64) {
                        acc[0][k] += v0; acc[1][k] += v1; acc[2][k] += v2;
                        acc[3][k] += v3; acc[4][k] += v4; acc[5][k] += v5;
                        acc[6][k] += v6; acc[7][k] += v7; acc[8][k] += v8;
                    } else {
                        atomicAdd(&acc[0][k], v0); atomicAdd(&acc[1][k], v1); atomicAdd(&acc[2][k], v2);
                        atomicAdd(&acc[3][k], v3); atomicAdd(&acc[4][k], v4); atomicAdd(&acc[5][k], v5);
                        atomicAdd(&acc[6][k], v6); atomicAdd(&acc[7][k], v7); atomicAdd(&acc[8][k], v8);
                    }
                }
            }
        }
        __syncthreads();
        // flush: record gradients d/d(u, v, A, B, C, o, r, g, b) with the
        // conic unscaled (A = -2 A'/log2 e, B = -B'/log2 e, C = -2 C'/log2 e)
        for (int k = threadIdx.x; k < m; k += NT) {
            const float s4 = acc[4][k], s5 = acc[5][k], s6 = acc[6][k], s7 = acc[7][k], s8 = acc[8][k];
            const float s3 = acc[3][k], s0 = acc[0][k], s1 = acc[1][k], s2 = acc[2][k];
            for (int c = 0; c < 9; ++c) acc[c][k] = 0.0f;
            if (s0 == 0.0f && s1 == 0.0f && s2 == 0.0f && s3 == 0.0f && s4 == 0.0f && s5 == 0.0f &&
                s6 == 0.0f && s7 == 0.0f && s8 == 0.0f)
                continue;
            const float4 b = sb[k];
            const float A = -2.0f * b.x / kLog2e, B = -b.y / kLog2e, C = -2.0f * b.z / kLog2e;
            const uint32_t r = srec[k];
            // dQ/ddx = 2(A dx + B dy), ddx/du = -1
            atomicAdd(rec_grad + 0 * R + r, -2.0f * (A * s7 + B * s8));
            atomicAdd(rec_grad + 1 * R + r, -2.0f * (B * s7 + C * s8));
            atomicAdd(rec_grad + 2 * R + r, s4);
            atomicAdd(rec_grad + 3 * R + r, 2.0f * s5);
            atomicAdd(rec_grad + 4 * R + r, s6);
            atomicAdd(rec_grad + 5 * R + r, s3);
            atomicAdd(rec_grad + 6 * R + r, s0);
            atomicAdd(rec_grad + 7 * R + r, s1);
            atomicAdd(rec_grad + 8 * R + r, s2);
        }
        __syncthreads();
        b_end = b_start;
    }
}

__global__ void __launch_bounds__(256)
k_loss_reduce(const double *__restrict__ part, int nparts, double inv_3p, double *__restrict__ stats) {
    __shared__ double sa[256], sb[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) {
        a += part[2 * (size_t)i];
        b += part[2 * (size_t)i + 1];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            sb[threadIdx.x] += sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stats[0] = sa[0];
        stats[1] = sb[0] * inv_3p;
    }
}

template <int TW, int TH, int BATCH>
void fwd_launch(hipStream_t s, const swgs_plan &p, uint8_t *ws, float *images, const float *targets,
                uint32_t tile_lo, uint32_t tile_hi, unsigned long long *counters) {
    hipLaunchKernelGGL((k_blend_fwd<TW, TH, BATCH>), dim3(tile_hi - tile_lo), dim3(TW * TH), 0, s,
                       wsp<uint2>(ws, p, WB_TILE_RANGE), wsp<uint32_t>(ws, p, WB_PAIR_VAL),
                       wsp<float4>(ws, p, WB_SPLAT), wsp<ViewDev>(ws, p, WB_VIEWS),
                       (int)p.views.size(), tile_lo, images, wsp<float>(ws, p, WB_T_FINAL),
                       wsp<uint32_t>(ws, p, WB_LAST), targets, wsp<float>(ws, p, WB_DLDC),
                       wsp<double>(ws, p, WB_LOSS_PART) + 2 * (size_t)tile_lo, counters);
}

template <int TW, int TH, int BATCH>
void bwd_launch(hipStream_t s, const swgs_plan &p, uint8_t *ws, const float *dLdC, uint32_t tile_lo,
                uint32_t tile_hi, unsigned long long *counters) {
    hipLaunchKernelGGL((k_blend_bwd<TW, TH, BATCH>), dim3(tile_hi - tile_lo), dim3(TW * TH), 0, s,
                       wsp<uint2>(ws, p, WB_TILE_RANGE), wsp<uint32_t>(ws, p, WB_PAIR_VAL),
                       wsp<float4>(ws, p, WB_SPLAT), wsp<ViewDev>(ws, p, WB_VIEWS),
                       (int)p.views.size(), tile_lo, wsp<float>(ws, p, WB_T_FINAL),
                       wsp<uint32_t>(ws, p, WB_LAST), dLdC, wsp<float>(ws, p, WB_REC_GRAD), (size_t)p.R, counters);
}

}  // namespace

#define SWGS_DISPATCH_TILE(FN, ...)                                                        \
    do {                                                                                  \
        const int tw = p.tile_w, th = p.tile_h, lb = p.lds_batch;                         \
        if (tw == 16 && th == 16) {                                                       \
            if (lb == 128) FN<16, 16, 128>(__VA_ARGS__); else FN<16, 16, 256>(__VA_ARGS__); \
        } else if (tw == 8 && th == 8) {                                                  \
            if (lb == 128) FN<8, 8, 128>(__VA_ARGS__);                                    \
            else if (lb == 256) FN<8, 8, 256>(__VA_ARGS__); else FN<8, 8, 64>(__VA_ARGS__); \
        } else {                                                                          \
            if (lb == 128) FN<32, 8, 128>(__VA_ARGS__); else FN<32, 8, 256>(__VA_ARGS__);  \
        }                                                                                 \
    } while (0)

void launch_blend_forward(hipStream_t s, const swgs_plan &p, uint8_t *ws, float *images,
                          const float *targets, uint32_t tile_lo, uint32_t tile_hi,
                          unsigned long long *counters) {
    if (tile_hi <= tile_lo) return;
    SWGS_DISPATCH_TILE(fwd_launch, s, p, ws, images, targets, tile_lo, tile_hi, counters);
}

void launch_blend_backward(hipStream_t s, const swgs_plan &p, uint8_t *ws, const float *dLdC,
                           uint32_t tile_lo, uint32_t tile_hi, unsigned long long *counters) {
    if (tile_hi <= tile_lo) return;
    SWGS_DISPATCH_TILE(bwd_launch, s, p, ws, dLdC, tile_lo, tile_hi, counters);
}

void launch_loss_reduce(hipStream_t s, const swgs_plan &p, uint8_t *ws, const swgs_step_cfg *cfg,
                        bool with_reg) {
    (void)cfg;
    (void)with_reg;
    hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(256), 0, s, wsp<double>(ws, p, WB_LOSS_PART), (int)p.T,
                       1.0 / (3.0 * (double)p.P), wsp<double>(ws, p, WB_STATS));
}

}  // namespace swgs

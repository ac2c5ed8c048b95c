// D-SSIM image term of the window loss and its gradient.
//
// The loss follows 3DGS-MCMC's practice (Sec. 4.4): per view,
// (1 - lambda) mean|C - GT| + lambda (1 - SSIM(C, GT)), averaged over the
// views.  SSIM is the structural similarity of Wang et al. (2004): an 11x11
// Gaussian window (sigma 1.5, weights summing to 1, zero outside the image)
// gives the local means mu_x, mu_y and second moments E[x^2], E[y^2], E[xy];
// per pixel
//     S = (2 mu_x mu_y + C1)(2 cov_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(var_x + var_y + C2))
// with C1 = 0.01^2, C2 = 0.03^2; SSIM is the mean of S over pixels and
// channels.
//
// k_ssim_fwd: one workgroup per (16x16 output tile, channel) stages the
// 26x26 neighbourhood of C and GT in LDS, runs the separable 11-tap window
// (rows, then columns) over x, y, x^2, y^2, xy, and writes per pixel the
// partial derivatives of S with respect to mu_x, E[x^2] and E[xy], plus the
// tile's sum of S weighted for the loss.
// k_ssim_bwd: the window is symmetric, so the adjoint of a window sum is the
// same window sum; it is applied to the three partial maps and
//     dSSIM/dx(q) = (W*Sm)(q) + 2 x(q) (W*Sxx)(q) + y(q) (W*Sxy)(q)
// (divided by the view's 3HW) is added, times -lambda / V, into dL/dC.
#include <cmath>

#include "swgs_internal.h"

namespace swgs {
namespace {

constexpr int kT = 16;                 // output tile
constexpr int kR = 5;                  // window radius
constexpr int kH = kT + 2 * kR;        // staged neighbourhood
constexpr float kC1 = 1e-4f, kC2 = 9e-4f;

// 1D Gaussian weights (sigma 1.5, normalised), computed once on the host
struct Taps {
    float w[2 * kR + 1];
};

// view owning an SSIM tile
__device__ __forceinline__ int view_of_ssim_tile(const ViewDev *views, int n_views, uint32_t t) {
    int a = 0, b = n_views;
    while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (views[m].ssim_tile_base <= t) a = m; else b = m;
    }
    return a;
}

// Both kernels work in two separable passes over the staged neighbourhood,
// two outputs per thread to cut LDS traffic: the row pass makes outputs
// (r, c0), (r, c0 + 1) of every staged row from 12 staged columns; the
// column pass makes outputs (r0, c), (r0 + 1, c) from 12 row sums.
constexpr int kRowItems = kH * (kT / 2);   // row-pass work items (208)
constexpr int kColItems = (kT / 2) * kT;   // column-pass work items (128)

__global__ void __launch_bounds__(kT *kT)
k_ssim_fwd(const ViewDev *__restrict__ views, int n_views, uint32_t t_lo, const float *__restrict__ img,
           const float *__restrict__ tgt, float *__restrict__ part, double *__restrict__ tile_sum, float lambda,
           Taps taps) {
    __shared__ __align__(16) float2 sxy[kH][kH];               // (x, y) over the staged neighbourhood
    __shared__ __align__(16) float4 hq[kH][kT];                // row sums of x, y, x^2, y^2
    __shared__ float hxy[kH][kT];                // row sums of x y
    __shared__ double red[kT * kT / 64];
    // work item (channel, tile), channel-major, dealt to the XCDs in
    // contiguous ranges so halo rows of neighbouring tiles share an L2
    const uint32_t nt = gridDim.x / 3;
    const uint32_t item = xcd_order(blockIdx.x, gridDim.x);
    const int ch = (int)(item / nt);
    const uint32_t t_local = item - (uint32_t)ch * nt;
    const uint32_t t = t_lo + t_local;
    const ViewDev &V = views[view_of_ssim_tile(views, n_views, t)];
    const uint32_t lt = t - V.ssim_tile_base;
    const int ntx = (V.width + kT - 1) / kT;
    const int x0 = (int)(lt % (uint32_t)ntx) * kT, y0 = (int)(lt / (uint32_t)ntx) * kT;
    const size_t HW = (size_t)V.width * V.height;
    const float *X = img + 3 * (size_t)V.pix_base + (size_t)ch * HW;
    const float *Y = tgt + 3 * (size_t)V.pix_base + (size_t)ch * HW;
    for (int i = threadIdx.x; i < kH * kH; i += kT * kT) {
        const int r = i / kH, c = i % kH;
        const int yy = y0 + r - kR, xx = x0 + c - kR;
        const bool in = xx >= 0 && xx < V.width && yy >= 0 && yy < V.height;
        const size_t o = (size_t)yy * V.width + xx;
        sxy[r][c] = make_float2(in ? X[o] : 0.0f, in ? Y[o] : 0.0f);
    }
    __syncthreads();
    if (threadIdx.x < kRowItems) {
        const int r = threadIdx.x / (kT / 2), c0 = 2 * (threadIdx.x % (kT / 2));
        float u[2 * kR + 2], v[2 * kR + 2];
#pragma unroll
        for (int k = 0; k < 2 * kR + 2; k += 2) {
            const float4 e = *reinterpret_cast<const float4 *>(&sxy[r][c0 + k]);
            u[k] = e.x; v[k] = e.y; u[k + 1] = e.z; v[k + 1] = e.w;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            float a = 0.0f, b = 0.0f, aa = 0.0f, bb = 0.0f, ab = 0.0f;
#pragma unroll
            for (int k = 0; k <= 2 * kR; ++k) {
                const float w = taps.w[k], uu = u[j + k], vv = v[j + k];
                a = fmaf(w, uu, a);
                b = fmaf(w, vv, b);
                aa = fmaf(w * uu, uu, aa);
                bb = fmaf(w * vv, vv, bb);
                ab = fmaf(w * uu, vv, ab);
            }
            hq[r][c0 + j] = make_float4(a, b, aa, bb);
            hxy[r][c0 + j] = ab;
        }
    }
    __syncthreads();
    double s_val = 0.0;
    if (threadIdx.x < kColItems) {
        const int c = threadIdx.x % kT, r0 = 2 * (threadIdx.x / kT);
        float4 q[2 * kR + 2];
        float e[2 * kR + 2];
#pragma unroll
        for (int k = 0; k < 2 * kR + 2; ++k) {
            q[k] = hq[r0 + k][c];
            e[k] = hxy[r0 + k][c];
        }
        float *P = part + 9 * (size_t)V.pix_base + (size_t)ch * 3 * HW;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            float mx = 0.0f, my = 0.0f, exx = 0.0f, eyy = 0.0f, exy = 0.0f;
#pragma unroll
            for (int k = 0; k <= 2 * kR; ++k) {
                const float w = taps.w[k];
                mx = fmaf(w, q[j + k].x, mx);
                my = fmaf(w, q[j + k].y, my);
                exx = fmaf(w, q[j + k].z, exx);
                eyy = fmaf(w, q[j + k].w, eyy);
                exy = fmaf(w, e[j + k], exy);
            }
            const int x = x0 + c, y = y0 + r0 + j;
            if (x < V.width && y < V.height) {
                const float A = 2.0f * mx * my + kC1;
                const float B = 2.0f * (exy - mx * my) + kC2;
                const float C = mx * mx + my * my + kC1;
                const float D = (exx - mx * mx) + (eyy - my * my) + kC2;
                const float rC = __builtin_amdgcn_rcpf(C), rD = __builtin_amdgcn_rcpf(D);
                const float rCD = rC * rD;
                const float S = A * B * rCD;
                const size_t o = (size_t)y * V.width + x;
                P[o] = 2.0f * my * (B - A) * rCD - 2.0f * mx * S * rC + 2.0f * mx * S * rD;
                P[o + HW] = -S * rD;
                P[o + 2 * HW] = 2.0f * A * rCD;
                s_val += (double)S;
            }
        }
    }
    // tile sum of S, weighted lambda / (V 3 H W) = lambda * inv_norm
    for (int o = 32; o > 0; o >>= 1) s_val += __shfl_xor(s_val, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s_val;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int w = 0; w < kT * kT / 64; ++w) a += red[w];
        tile_sum[3 * (size_t)t_local + ch] = a * (double)lambda * (double)V.inv_norm;
    }
}

__global__ void __launch_bounds__(kT *kT)
k_ssim_bwd(const ViewDev *__restrict__ views, int n_views, uint32_t t_lo, const float *__restrict__ img,
           const float *__restrict__ tgt, const float *__restrict__ part, float *__restrict__ dLdC,
           float lambda, Taps taps) {
    __shared__ __align__(16) float4 sp[kH][kH];                // the three map derivatives (w unused)
    __shared__ __align__(16) float4 hs[kH][kT];                // their row sums
    const uint32_t nt = gridDim.x / 3;
    const uint32_t item = xcd_order(blockIdx.x, gridDim.x);
    const int ch = (int)(item / nt);
    const uint32_t t = t_lo + (item - (uint32_t)ch * nt);
    const ViewDev &V = views[view_of_ssim_tile(views, n_views, t)];
    const uint32_t lt = t - V.ssim_tile_base;
    const int ntx = (V.width + kT - 1) / kT;
    const int x0 = (int)(lt % (uint32_t)ntx) * kT, y0 = (int)(lt / (uint32_t)ntx) * kT;
    const size_t HW = (size_t)V.width * V.height;
    const float *P = part + 9 * (size_t)V.pix_base + (size_t)ch * 3 * HW;
    for (int i = threadIdx.x; i < kH * kH; i += kT * kT) {
        const int r = i / kH, c = i % kH;
        const int yy = y0 + r - kR, xx = x0 + c - kR;
        const bool in = xx >= 0 && xx < V.width && yy >= 0 && yy < V.height;
        const size_t o = (size_t)yy * V.width + xx;
        sp[r][c] = in ? make_float4(P[o], P[o + HW], P[o + 2 * HW], 0.0f) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    __syncthreads();
    if (threadIdx.x < kRowItems) {
        const int r = threadIdx.x / (kT / 2), c0 = 2 * (threadIdx.x % (kT / 2));
        float4 e[2 * kR + 2];
#pragma unroll
        for (int k = 0; k < 2 * kR + 2; ++k) e[k] = sp[r][c0 + k];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            float a = 0.0f, b = 0.0f, g = 0.0f;
#pragma unroll
            for (int k = 0; k <= 2 * kR; ++k) {
                const float w = taps.w[k];
                a = fmaf(w, e[j + k].x, a);
                b = fmaf(w, e[j + k].y, b);
                g = fmaf(w, e[j + k].z, g);
            }
            hs[r][c0 + j] = make_float4(a, b, g, 0.0f);
        }
    }
    __syncthreads();
    if (threadIdx.x >= kColItems) return;
    const int c = threadIdx.x % kT, r0 = 2 * (threadIdx.x / kT);
    float4 q[2 * kR + 2];
#pragma unroll
    for (int k = 0; k < 2 * kR + 2; ++k) q[k] = hs[r0 + k][c];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        float a = 0.0f, b = 0.0f, g = 0.0f;
#pragma unroll
        for (int k = 0; k <= 2 * kR; ++k) {
            const float w = taps.w[k];
            a = fmaf(w, q[j + k].x, a);
            b = fmaf(w, q[j + k].y, b);
            g = fmaf(w, q[j + k].z, g);
        }
        const int x = x0 + c, y = y0 + r0 + j;
        if (x >= V.width || y >= V.height) continue;
        const size_t o = 3 * (size_t)V.pix_base + (size_t)ch * HW + (size_t)y * V.width + x;
        // d/dC of lambda (1 - SSIM_v) / V with SSIM_v = sum S / (3 H W):
        // -lambda inv_norm (W*Sm + 2 x W*Sxx + y W*Sxy), inv_norm = 1 / (V 3 H W)
        dLdC[o] -= lambda * V.inv_norm * (a + 2.0f * img[o] * b + tgt[o] * g);
    }
}

// sum of the tile sums (fixed chunks, then one block): lambda * mean SSIM over views
constexpr int kSumBlocks = 256;

__device__ __forceinline__ double block_sum(double a) {
    __shared__ double sa[256];
    sa[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sa[threadIdx.x] += sa[threadIdx.x + s];
        __syncthreads();
    }
    return sa[0];
}

__global__ void __launch_bounds__(256)
k_ssim_partial(const double *__restrict__ tile_sum, int n, double *__restrict__ sums) {
    const int chunk = (n + kSumBlocks - 1) / kSumBlocks;
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double a = 0.0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += 256) a += tile_sum[i];
    a = block_sum(a);
    if (threadIdx.x == 0) sums[blockIdx.x] = a;
}

// stats[0] (image loss) += lambda - lambda * mean_v SSIM_v
__global__ void __launch_bounds__(256)
k_ssim_final(const double *__restrict__ sums, double lambda, double *__restrict__ stats) {
    const double a = block_sum(sums[threadIdx.x]);
    if (threadIdx.x == 0) stats[0] += lambda - a;
}

Taps window_taps() {
    Taps t;
    double w[2 * kR + 1], sum = 0.0;
    for (int k = -kR; k <= kR; ++k) sum += (w[k + kR] = std::exp(-(double)(k * k) / (2.0 * 1.5 * 1.5)));
    for (int k = 0; k <= 2 * kR; ++k) t.w[k] = (float)(w[k] / sum);
    return t;
}

}  // namespace

size_t ssim_tiles(int width, int height) {
    return (size_t)((width + kT - 1) / kT) * (size_t)((height + kT - 1) / kT);
}

void launch_ssim(hipStream_t s, const swgs_plan &p, uint8_t *ws, int view_lo, int view_hi, const float *images,
                 const float *targets, float lambda) {
    if (!images || !targets) return;   // callers always pass both (the window step renders into the workspace)
    const uint32_t t_lo = p.vdev[view_lo].ssim_tile_base;
    const uint32_t t_hi = view_hi < (int)p.views.size() ? p.vdev[view_hi].ssim_tile_base : (uint32_t)p.T16;
    if (t_hi <= t_lo) return;
    const dim3 grid(3 * (t_hi - t_lo));
    double *tsum = wsp<double>(ws, p, WB_SSIM_SUM);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(kT * kT), 0, s, wsp<ViewDev>(ws, p, WB_VIEWS), (int)p.views.size(),
                       t_lo, images, targets, wsp<float>(ws, p, WB_SSIM_PART), tsum + 3 * (size_t)t_lo, lambda,
                       window_taps());
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(kT * kT), 0, s, wsp<ViewDev>(ws, p, WB_VIEWS), (int)p.views.size(),
                       t_lo, images, targets, wsp<float>(ws, p, WB_SSIM_PART), wsp<float>(ws, p, WB_DLDC), lambda,
                       window_taps());
}

void launch_ssim_reduce(hipStream_t s, const swgs_plan &p, uint8_t *ws, float lambda) {
    double *tsum = wsp<double>(ws, p, WB_SSIM_SUM);
    const int n = 3 * (int)p.T16;
    double *sums = tsum + n;
    hipLaunchKernelGGL(k_ssim_partial, dim3(kSumBlocks), dim3(256), 0, s, tsum, n, sums);
    hipLaunchKernelGGL(k_ssim_final, dim3(1), dim3(256), 0, s, sums, (double)lambda, wsp<double>(ws, p, WB_STATS));
}

}  // namespace swgs

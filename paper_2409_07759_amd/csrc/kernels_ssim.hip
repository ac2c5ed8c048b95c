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

__global__ void __launch_bounds__(kT *kT)
k_ssim_fwd(const ViewDev *__restrict__ views, int n_views, uint32_t t_lo, const float *__restrict__ img,
           const float *__restrict__ tgt, float *__restrict__ part, double *__restrict__ tile_sum, float lambda,
           Taps taps) {
    __shared__ float sq[5][kH][kH];      // x, y, x^2, y^2, x y over the staged neighbourhood
    __shared__ float hsum[5][kH][kT];
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
        const float u = in ? X[o] : 0.0f, v = in ? Y[o] : 0.0f;
        sq[0][r][c] = u;
        sq[1][r][c] = v;
        sq[2][r][c] = u * u;
        sq[3][r][c] = v * v;
        sq[4][r][c] = u * v;
    }
    __syncthreads();
    // rows: horizontal window for the kH staged rows
    for (int i = threadIdx.x; i < kH * kT; i += kT * kT) {
        const int r = i / kT, c = i % kT;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            float a = 0.0f;
#pragma unroll
            for (int k = 0; k <= 2 * kR; ++k) a = fmaf(taps.w[k], sq[q][r][c + k], a);
            hsum[q][r][c] = a;
        }
    }
    __syncthreads();
    const int lx = threadIdx.x % kT, ly = threadIdx.x / kT;
    float m[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        float a = 0.0f;
#pragma unroll
        for (int k = 0; k <= 2 * kR; ++k) a = fmaf(taps.w[k], hsum[q][ly + k][lx], a);
        m[q] = a;
    }
    const float mx = m[0], my = m[1], exx = m[2], eyy = m[3], exy = m[4];
    const int x = x0 + lx, y = y0 + ly;
    double s_val = 0.0;
    if (x < V.width && y < V.height) {
        const float A = 2.0f * mx * my + kC1;
        const float B = 2.0f * (exy - mx * my) + kC2;
        const float C = mx * mx + my * my + kC1;
        const float D = (exx - mx * mx) + (eyy - my * my) + kC2;
        const float rC = __builtin_amdgcn_rcpf(C), rD = __builtin_amdgcn_rcpf(D);
        const float rCD = rC * rD;
        const float S = A * B * rCD;
        const size_t o = (size_t)ch * 3 * HW + (size_t)y * V.width + x;
        float *P = part + 9 * (size_t)V.pix_base;
        P[o] = 2.0f * my * (B - A) * rCD - 2.0f * mx * S * rC + 2.0f * mx * S * rD;
        P[o + HW] = -S * rD;
        P[o + 2 * HW] = 2.0f * A * rCD;
        s_val = (double)S;
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
    __shared__ float sp[3][kH][kH];
    __shared__ float hsum[3][kH][kT];
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
    const float *P = part + 9 * (size_t)V.pix_base + (size_t)ch * 3 * HW;
    for (int i = threadIdx.x; i < kH * kH; i += kT * kT) {
        const int r = i / kH, c = i % kH;
        const int yy = y0 + r - kR, xx = x0 + c - kR;
        const bool in = xx >= 0 && xx < V.width && yy >= 0 && yy < V.height;
        const size_t o = (size_t)yy * V.width + xx;
        sp[0][r][c] = in ? P[o] : 0.0f;
        sp[1][r][c] = in ? P[o + HW] : 0.0f;
        sp[2][r][c] = in ? P[o + 2 * HW] : 0.0f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kH * kT; i += kT * kT) {
        const int r = i / kT, c = i % kT;
        float a = 0.0f, b = 0.0f, e = 0.0f;
#pragma unroll
        for (int k = 0; k <= 2 * kR; ++k) {
            const float w = taps.w[k];
            a = fmaf(w, sp[0][r][c + k], a);
            b = fmaf(w, sp[1][r][c + k], b);
            e = fmaf(w, sp[2][r][c + k], e);
        }
        hsum[0][r][c] = a;
        hsum[1][r][c] = b;
        hsum[2][r][c] = e;
    }
    __syncthreads();
    const int lx = threadIdx.x % kT, ly = threadIdx.x / kT;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= V.width || y >= V.height) return;
    float a = 0.0f, b = 0.0f, e = 0.0f;
#pragma unroll
    for (int k = 0; k <= 2 * kR; ++k) {
        const float w = taps.w[k];
        a = fmaf(w, hsum[0][ly + k][lx], a);
        b = fmaf(w, hsum[1][ly + k][lx], b);
        e = fmaf(w, hsum[2][ly + k][lx], e);
    }
    const size_t o = 3 * (size_t)V.pix_base + (size_t)ch * HW + (size_t)y * V.width + x;
    const float xv = img[o], yv = tgt[o];
    // d/dC of lambda (1 - SSIM_v) / V with SSIM_v = sum S / (3 H W):
    // -lambda inv_norm (W*Sm + 2 x W*Sxx + y W*Sxy), inv_norm = 1 / (V 3 H W)
    dLdC[o] -= lambda * V.inv_norm * (a + 2.0f * xv * b + yv * e);
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

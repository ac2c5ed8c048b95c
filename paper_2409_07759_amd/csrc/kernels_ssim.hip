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
// k_ssim_fwd: one workgroup per (32x32 output tile, channel) stages the
// 42x42 neighbourhood of C and GT in LDS, runs the separable 11-tap window
// (rows, then columns) over x, y, x^2 + y^2 and xy (S takes E[x^2] and
// E[y^2] only through their sum, in var_x + var_y), and writes per pixel the
// partial derivatives of S with respect to mu_x, E[x^2] and E[xy], plus the
// tile's sum of S weighted for the loss.  In both kernels the staged inputs
// and the row sums share one LDS buffer: the row pass holds its sums in
// registers until every thread is done reading the staging.
// k_ssim_bwd: the window is symmetric, so the adjoint of a window sum is the
// same window sum; it is applied to the three partial maps and
//     dSSIM/dx(q) = (W*Sm)(q) + 2 x(q) (W*Sxx)(q) + y(q) (W*Sxy)(q)
// (divided by the view's 3HW), times -lambda / V, plus the L1 term
// (1 - lambda) sign(x - y) / (V 3 H W), is written as dL/dC (the blend
// forward leaves dL/dC to this kernel when the loss has a D-SSIM term).
#include <cmath>

#include "swgs_internal.h"

namespace swgs {
namespace {

constexpr int kT = 32;                 // output tile
constexpr int kR = 5;                  // window radius
constexpr int kH = kT + 2 * kR;        // staged neighbourhood
constexpr int kW = 2 * kR + 1;         // taps
constexpr int kSeg = 4;                // outputs per work item (both passes)
constexpr int kSpan = kSeg + 2 * kR;   // inputs per work item
constexpr int kThreads = 256;
constexpr int kRowItems = kH * (kT / kSeg);   // row pass: every staged row x 8 segments (336)
constexpr int kColItems = kT * (kT / kSeg);   // column pass: 32 columns x 8 segments (256)
static_assert(kColItems == kThreads, "one column item per thread");
constexpr int kItemRounds = (kRowItems + kThreads - 1) / kThreads;   // row items per thread (2)
constexpr int kWaves = kThreads / 64;
constexpr int kStageRows = (kH + kWaves - 1) / kWaves;         // staged rows per wave (11)
static_assert(kH <= 64, "one lane per staged column");
// LDS row pitches: in the row pass consecutive lanes take consecutive rows,
// so a row's pitch in dwords is kept an odd multiple of 4 and the 16-byte
// accesses of 8 consecutive lanes fall on disjoint banks
constexpr int kHP = kH;                // forward staging (x, y): 84 dwords per row
constexpr int kPP = kH + 2;            // backward staging, one plane per map: 44 dwords per row
constexpr int kTP = kT + 1;            // row sums (float4): 132 dwords per row
constexpr int kLds = kH * kTP;         // float4 elements of the shared buffer (22176 B)
static_assert(kH * kHP * 2 <= 4 * kLds && 3 * kH * kPP <= 4 * kLds, "staging fits the shared buffer");
static_assert((kT - kSeg) + 16 <= kPP && kSpan <= 16, "16-float row reads stay in the plane row");
constexpr float kC1 = 1e-4f, kC2 = 9e-4f;

// 1D Gaussian weights (sigma 1.5, normalised), computed once on the host
struct Taps {
    float w[kW];
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

struct SsimTile {
    int ch, x0, y0;
    uint32_t t_local;
    const ViewDev *V;
};

// work item (channel, tile), channel-major, dealt to the XCDs in contiguous
// ranges so halo rows of neighbouring tiles share an L2
__device__ __forceinline__ SsimTile ssim_tile(const ViewDev *views, int n_views, uint32_t t_lo) {
    SsimTile r;
    const uint32_t nt = gridDim.x / 3;
    const uint32_t item = xcd_order(blockIdx.x, gridDim.x);
    r.ch = (int)(item / nt);
    r.t_local = item - (uint32_t)r.ch * nt;
    const uint32_t t = t_lo + r.t_local;
    r.V = &views[view_of_ssim_tile(views, n_views, t)];
    const uint32_t lt = t - r.V->ssim_tile_base;
    const int ntx = (r.V->width + kT - 1) / kT;
    r.x0 = (int)(lt % (uint32_t)ntx) * kT;
    r.y0 = (int)(lt / (uint32_t)ntx) * kT;
    return r;
}

// Both passes give each work item kSeg consecutive outputs from kSpan
// staged inputs, every input weighted into the outputs whose window holds
// it (taps in increasing order per output).
__global__ void __launch_bounds__(kThreads)
k_ssim_fwd(const ViewDev *__restrict__ views, int n_views, uint32_t t_lo, const float *__restrict__ img,
           const float *__restrict__ tgt, float *__restrict__ part, double *__restrict__ tile_sum, float lambda,
           Taps taps) {
    __shared__ __align__(16) float4 lds[kLds];
    __shared__ double red[kThreads / 64];
    float2(*sxy)[kHP] = reinterpret_cast<float2(*)[kHP]>(lds);   // (x, y) over the staged neighbourhood
    float4(*hq)[kTP] = reinterpret_cast<float4(*)[kTP]>(lds);    // row sums of x, y, x^2 + y^2, x y
    const SsimTile tl = ssim_tile(views, n_views, t_lo);
    const ViewDev &V = *tl.V;
    const size_t HW = (size_t)V.width * V.height;
    const float *X = img + 3 * (size_t)V.pix_base + (size_t)tl.ch * HW;
    const float *Y = tgt + 3 * (size_t)V.pix_base + (size_t)tl.ch * HW;
    {
        // lane l stages column l, wave w rows w, w + 4, ... (row offsets and
        // row bounds are wave-uniform); all of a thread's loads are in
        // flight before its LDS stores
        const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int xx = tl.x0 + lane - kR;
        const bool col = lane < kH && xx >= 0 && xx < V.width;
        const uint32_t cx = col ? (uint32_t)xx : 0u;
        float2 v[kStageRows];
#pragma unroll
        for (int u = 0; u < kStageRows; ++u) {
            const int r = wave + kWaves * u, yy = tl.y0 + r - kR;
            const bool row = r < kH && yy >= 0 && yy < V.height;   // wave-uniform
            // every load in bounds (pixel 0 outside the image), no branch
            const uint32_t o = col && row ? (uint32_t)yy * (uint32_t)V.width + cx : 0u;
            const float xv = X[o], yv = Y[o];
            v[u] = make_float2(col && row ? xv : 0.0f, col && row ? yv : 0.0f);
        }
#pragma unroll
        for (int u = 0; u < kStageRows; ++u) {
            const int r = wave + kWaves * u;
            if (lane < kH && r < kH) sxy[r][lane] = v[u];
        }
    }
    __syncthreads();
    float4 rs[kItemRounds][kSeg];
#pragma unroll
    for (int u = 0; u < kItemRounds; ++u) {
        const int it = threadIdx.x + u * kThreads;
        if (it >= kRowItems) break;
        const int r = it % kH, c0 = kSeg * (it / kH);    // consecutive lanes: consecutive rows
        float a[kSeg], b[kSeg], ss[kSeg], ab[kSeg];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) a[j] = b[j] = ss[j] = ab[j] = 0.0f;
#pragma unroll
        for (int p = 0; p < kSpan; p += 2) {
            const float4 e = *reinterpret_cast<const float4 *>(&sxy[r][c0 + p]);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float x = h ? e.z : e.x, y = h ? e.w : e.y;
                const float sq = fmaf(x, x, y * y), xy = x * y;
#pragma unroll
                for (int j = 0; j < kSeg; ++j) {
                    const int k = p + h - j;
                    if (k < 0 || k >= kW) continue;
                    const float w = taps.w[k];
                    a[j] = fmaf(w, x, a[j]);
                    b[j] = fmaf(w, y, b[j]);
                    ss[j] = fmaf(w, sq, ss[j]);
                    ab[j] = fmaf(w, xy, ab[j]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kSeg; ++j) rs[u][j] = make_float4(a[j], b[j], ss[j], ab[j]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kItemRounds; ++u) {
        const int it = threadIdx.x + u * kThreads;
        if (it >= kRowItems) break;
        const int r = it % kH, c0 = kSeg * (it / kH);
#pragma unroll
        for (int j = 0; j < kSeg; ++j) hq[r][c0 + j] = rs[u][j];
    }
    __syncthreads();
    float s_thr = 0.0f;   // this thread's (at most four) S values
    {
        const int c = threadIdx.x % kT, r0 = kSeg * (threadIdx.x / kT);
        float mx[kSeg], my[kSeg], ess[kSeg], exy[kSeg];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) mx[j] = my[j] = ess[j] = exy[j] = 0.0f;
#pragma unroll
        for (int p = 0; p < kSpan; ++p) {
            const float4 q = hq[r0 + p][c];
#pragma unroll
            for (int j = 0; j < kSeg; ++j) {
                const int k = p - j;
                if (k < 0 || k >= kW) continue;
                const float w = taps.w[k];
                mx[j] = fmaf(w, q.x, mx[j]);
                my[j] = fmaf(w, q.y, my[j]);
                ess[j] = fmaf(w, q.z, ess[j]);
                exy[j] = fmaf(w, q.w, exy[j]);
            }
        }
        float *P = part + 9 * (size_t)V.pix_base + (size_t)tl.ch * 3 * HW;
        const int x = tl.x0 + c;
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            const int y = tl.y0 + r0 + j;
            if (x >= V.width || y >= V.height) continue;
            const float mxy = mx[j] * my[j], m2 = mx[j] * mx[j] + my[j] * my[j];
            const float A = 2.0f * mxy + kC1;
            const float B = 2.0f * (exy[j] - mxy) + kC2;
            const float C = m2 + kC1;
            const float D = (ess[j] - m2) + kC2;               // var_x + var_y + C2
            const float rC = __builtin_amdgcn_rcpf(C), rD = __builtin_amdgcn_rcpf(D);
            const float rCD = rC * rD;
            const float S = A * B * rCD;
            const size_t o = (size_t)y * V.width + x;
            P[o] = 2.0f * my[j] * (B - A) * rCD - 2.0f * mx[j] * S * rC + 2.0f * mx[j] * S * rD;
            P[o + HW] = -S * rD;
            P[o + 2 * HW] = 2.0f * A * rCD;
            s_thr += S;
        }
    }
    // tile sum of S, weighted lambda / (V 3 H W) = lambda * inv_norm
    double s_val = (double)s_thr;
    for (int o = 32; o > 0; o >>= 1) s_val += __shfl_xor(s_val, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s_val;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) acc += red[w];
        tile_sum[3 * (size_t)tl.t_local + tl.ch] = acc * (double)lambda * (double)V.inv_norm;
    }
}

__global__ void __launch_bounds__(kThreads)
k_ssim_bwd(const ViewDev *__restrict__ views, int n_views, uint32_t t_lo, const float *__restrict__ img,
           const float *__restrict__ tgt, const float *__restrict__ part, float *__restrict__ dLdC,
           float lambda, float l1_weight, Taps taps) {
    __shared__ __align__(16) float4 lds[kLds];
    float(*sp)[kH][kPP] = reinterpret_cast<float(*)[kH][kPP]>(lds);   // the three map derivatives, planar
    float4(*hs)[kTP] = reinterpret_cast<float4(*)[kTP]>(lds);         // their row sums (w unused)
    const SsimTile tl = ssim_tile(views, n_views, t_lo);
    const ViewDev &V = *tl.V;
    const size_t HW = (size_t)V.width * V.height;
    const float *P = part + 9 * (size_t)V.pix_base + (size_t)tl.ch * 3 * HW;
    {
        // staged as in the forward: lane l column l, wave w rows w, w + 4, ...
        const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int xx = tl.x0 + lane - kR;
        const bool col = lane < kH && xx >= 0 && xx < V.width;
        const uint32_t cx = col ? (uint32_t)xx : 0u;
        float v[3][kStageRows];
#pragma unroll
        for (int u = 0; u < kStageRows; ++u) {
            const int r = wave + kWaves * u, yy = tl.y0 + r - kR;
            const bool row = r < kH && yy >= 0 && yy < V.height;   // wave-uniform
            // every load in bounds (pixel 0 outside the image), no branch
            const uint32_t o = col && row ? (uint32_t)yy * (uint32_t)V.width + cx : 0u;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const float pv = P[(size_t)m * HW + o];
                v[m][u] = col && row ? pv : 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < kStageRows; ++u) {
            const int r = wave + kWaves * u;
            if (lane >= kH || r >= kH) continue;
#pragma unroll
            for (int m = 0; m < 3; ++m) sp[m][r][lane] = v[m][u];
        }
    }
    __syncthreads();
    float4 rs[kItemRounds][kSeg];
#pragma unroll
    for (int u = 0; u < kItemRounds; ++u) {
        const int it = threadIdx.x + u * kThreads;
        if (it >= kRowItems) break;
        const int r = it % kH, c0 = kSeg * (it / kH);    // consecutive lanes: consecutive rows
        float acc[3][kSeg];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            // the item's kSpan inputs of plane m as four 16-byte reads (the
            // last two floats are not used)
            float e[16];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 f = *reinterpret_cast<const float4 *>(&sp[m][r][c0 + 4 * q]);
                e[4 * q] = f.x;
                e[4 * q + 1] = f.y;
                e[4 * q + 2] = f.z;
                e[4 * q + 3] = f.w;
            }
#pragma unroll
            for (int j = 0; j < kSeg; ++j) {
                float t = 0.0f;
#pragma unroll
                for (int k = 0; k < kW; ++k) t = fmaf(taps.w[k], e[j + k], t);
                acc[m][j] = t;
            }
        }
#pragma unroll
        for (int j = 0; j < kSeg; ++j) rs[u][j] = make_float4(acc[0][j], acc[1][j], acc[2][j], 0.0f);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kItemRounds; ++u) {
        const int it = threadIdx.x + u * kThreads;
        if (it >= kRowItems) break;
        const int r = it % kH, c0 = kSeg * (it / kH);
#pragma unroll
        for (int j = 0; j < kSeg; ++j) hs[r][c0 + j] = rs[u][j];
    }
    __syncthreads();
    const int c = threadIdx.x % kT, r0 = kSeg * (threadIdx.x / kT);
    const int x = tl.x0 + c;
    // this thread's pixels: their image and target loads go out before the
    // column pass
    size_t o[kSeg];
    float xi[kSeg], ti[kSeg];
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        const int y = tl.y0 + r0 + j;
        const bool in = x < V.width && y < V.height;
        // (out of the image: the view's first pixel, loaded and not used)
        o[j] = 3 * (size_t)V.pix_base + (size_t)tl.ch * HW + (in ? (size_t)y * V.width + x : 0);
        const float xv = img[o[j]], tv = tgt[o[j]];
        xi[j] = in ? xv : 0.0f;
        ti[j] = in ? tv : 0.0f;
    }
    float a[kSeg], b[kSeg], g[kSeg];
#pragma unroll
    for (int j = 0; j < kSeg; ++j) a[j] = b[j] = g[j] = 0.0f;
#pragma unroll
    for (int p = 0; p < kSpan; ++p) {
        const float4 q = hs[r0 + p][c];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            const int k = p - j;
            if (k < 0 || k >= kW) continue;
            const float w = taps.w[k];
            a[j] = fmaf(w, q.x, a[j]);
            b[j] = fmaf(w, q.y, b[j]);
            g[j] = fmaf(w, q.z, g[j]);
        }
    }
    if (x >= V.width) return;
    const float scale = lambda * V.inv_norm, s1 = V.inv_norm * l1_weight;
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        if (tl.y0 + r0 + j >= V.height) continue;
        // the L1 term as the blend forward forms it (the same FP32 values
        // and operations), then d/dC of lambda (1 - SSIM_v) / V with
        // SSIM_v = sum S / (3 H W): -lambda inv_norm (W*Sm + 2 x W*Sxx +
        // y W*Sxy), inv_norm = 1 / (V 3 H W)
        const float d = xi[j] - ti[j];
        const float gl1 = d > 0.0f ? s1 : (d < 0.0f ? -s1 : 0.0f);
        dLdC[o[j]] = gl1 - scale * (a[j] + 2.0f * xi[j] * b[j] + ti[j] * g[j]);
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
    double w[kW], sum = 0.0;
    for (int k = -kR; k <= kR; ++k) sum += (w[k + kR] = std::exp(-(double)(k * k) / (2.0 * 1.5 * 1.5)));
    for (int k = 0; k < kW; ++k) t.w[k] = (float)(w[k] / sum);
    return t;
}

}  // namespace

size_t ssim_tiles(int width, int height) {
    return (size_t)((width + kT - 1) / kT) * (size_t)((height + kT - 1) / kT);
}

void launch_ssim(hipStream_t s, const swgs_plan &p, uint8_t *ws, int view_lo, int view_hi, const float *images,
                 const float *targets, float lambda, float l1_weight) {
    if (!images || !targets) return;   // callers always pass both (the window step renders into the workspace)
    const uint32_t t_lo = p.vdev[view_lo].ssim_tile_base;
    const uint32_t t_hi = view_hi < (int)p.views.size() ? p.vdev[view_hi].ssim_tile_base : (uint32_t)p.Tssim;
    if (t_hi <= t_lo) return;
    const dim3 grid(3 * (t_hi - t_lo));
    double *tsum = wsp<double>(ws, p, WB_SSIM_SUM);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(kThreads), 0, s, wsp<ViewDev>(ws, p, WB_VIEWS), (int)p.views.size(),
                       t_lo, images, targets, wsp<float>(ws, p, WB_SSIM_PART), tsum + 3 * (size_t)t_lo, lambda,
                       window_taps());
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(kThreads), 0, s, wsp<ViewDev>(ws, p, WB_VIEWS), (int)p.views.size(),
                       t_lo, images, targets, wsp<float>(ws, p, WB_SSIM_PART), wsp<float>(ws, p, WB_DLDC), lambda,
                       l1_weight, window_taps());
}

void launch_ssim_reduce(hipStream_t s, const swgs_plan &p, uint8_t *ws, float lambda) {
    double *tsum = wsp<double>(ws, p, WB_SSIM_SUM);
    const int n = 3 * (int)p.Tssim;
    double *sums = tsum + n;
    hipLaunchKernelGGL(k_ssim_partial, dim3(kSumBlocks), dim3(256), 0, s, tsum, n, sums);
    hipLaunchKernelGGL(k_ssim_final, dim3(1), dim3(256), 0, s, sums, (double)lambda, wsp<double>(ws, p, WB_STATS));
}

}  // namespace swgs

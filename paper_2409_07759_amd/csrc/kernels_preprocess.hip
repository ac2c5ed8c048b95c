// Preprocess and binning.
//
// k_preprocess turns each live (frame group, slot) into one screen-space
// record per view of that frame: the 3D covariance R(q) diag(e^{2s}) R(q)^T
// of Eq. 2 projected by the EWA first-order approximation of the pinhole
// map (Sec. 2.1: the 3D Gaussian is sampled through its 2D projection), its
// conic, opacity, view-dependent SH colour, depth key and the tile range of
// its exact support {alpha >= 1/255}.  Parameters are read once per frame
// and reused for every camera of that frame.
//
// Arithmetic is FP64 (memory-bound kernel; gfx950 runs FP64 vector at half
// the FP32 rate), so every integer decision taken here -- culling, tile
// range, FP32 depth key -- is the FP64 decision, and the record values are
// correctly rounded FP32.  The screen position is stored split as
// (floor(u), 0.5 - frac(u)) so the blend computes pixel offsets to ~1e-7 px
// even at 1352-px widths.
#include "swgs_internal.h"

namespace swgs {
namespace {

constexpr int kBlock = 256;

// Real SH basis, degree <= 3, sign/order of the 3DGS renderer.
__device__ __forceinline__ void sh_basis64(int deg, double x, double y, double z, double *Y) {
    Y[0] = 0.28209479177387814;
    if (deg < 1) return;
    const double c1 = 0.4886025119029199;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (deg < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792 * x * y;
    Y[5] = -1.0925484305920792 * y * z;
    Y[6] = 0.31539156525252005 * (2.0 * zz - xx - yy);
    Y[7] = -1.0925484305920792 * x * z;
    Y[8] = 0.5462742152960396 * (xx - yy);
    if (deg < 3) return;
    Y[9] = -0.5900435899266435 * y * (3.0 * xx - yy);
    Y[10] = 2.890611442640554 * x * y * z;
    Y[11] = -0.4570457994644658 * y * (4.0 * zz - xx - yy);
    Y[12] = 0.3731763325901154 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -0.4570457994644658 * x * (4.0 * zz - xx - yy);
    Y[14] = 1.445305721320277 * z * (xx - yy);
    Y[15] = -0.5900435899266435 * x * (xx - 3.0 * yy);
}

// The same basis, each term added into the three channel sums as soon as it
// is formed (acc[c] += Y_k sh[3 k + c], k ascending: the sums of the loop
// over sh_basis64's terms, without holding all sixteen terms at once).
__device__ __forceinline__ void sh_accumulate64(int deg, double x, double y, double z, const float *sh,
                                                double *acc) {
    auto add = [&](int k, double yk) {
        acc[0] += yk * (double)sh[3 * k];
        acc[1] += yk * (double)sh[3 * k + 1];
        acc[2] += yk * (double)sh[3 * k + 2];
    };
    add(0, 0.28209479177387814);
    if (deg < 1) return;
    const double c1 = 0.4886025119029199;
    add(1, -c1 * y);
    add(2, c1 * z);
    add(3, -c1 * x);
    if (deg < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    add(4, 1.0925484305920792 * x * y);
    add(5, -1.0925484305920792 * y * z);
    add(6, 0.31539156525252005 * (2.0 * zz - xx - yy));
    add(7, -1.0925484305920792 * x * z);
    add(8, 0.5462742152960396 * (xx - yy));
    if (deg < 3) return;
    add(9, -0.5900435899266435 * y * (3.0 * xx - yy));
    add(10, 2.890611442640554 * x * y * z);
    add(11, -0.4570457994644658 * y * (4.0 * zz - xx - yy));
    add(12, 0.3731763325901154 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy));
    add(13, -0.4570457994644658 * x * (4.0 * zz - xx - yy));
    add(14, 1.445305721320277 * z * (xx - yy));
    add(15, -0.5900435899266435 * x * (xx - 3.0 * yy));
}

__device__ __forceinline__ int clip_tile(double f, int n) {
    return f < 0.0 ? 0 : (f > (double)n ? n : (int)f);
}

// HOIST_SH: load the slot's SH rows into registers once, before the camera
// loop (frames seen by several cameras); else per camera, after the
// basis (one camera per frame: fewer registers, higher occupancy).
// (With the SH rows in registers the kernel asks for three waves per SIMD:
// at most 168 VGPRs, a few spilled, against 202 and two waves otherwise.)
template <bool HOIST_SH>
__global__ void __launch_bounds__(kBlock, HOIST_SH ? 3 : 1)
k_preprocess(const float *__restrict__ params, int n_slots, int deg, const GroupDev *__restrict__ groups,
             const int32_t *__restrict__ group_views, const ViewDev *__restrict__ views,
             const uint32_t *__restrict__ lists, int g_lo, int only_view, int tile_w, int tile_h,
             float4 *__restrict__ splat, uint32_t *__restrict__ depth_key, uint32_t *__restrict__ tile_count,
             uint2 *__restrict__ rect, uint32_t *__restrict__ rec_idx, uint8_t *__restrict__ cflags) {
    const GroupDev G = groups[g_lo + blockIdx.y];
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= G.n_live) return;
    const size_t S = (size_t)n_slots;
    const uint32_t slot = lists[G.list_base + j];

    const double mx = params[0 * S + slot], my = params[1 * S + slot], mz = params[2 * S + slot];
    // Sigma = M M^T, M = R(q) diag(e^s)
    double qw = params[6 * S + slot], qx = params[7 * S + slot], qy = params[8 * S + slot], qz = params[9 * S + slot];
    const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qn; qx *= qn; qy *= qn; qz *= qn;
    const double s0 = exp((double)params[3 * S + slot]);
    const double s1 = exp((double)params[4 * S + slot]);
    const double s2 = exp((double)params[5 * S + slot]);
    const double r00 = 1.0 - 2.0 * (qy * qy + qz * qz), r01 = 2.0 * (qx * qy - qw * qz), r02 = 2.0 * (qx * qz + qw * qy);
    const double r10 = 2.0 * (qx * qy + qw * qz), r11 = 1.0 - 2.0 * (qx * qx + qz * qz), r12 = 2.0 * (qy * qz - qw * qx);
    const double r20 = 2.0 * (qx * qz - qw * qy), r21 = 2.0 * (qy * qz + qw * qx), r22 = 1.0 - 2.0 * (qx * qx + qy * qy);
    const double m00 = r00 * s0, m01 = r01 * s1, m02 = r02 * s2;
    const double m10 = r10 * s0, m11 = r11 * s1, m12 = r12 * s2;
    const double m20 = r20 * s0, m21 = r21 * s1, m22 = r22 * s2;
    const double S00 = m00 * m00 + m01 * m01 + m02 * m02;
    const double S01 = m00 * m10 + m01 * m11 + m02 * m12;
    const double S02 = m00 * m20 + m01 * m21 + m02 * m22;
    const double S11 = m10 * m10 + m11 * m11 + m12 * m12;
    const double S12 = m10 * m20 + m11 * m21 + m12 * m22;
    const double S22 = m20 * m20 + m21 * m21 + m22 * m22;

    const double op = 1.0 / (1.0 + exp(-(double)params[10 * S + slot]));
    const bool faint = 255.0 * op <= 1.0;
    const double kappa = faint ? 0.0 : 2.0 * log(255.0 * op);
    const int nk = (deg + 1) * (deg + 1);
    // the slot's SH coefficients, loaded once for all cameras (their loads
    // overlap the covariance arithmetic)
    float sh[HOIST_SH ? 48 : 1];
    if constexpr (HOIST_SH) {
#pragma unroll
        for (int q = 0; q < 48; ++q) sh[q] = q < 3 * nk ? params[(11 + q) * S + slot] : 0.0f;
    }

    for (int k = 0; k < G.n_views; ++k) {
        const int vi = group_views[G.view_first + k];
        if (only_view >= 0 && vi != only_view) continue;
        const ViewDev &V = views[vi];
        const uint32_t r = V.rec_base + j;
        rec_idx[r] = r;
        bool vis = !faint;
        // camera space
        const double px = V.R[0] * mx + V.R[1] * my + V.R[2] * mz + V.t[0];
        const double py = V.R[3] * mx + V.R[4] * my + V.R[5] * mz + V.t[1];
        const double pz = V.R[6] * mx + V.R[7] * my + V.R[8] * mz + V.t[2];
        vis = vis && pz > 0.2;
        double u = 0, v = 0, A = 0, B = 0, C = 0;
        int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
        uint32_t flags = 0;   // bits 0-2: rgb channel clamped at 0; bit 3/4: FoV clamp in x/y
        if (vis) {
            const double iz = 1.0 / pz;
            u = V.fx * px * iz + V.cx;
            v = V.fy * py * iz + V.cy;
            double tx = px * iz, ty = py * iz;
            flags |= (tx < -V.limx || tx > V.limx) ? 8u : 0u;
            flags |= (ty < -V.limy || ty > V.limy) ? 16u : 0u;
            tx = tx < -V.limx ? -V.limx : (tx > V.limx ? V.limx : tx);
            ty = ty < -V.limy ? -V.limy : (ty > V.limy ? V.limy : ty);
            // T = J R_view, J = [[fx/z, 0, -fx tx/z], [0, fy/z, -fy ty/z]]
            const double j00 = V.fx * iz, j02 = -V.fx * tx * iz;
            const double j11 = V.fy * iz, j12 = -V.fy * ty * iz;
            const double t00 = j00 * V.R[0] + j02 * V.R[6];
            const double t01 = j00 * V.R[1] + j02 * V.R[7];
            const double t02 = j00 * V.R[2] + j02 * V.R[8];
            const double t10 = j11 * V.R[3] + j12 * V.R[6];
            const double t11 = j11 * V.R[4] + j12 * V.R[7];
            const double t12 = j11 * V.R[5] + j12 * V.R[8];
            // Sigma T0, Sigma T1
            const double a0 = S00 * t00 + S01 * t01 + S02 * t02;
            const double a1 = S01 * t00 + S11 * t01 + S12 * t02;
            const double a2 = S02 * t00 + S12 * t01 + S22 * t02;
            const double b0 = S00 * t10 + S01 * t11 + S02 * t12;
            const double b1 = S01 * t10 + S11 * t11 + S12 * t12;
            const double b2 = S02 * t10 + S12 * t11 + S22 * t12;
            const double ca = t00 * a0 + t01 * a1 + t02 * a2 + 0.3;
            const double cb = t00 * b0 + t01 * b1 + t02 * b2;
            const double cc = t10 * b0 + t11 * b1 + t12 * b2 + 0.3;
            const double det = ca * cc - cb * cb;
            vis = det > 0.0;
            if (vis) {
                const double id = 1.0 / det;
                A = cc * id;
                B = -cb * id;
                C = ca * id;
                const double hx = sqrt(kappa * ca), hy = sqrt(kappa * cc);
                // tile sizes are powers of two: the product with the
                // reciprocal is the quotient exactly
                const double itw = 1.0 / (double)tile_w, ith = 1.0 / (double)tile_h;
                x0 = clip_tile(floor((u - hx - 1.0) * itw), V.tiles_x);
                x1 = clip_tile(floor((u + hx + 1.0) * itw) + 1.0, V.tiles_x);
                y0 = clip_tile(floor((v - hy - 1.0) * ith), V.tiles_y);
                y1 = clip_tile(floor((v + hy + 1.0) * ith) + 1.0, V.tiles_y);
                vis = x0 < x1 && y0 < y1;
            }
        }
        if (!vis) {
            depth_key[r] = 0xFFFFFFFFu;
            tile_count[r] = 0;
            rect[r] = make_uint2(0, 0);
            splat[3 * (size_t)r + 0] = make_float4(0, 0, 0, 0);
            splat[3 * (size_t)r + 1] = make_float4(0, 0, 0, 0);
            splat[3 * (size_t)r + 2] = make_float4(0, 0, 0, 0);
            continue;
        }
        // colour: SH at the unit direction camera -> mean
        double dx = mx - V.campos[0], dy = my - V.campos[1], dz = mz - V.campos[2];
        const double dn = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
        dx *= dn; dy *= dn; dz *= dn;
        double col[3];
        if constexpr (HOIST_SH) {
            double acc[3] = {0.0, 0.0, 0.0};
            sh_accumulate64(deg, dx, dy, dz, sh, acc);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const double a = acc[ch] + 0.5;
                col[ch] = a > 0.0 ? a : 0.0;
                flags |= a > 0.0 ? 0u : (1u << ch);
            }
        } else {
            double Y[16];
            sh_basis64(deg, dx, dy, dz, Y);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                double acc = 0.0;
                for (int kk = 0; kk < nk; ++kk) acc += Y[kk] * (double)params[(11 + 3 * kk + ch) * S + slot];
                acc += 0.5;
                col[ch] = acc > 0.0 ? acc : 0.0;
                flags |= acc > 0.0 ? 0u : (1u << ch);
            }
        }
        cflags[r] = (uint8_t)flags;
        const float zf = (float)pz;
        const double ui = floor(u), vi_ = floor(v);
        splat[3 * (size_t)r + 0] = make_float4((float)ui, (float)vi_, (float)(0.5 - (u - ui)), (float)(0.5 - (v - vi_)));
        // conic pre-scaled so that exp(-Q/2) = 2^(A' dx^2 + B' dx dy + C' dy^2)
        const double L2E = 1.4426950408889634;
        splat[3 * (size_t)r + 1] = make_float4((float)(-0.5 * L2E * A), (float)(-L2E * B), (float)(-0.5 * L2E * C), (float)op);
        splat[3 * (size_t)r + 2] = make_float4((float)col[0], (float)col[1], (float)col[2], zf);
        depth_key[r] = __float_as_uint(zf);
        tile_count[r] = (uint32_t)((x1 - x0) * (y1 - y0));
        rect[r] = make_uint2((uint32_t)x0 | ((uint32_t)y0 << 16), (uint32_t)x1 | ((uint32_t)y1 << 16));
    }
}

// Pair emission in depth order.  A wave takes 64 consecutive records of
// the depth order, whose pair slots form one contiguous stretch, and its
// lanes write the stretch together: the record of a slot is the last of
// the 64 whose first slot is at or below it (a binary search over the
// lanes' offsets), and the slot's tile is the record's rect tile at the
// slot's row-major index.  Stores are coalesced, and a record covering
// many tiles spreads over the wave instead of holding it up.  The rects
// come in depth order (gathered by the depth sort's last pass).
__global__ void __launch_bounds__(kBlock)
k_emit_pairs(const uint32_t *__restrict__ sorted_rec, const uint32_t *__restrict__ offsets,
             const uint32_t *__restrict__ total_ptr, const uint2 *__restrict__ rect_sorted,
             const uint32_t *__restrict__ rec_view_base, int n_views, const ViewDev *__restrict__ views,
             uint32_t n, uint32_t cap, uint32_t *__restrict__ pair_key, uint32_t *__restrict__ pair_val) {
    const int lane = threadIdx.x & 63;
    const uint32_t j0 = blockIdx.x * kBlock + (threadIdx.x & ~63u);   // the wave's first record
    if (j0 >= n) return;                                                 // whole waves only
    const uint32_t j = j0 + (uint32_t)lane;
    const bool has = j < n;
    const uint32_t total = *total_ptr;
    const uint32_t off = has ? offsets[j] : total;
    const uint32_t end = j0 + 64 < n ? offsets[j0 + 64] : total;
    uint32_t r = 0, xy0 = 0, w = 1, tbase = 0, tiles_x = 1;
    if (has) {
        r = sorted_rec[j];
        // view of record r: last view whose base <= r
        int a = 0, b = n_views;
        while (b - a > 1) {
            const int m = (a + b) >> 1;
            if (rec_view_base[m] <= r) a = m; else b = m;
        }
        tbase = views[a].tile_base;
        tiles_x = (uint32_t)views[a].tiles_x;
        const uint2 rc = rect_sorted[j];
        xy0 = rc.x;
        w = max((rc.y & 0xFFFFu) - (rc.x & 0xFFFFu), 1u);
    }
    const uint32_t start = __shfl(off, 0, 64);
    for (uint32_t base = start; base < end; base += 64) {   // uniform trip count: all lanes shuffle
        const uint32_t slot = base + (uint32_t)lane;
        int l = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            const uint32_t o = __shfl(off, l + step, 64);
            if (o <= slot) l += step;
        }
        const uint32_t lr = __shfl(r, l, 64), lxy = __shfl(xy0, l, 64), lw = __shfl(w, l, 64);
        const uint32_t lbase = __shfl(tbase, l, 64), ltx = __shfl(tiles_x, l, 64);
        const uint32_t loc = slot - __shfl(off, l, 64);
        uint32_t q = (uint32_t)((float)loc / (float)lw);       // loc / lw, corrected below
        if (q * lw > loc) --q;
        else if ((q + 1) * lw <= loc) ++q;
        const uint32_t tx = (lxy & 0xFFFFu) + (loc - q * lw), ty = (lxy >> 16) + q;
        if (slot < end && slot < cap) {
            pair_key[slot] = lbase + ty * ltx + tx;
            pair_val[slot] = lr;
        }
    }
}

__global__ void k_pair_total(const uint32_t *__restrict__ total, uint32_t cap, uint32_t *__restrict__ pair_count) {
    uint32_t k = *total;
    pair_count[0] = k;
    pair_count[1] = k > cap ? 1u : 0u;
}

// Tile ranges from the sorted pair keys: entry i opens its tile when the
// key before it differs and closes it when the key after it differs.  A
// thread takes four consecutive keys with one 16-byte load; the neighbours
// of its first and last key come from the adjacent lanes (from memory at
// the wave's ends).  The loop's trip count is uniform over a block, so
// every lane reaches the lane exchanges.
__global__ void __launch_bounds__(kBlock)
k_tile_ranges(const uint32_t *__restrict__ pair_key, const uint32_t *__restrict__ pair_count, uint32_t cap,
              uint2 *__restrict__ ranges) {
    uint32_t n = pair_count[0];
    if (n > cap) n = cap;
    const uint32_t nq = (n + 3) / 4;
    const int lane = threadIdx.x & 63;
    constexpr uint32_t kNone = 0xFFFFFFFFu;   // no tile id (ids are below the tile count)
    for (uint32_t t0 = blockIdx.x * kBlock; t0 < nq; t0 += gridDim.x * kBlock) {
        const uint32_t i0 = 4 * (t0 + threadIdx.x);
        uint32_t k[4];
        if (i0 + 4 <= n) {
            const uint4 v = *reinterpret_cast<const uint4 *>(pair_key + i0);
            k[0] = v.x; k[1] = v.y; k[2] = v.z; k[3] = v.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) k[j] = i0 + j < n ? pair_key[i0 + j] : kNone;
        }
        uint32_t prev = __shfl_up(k[3], 1, 64), next = __shfl_down(k[0], 1, 64);
        if (lane == 0) prev = i0 > 0 && i0 <= n ? pair_key[i0 - 1] : kNone;
        if (lane == 63) next = i0 + 4 < n ? pair_key[i0 + 4] : kNone;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = i0 + j;
            if (i >= n) break;
            const uint32_t pk = j == 0 ? prev : k[j > 0 ? j - 1 : 0], nk = j == 3 ? next : k[j < 3 ? j + 1 : 3];
            if (i == 0 || pk != k[j]) ranges[k[j]].x = i;
            if (i == n - 1 || nk != k[j]) ranges[k[j]].y = i + 1;
        }
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f32(float *p, float v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

inline int fill_grid(size_t n) {
    size_t b = (n + kBlock - 1) / kBlock;
    if (b > 4096) b = 4096;
    return b < 1 ? 1 : (int)b;
}

}  // namespace

void launch_fill_u32(hipStream_t s, uint32_t *p, uint32_t v, size_t n) {
    if (n) hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, v, n);
}
void launch_fill_f32(hipStream_t s, float *p, float v, size_t n) {
    if (n) hipLaunchKernelGGL(k_fill_f32, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, v, n);
}
void launch_fill_f64(hipStream_t s, double *p, double v, size_t n) {
    if (n) hipLaunchKernelGGL(k_fill_f64, dim3(fill_grid(n)), dim3(kBlock), 0, s, p, v, n);
}

void launch_preprocess(hipStream_t s, const swgs_plan &p, uint8_t *ws, int view_lo, int view_hi) {
    // all views (view_lo < 0) or the single view view_lo (plain mode)
    int g_lo = 0, g_n = (int)p.groups.size(), only = -1;
    uint32_t maxn = 0;
    if (view_lo >= 0) {
        only = view_lo;
        g_lo = p.vdev[view_lo].group;
        g_n = 1;
        maxn = p.groups[g_lo].n_live;
    } else {
        for (auto &g : p.groups) maxn = maxn > g.n_live ? maxn : g.n_live;
    }
    (void)view_hi;
    if (maxn == 0) return;
    dim3 grid((maxn + kBlock - 1) / kBlock, g_n);
    // frames seen by two or more cameras on average: SH rows hoisted
    size_t nv = 0;
    for (int g = g_lo; g < g_lo + g_n; ++g) nv += (size_t)p.groups[g].n_views;
    const bool hoist = only < 0 && nv >= 2 * (size_t)g_n;
    hipLaunchKernelGGL(hoist ? k_preprocess<true> : k_preprocess<false>, grid, dim3(kBlock), 0, s, p.pool.params, p.pool.n_slots, p.sh_degree,
                       wsp<GroupDev>(ws, p, WB_GROUPS) , wsp<int32_t>(ws, p, WB_GROUP_VIEWS),
                       wsp<ViewDev>(ws, p, WB_VIEWS), wsp<uint32_t>(ws, p, WB_ACTIVE_LIST), g_lo, only,
                       p.tile_w, p.tile_h, wsp<float4>(ws, p, WB_SPLAT), wsp<uint32_t>(ws, p, WB_DEPTH_KEY),
                       wsp<uint32_t>(ws, p, WB_TILE_COUNT), wsp<uint2>(ws, p, WB_RECT),
                       wsp<uint32_t>(ws, p, WB_REC_IDX), wsp<uint8_t>(ws, p, WB_CFLAGS));
}

void launch_pair_offsets(hipStream_t s, const swgs_plan &p, uint8_t *ws, uint32_t rec_lo, uint32_t rec_hi) {
    // the tile counts of the records in depth order (left in PAIR_OFFSET by
    // the depth sort's last pass) become, in place, their first pair slots;
    // then the pair total + overflow flag
    uint32_t *pc = wsp<uint32_t>(ws, p, WB_PAIR_COUNT);
    uint32_t *off = wsp<uint32_t>(ws, p, WB_PAIR_OFFSET);
    exclusive_scan_u32(s, off, off, rec_hi - rec_lo, pc + 2, wsp<uint32_t>(ws, p, WB_SORT_TOTAL));
    hipLaunchKernelGGL(k_pair_total, dim3(1), dim3(1), 0, s, pc + 2, (uint32_t)p.pair_cap, pc);
}

void launch_emit_pairs(hipStream_t s, const swgs_plan &p, uint8_t *ws, uint32_t rec_lo, uint32_t rec_hi) {
    if (rec_hi <= rec_lo) return;
    const uint32_t n = rec_hi - rec_lo;
    // into the buffers the tile sort reads its input from
    const bool alt = radix_input_in_alt(p.tile_key_bits);
    hipLaunchKernelGGL(k_emit_pairs, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       wsp<uint32_t>(ws, p, WB_REC_IDX) + rec_lo, wsp<uint32_t>(ws, p, WB_PAIR_OFFSET),
                       wsp<uint32_t>(ws, p, WB_PAIR_COUNT) + 2, wsp<uint2>(ws, p, WB_RECT_SORTED),
                       wsp<uint32_t>(ws, p, WB_REC_VIEW_BASE), (int)p.views.size(), wsp<ViewDev>(ws, p, WB_VIEWS),
                       n, (uint32_t)p.pair_cap, wsp<uint32_t>(ws, p, alt ? WB_PAIR_KEY_ALT : WB_PAIR_KEY),
                       wsp<uint32_t>(ws, p, alt ? WB_PAIR_VAL_ALT : WB_PAIR_VAL));
}

void launch_row_offsets(hipStream_t s, const swgs_plan &p, uint8_t *ws, uint32_t rec_lo, uint32_t rec_hi) {
    // The backward stores a pair's nine gradient terms as one row, and a
    // record's rows are consecutive, row-major over its tile rect, with the
    // records' rows in record order: a record's first row is the exclusive
    // scan of the tile counts in record order, so the per-record reduce
    // reads and writes contiguous memory.  The pair of tile (tx, ty) is at
    // row first + (ty - y0) w + (tx - x0) = base + ty w + tx, base = first -
    // y0 w - x0 in modulo-2^32 arithmetic: the backward's one lookup per
    // pair.
    if (rec_hi <= rec_lo || p.forward_only) return;
    exclusive_scan_rows(s, wsp<uint32_t>(ws, p, WB_TILE_COUNT) + rec_lo, wsp<uint2>(ws, p, WB_RECT) + rec_lo,
                        rec_hi - rec_lo, wsp<uint32_t>(ws, p, WB_ROW_OFFSET) + rec_lo,
                        wsp<uint2>(ws, p, WB_PAIR_BASE) + rec_lo, wsp<uint32_t>(ws, p, WB_SORT_TOTAL));
}

void launch_tile_ranges(hipStream_t s, const swgs_plan &p, uint8_t *ws, uint32_t tile_lo, uint32_t tile_hi) {
    uint2 *ranges = wsp<uint2>(ws, p, WB_TILE_RANGE);
    launch_fill_u32(s, reinterpret_cast<uint32_t *>(ranges + tile_lo), 0, 2 * (size_t)(tile_hi - tile_lo));
    int nb = (int)((p.pair_cap + 4 * kBlock - 1) / (4 * kBlock));   // four keys per thread
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_tile_ranges, dim3(nb), dim3(kBlock), 0, s, wsp<uint32_t>(ws, p, WB_PAIR_KEY),
                       wsp<uint32_t>(ws, p, WB_PAIR_COUNT), (uint32_t)p.pair_cap, ranges);
}

}  // namespace swgs

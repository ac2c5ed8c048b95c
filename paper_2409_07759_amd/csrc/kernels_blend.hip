// Tile blend, forward (Eq. 3) and its adjoint (Algorithm 1's backward).
//
// One workgroup per (view, tile); one lane per pixel.  The tile's sorted
// list of splats is staged through LDS in batches; every lane walks the
// batch front to back:
//     alpha = min(0.99, o exp(-Q/2)),  skip alpha < 1/255,
//     stop before T (1 - alpha) < 1e-4,  C += c alpha T,  T *= 1 - alpha.
// The record stores the conic pre-scaled by -log2(e)/2 so exp(-Q/2) is one
// v_exp_f32, and the screen position split into an integer part and
// 0.5 - fraction; staging turns it into the offset of the first pixel of
// the 64x64-aligned block holding the tile, (x0 - integer part) +
// (0.5 - fraction) (the difference of integers is exact), so a lane's offset
// is its pixel index inside that block plus one staged value.  Every tile
// shape lies inside one such block, so the rounding, and with it every
// image bit, does not depend on the tile shape.
//
// The forward also stores, per pair, a byte of per-wave support bits (which
// 8x8 pixel blocks of the tile the splat can reach with alpha >= 1/255).
// The backward walks the same list back to front from each pixel's last
// contributor, reading those bits instead of repeating the test and
// recovering the transmittance in front of each splat by
// T <- T / (1 - alpha) (only the final transmittance is stored per pixel),
// and keeping W, the colour behind the splat including the background seen
// through it (W <- c alpha + (1 - alpha) W from W = bg), so that
//     dC/dalpha_k = T_k (c_k - W_k).
// Each wave takes its splats eight at a time in two phases: with a lane per
// pixel it runs the recurrence and leaves two values per (splat, pixel) in
// LDS, then with a lane per (pixel row, splat) it sums them along the row
// into the splat's nine gradient terms (closed forms in the pixel's column
// offset) and adds the eight rows by lane swaps and a DPP step.  The wave
// partials are combined per batch through LDS in wave order, and each
// pair's nine terms are stored as one row at the pair's
// gradient row (a record's rows consecutive, row-major over its tile rect,
// records in record order); an ordered per-record reduce then sums a
// record's rows in row order.  No float atomics: gradients are
// bit-reproducible.
#include <type_traits>

#include "swgs_internal.h"

namespace swgs {
namespace {

constexpr float kLn2 = 0.6931471805599453f;      // 1 / log2(e)
constexpr int kCounterSlots = 256;

// alpha of a staged splat at a pixel; identical instruction sequence in the
// forward and the backward so both take the same skip/stop decisions.
#pragma clang fp contract(off)
struct Px {
    float dx, dy, g, og;  // offsets, 2^p2 (= exp(-Q/2)), o * g
};
// staged offsets, from the splat centre, of the first pixel of the
// 64x64-aligned block holding the tile at (tx0, ty0)
__device__ __forceinline__ float4 block_offset(const float4 a, int tx0, int ty0) {
    return make_float4(((float)(tx0 & ~63) - a.x) + a.z, ((float)(ty0 & ~63) - a.y) + a.w, 0.0f, 0.0f);
}
// (lx, ly): the pixel's index inside its 64x64-aligned block, as floats
__device__ __forceinline__ Px eval_splat(float lx, float ly, const float4 a, const float4 b) {
    Px r;
    r.dx = lx + a.x;
    r.dy = ly + a.y;
    // p2 = A' dx^2 + B' dx dy + C' dy^2 (A', B', C' = -log2(e) (A/2, B, C/2))
    const float t = fmaf(b.y, r.dy, b.x * r.dx);
    const float p2 = fmaf(b.z * r.dy, r.dy, t * r.dx);
    r.g = __builtin_amdgcn_exp2f(p2);
    r.og = b.w * r.g;
    return r;
}
#pragma clang fp contract(fast)

// DPP move (row-level lane permutation), as float
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, true));
}

// sum over the 16 lanes of each DPP row; every lane of a row holds its row sum
__device__ __forceinline__ float row_sum16(float x) {
    x += dpp_f<0xB1, 0xf>(x);   // quad_perm [1,0,3,2]
    x += dpp_f<0x4E, 0xf>(x);   // quad_perm [2,3,0,1]
    x += dpp_f<0x124, 0xf>(x);  // row_ror:4
    x += dpp_f<0x128, 0xf>(x);  // row_ror:8
    return x;
}

// One exchange step of a transposed reduction: lanes whose `bit` is clear
// keep the partial sum of a, the others that of c, each adding the partner
// lane's copy (the partner, selected by CTRL, has the opposite bit).
template <int CTRL>
__device__ __forceinline__ float xstep(float a, float c, bool bit) {
    const float keep = bit ? c : a, send = bit ? a : c;
    return keep + dpp_f<CTRL, 0xf>(send);
}

// One exchange step across the two 32-lane halves (x = 32) or across the
// two rows of each row pair (x = 16) with gfx950's lane-swap instructions:
// the result holds a's pair sum in the lower half / even rows and c's in
// the upper half / odd rows (two instructions per step).
__device__ __forceinline__ float xswap32(float a, float c) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(c), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xswap16(float a, float c) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(c), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// max over the 16 lanes of each DPP row; every lane of a row holds it
__device__ __forceinline__ uint32_t row_max16(uint32_t x) {
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xf, 0xf, true));   // quad_perm [1,0,3,2]
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xf, 0xf, true));   // quad_perm [2,3,0,1]
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x124, 0xf, 0xf, true));  // row_ror:4
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xf, 0xf, true));  // row_ror:8
    return x;
}

// Whole-wave max / sum, every lane holding it: row reductions, then the
// half swap and the row-pair swap of each lane's value with itself (each
// lane meets its partner in the other half, then in the other row of its
// pair), 8 VALU operations.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    x = row_max16(x);
    const auto h = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    x = max(h[0], h[1]);
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return max(r[0], r[1]);
}
__device__ __forceinline__ float wave_sum_f32(float x) {
    x = row_sum16(x);
    x = xswap32(x, x);
    return xswap16(x, x);
}

// Pixel of a thread: each wave covers an 8x8 block of the tile (a 16x16
// tile is 2x2 blocks, 32x8 is 4x1), lanes row-major inside the block.
template <int TW, int TH>
__device__ __forceinline__ void lane_pixel(int tid, int &px, int &py) {
    if (TW == 8 && TH == 8) {
        px = tid & 7;
        py = tid >> 3;
    } else {
        const int w = tid >> 6, l = tid & 63;
        px = (w % (TW / 8)) * 8 + (l & 7);
        py = (w / (TW / 8)) * 8 + (l >> 3);
    }
}

// Bit w set if some pixel centre of wave w's 8x8 block of the tile at
// (tx0, ty0) can take alpha >= 1/255 from the splat (a: position record,
// b: pre-scaled conic and opacity).  With q(d) = -(A' dx^2 + B' dx dy +
// C' dy^2) the exponent's positive quadratic form, alpha >= 1/255 iff
// q <= log2(255 o).  The test takes the minimum of q over the rectangle of
// the block's pixel centres grown by 1/64 px on every side: zero when the
// splat centre lies inside, else attained on a face the centre sees (a
// convex function's minimum over a box lies where the segment to its
// unconstrained minimiser leaves the box), i.e. at the clamped 1D minimum
// along at most one vertical and one horizontal face.  Threshold and
// rectangle carry margins far above FP32 rounding, so no block holding a
// blended pixel is culled; a nearly singular FP32 conic is never culled.
template <int TW, int TH>
__device__ __forceinline__ uint32_t support_wave_mask(const float4 a, const float4 b, int tx0, int ty0) {
    constexpr int NWX = TW / 8, NW = (TW * TH) / 64;
    constexpr float kEps = 1.0f / 64.0f;
    const float qa = -b.x, qb = -b.y, qc = -b.z;
    const float disc = 4.0f * qa * qc;
    if (!(qa > 0.0f && qc > 0.0f && disc - qb * qb > 1e-3f * disc)) return (1u << NW) - 1u;
    const float lam = __log2f(255.0f * b.w);
    const float lim = lam + 1e-3f * (1.0f + fabsf(lam));
    const float h2a = 0.5f / qa, h2c = 0.5f / qc;
    uint32_t m = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        // offsets of the block's first pixel centre: (X0 - integer part) +
        // (0.5 - fraction), the difference of integers exact
        const float ex0 = (((float)(tx0 + (w % NWX) * 8) - a.x) + a.z) - kEps, ex1 = ex0 + (7.0f + 2.0f * kEps);
        const float ey0 = (((float)(ty0 + (w / NWX) * 8) - a.y) + a.w) - kEps, ey1 = ey0 + (7.0f + 2.0f * kEps);
        const bool inx = ex0 <= 0.0f && ex1 >= 0.0f, iny = ey0 <= 0.0f && ey1 >= 0.0f;
        const float xe = ex0 > 0.0f ? ex0 : ex1;       // the vertical face the centre sees
        const float ty = fminf(fmaxf(-qb * xe * h2c, ey0), ey1);
        const float qv = inx ? 3.0e38f : (qa * xe + qb * ty) * xe + qc * ty * ty;
        const float ye = ey0 > 0.0f ? ey0 : ey1;       // the horizontal face the centre sees
        const float tx = fminf(fmaxf(-qb * ye * h2a, ex0), ex1);
        const float qh = iny ? 3.0e38f : (qc * ye + qb * tx) * ye + qa * tx * tx;
        const float qmin = (inx && iny) ? 0.0f : fminf(qv, qh);
        m |= qmin <= lim ? (1u << w) : 0u;
    }
    return m;
}

// staged entry at a byte offset (16 x its index) of a float4 LDS array
__device__ __forceinline__ float4 at16(const float4 *base, int off) {
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + off);
}

// Each wave compacts, in ascending order, the batch entries whose mask has
// its bit set, as entry index x 16 (the byte offset of the entry's float4 in
// the staging arrays); returns the count (wave-uniform).
template <int CAP>
__device__ __forceinline__ int wave_list(const uint32_t *smask, int m, int wave, int lane, uint16_t *list) {
    int cnt = 0;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int c = 0; c < m; c += 64) {
        const int k = c + lane;
        const bool hit = k < m && ((smask[k] >> wave) & 1u);
        const uint64_t b = __ballot(hit);
        if (hit) list[cnt + __popcll(b & lt)] = (uint16_t)(16 * k);
        cnt += __popcll(b);
    }
    return cnt;
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

template <int TW, int TH, int BATCH, bool COUNT>
__global__ void __launch_bounds__(TW *TH)
k_blend_fwd(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ pair_val,
            const float4 *__restrict__ splat, const ViewDev *__restrict__ views,
            int n_views, uint32_t tile_lo, float *__restrict__ images,
            float *__restrict__ T_final, uint32_t *__restrict__ last_out,
            const float *__restrict__ targets, float *__restrict__ dLdC, double *__restrict__ loss_part,
            unsigned long long *__restrict__ counters, float l1_weight, uint8_t *__restrict__ pair_mask,
            uint32_t spread) {
    constexpr int NT = TW * TH;
    static_assert(64 % TW == 0 && 64 % TH == 0, "a tile lies inside one 64x64-aligned block");
    constexpr bool CULL = NT > 64;        // per-wave support-box lists
    constexpr int NW = NT / 64;
    __shared__ float4 sa[BATCH], sb[BATCH], sc[BATCH];
    __shared__ uint32_t smask[CULL ? BATCH : 1];
    __shared__ uint16_t slist[CULL ? NW : 1][CULL ? BATCH : 1];
    __shared__ float red[2][NT / 64];
    __shared__ unsigned long long cnt_evals, cnt_blend;
    // neighbouring tiles share an XCD's L2; a window of uneven views is
    // spread over the XCDs in chunks of tiles
    const uint32_t lt_idx = xcd_spread(xcd_order(blockIdx.x, gridDim.x), gridDim.x, spread);
    const uint32_t tile = tile_lo + lt_idx;
    const ViewDev &V = views[view_of_tile(views, n_views, tile)];
    const uint32_t lt = tile - V.tile_base;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    int lx, ly;
    lane_pixel<TW, TH>(threadIdx.x, lx, ly);
    const int x = tx * TW + lx, y = ty * TH + ly;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool inside = x < V.width && y < V.height;
    const float lxf = (float)(x & 63), lyf = (float)(y & 63);
    const uint2 rg = ranges[tile];
    const uint32_t n = rg.y - rg.x;

    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    uint32_t last = 0;
    uint32_t stop_at = inside ? n : 0;   // list entries this pixel evaluates (counted builds)
    uint32_t nblend = 0;                 // entries it blends (counted builds)
    bool done = !inside;
    for (uint32_t b0 = 0; b0 < n; b0 += BATCH) {
        if (__syncthreads_and(done)) break;
        for (int k = threadIdx.x; k < BATCH; k += NT) {
            if (b0 + k < n) {
                const uint32_t r = pair_val[rg.x + b0 + k];
                const float4 a = splat[3 * (size_t)r], b = splat[3 * (size_t)r + 1];
                sa[k] = block_offset(a, tx * TW, ty * TH);
                sb[k] = b;
                sc[k] = splat[3 * (size_t)r + 2];
                if (CULL) {
                    const uint32_t mk = support_wave_mask<TW, TH>(a, b, tx * TW, ty * TH);
                    smask[k] = mk;
                    if (pair_mask) pair_mask[rg.x + b0 + k] = (uint8_t)mk;   // for the backward
                }
            }
        }
        __syncthreads();
        const int m = (int)min((uint32_t)BATCH, n - b0);
        const int cnt = CULL ? wave_list<BATCH>(smask, m, wave, lane, slist[CULL ? wave : 0]) : m;
        // branch-free per lane: a splat is blended when alpha >= 1/255 and
        // the pixel has not stopped; the stop test fires on the splat that
        // would take T below 1e-4 (that splat is not blended).  The last
        // blended entry of the batch is kept as its byte offset (-16: none)
        int last_off = -16;
        for (int i = 0; i < cnt; ++i) {
            const int off = CULL ? (int)slist[CULL ? wave : 0][i] : 16 * i;
            const uint32_t idx = b0 + (uint32_t)(off >> 4) + 1;
            const Px e = eval_splat(lxf, lyf, at16(sa, off), at16(sb, off));
            const float alpha = fminf(0.99f, e.og);
            const float w0 = alpha * T;
            const float Tn = __fsub_rn(T, w0);             // T (1 - alpha), sharing alpha T
            const bool pass = !done && alpha >= (1.0f / 255.0f);
            const bool stop = pass && Tn < 1e-4f;
            const bool use = pass && !stop;
            const float w = use ? w0 : 0.0f;
            const float4 c = at16(sc, off);
            c0 = fmaf(c.x, w, c0);
            c1 = fmaf(c.y, w, c1);
            c2 = fmaf(c.z, w, c2);
            T = use ? Tn : T;
            last_off = use ? off : last_off;
            if (COUNT) {
                stop_at = stop ? idx : stop_at;
                nblend += use ? 1u : 0u;
            }
            done = done || stop;
        }
        if (last_off >= 0) last = b0 + (uint32_t)(last_off >> 4) + 1;
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
            const float s = V.inv_norm * l1_weight;
            if (dLdC) {   // (else the D-SSIM backward writes dL/dC, this L1 term included)
                dLdC[o3] = d0 > 0.0f ? s : (d0 < 0.0f ? -s : 0.0f);
                dLdC[o3 + HW] = d1 > 0.0f ? s : (d1 < 0.0f ? -s : 0.0f);
                dLdC[o3 + 2 * HW] = d2 > 0.0f ? s : (d2 < 0.0f ? -s : 0.0f);
            }
            l1 = (fabsf(d0) + fabsf(d1) + fabsf(d2)) * s;
            sq = d0 * d0 + d1 * d1 + d2 * d2;
        }
    }
    if (COUNT) {
        if (threadIdx.x == 0) { cnt_evals = 0; cnt_blend = 0; }
        __syncthreads();
        atomicAdd(&cnt_evals, (unsigned long long)stop_at);
        atomicAdd(&cnt_blend, (unsigned long long)nblend);
        __syncthreads();
        if (threadIdx.x == 0) {
            // spread over kCounterSlots slots: one address per block would serialise
            unsigned long long *c = counters + 4 * (blockIdx.x % kCounterSlots);
            atomicAdd(c, cnt_evals);
            atomicAdd(c + 2, cnt_blend);
        }
    }
    if (targets) {
        l1 = wave_sum_f32(l1);
        sq = wave_sum_f32(sq);
        if ((threadIdx.x & 63) == 0) {
            red[0][threadIdx.x >> 6] = l1;
            red[1][threadIdx.x >> 6] = sq;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < NT / 64; ++w) { a += red[0][w]; b += red[1][w]; }
            loss_part[2 * (size_t)lt_idx] = a;
            loss_part[2 * (size_t)lt_idx + 1] = b;
        }
    }
}

// Backward batches are BB splats; each wave stores, per splat of its list,
// its partial sums of the nine gradient terms to LDS: floats 0-8 colour 3,
// opacity, conic 3 (dx^2, dx dy, dy^2 products), offset x, offset y.
constexpr int kTerm = 9;
constexpr int kSub = 8;                   // splats per sub-batch (phase A -> phase B)
constexpr int kPitch = 65;                // float2 per (sub-batch splat) row: 64 pixels + 1 (bank spread)

// 3-bit reversal: the term a phase-B lane of pixel row r holds after the
// row reduction
__device__ __forceinline__ int brev3(int r) { return ((r & 1) << 2) | (r & 2) | ((r >> 2) & 1); }

// Phase-B step over column i of a pixel row: (w, m') of the lane's splat
// at pixel (r, i), that pixel's dL/dC from phase-A lane 8 r + i by a
// swizzle inside each 32-lane half (lane (l & 24) | i), and the row sums
// of g.w and of m', i' m', i'^2 m' (i' = i - 3.5)
template <int I>
__device__ __forceinline__ float swz_col(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 24 | (I << 5)));
}
template <int I>
__device__ __forceinline__ void row_step(const float2 *prow, float g0, float g1, float g2, float &C0, float &C1,
                                         float &C2, float &S0, float &S1, float &S2) {
    constexpr float c = (float)I - 3.5f;
    const float2 pm = prow[I];
    C0 = fmaf(swz_col<I>(g0), pm.x, C0);
    C1 = fmaf(swz_col<I>(g1), pm.x, C1);
    C2 = fmaf(swz_col<I>(g2), pm.x, C2);
    S0 += pm.y;
    S1 = fmaf(c, pm.y, S1);
    S2 = fmaf(c * c, pm.y, S2);
}

// orders one wave's LDS accesses across its lanes (stores before the
// following loads, loads before the following stores): the compiler keeps
// them on their side, and the LDS carries out one wave's accesses in order
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int TW, int TH, int BATCH, bool COUNT>
__global__ void __launch_bounds__(TW *TH, TW *TH >= 256 ? 6 : 1)
k_blend_bwd(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ pair_val,
            const float4 *__restrict__ splat, const ViewDev *__restrict__ views,
            int n_views, uint32_t tile_lo, const float *__restrict__ T_final,
            const uint32_t *__restrict__ last_in, const float *__restrict__ dLdC,
            const uint2 *__restrict__ slot_base, const uint32_t *__restrict__ pair_count,
            const uint8_t *__restrict__ pair_mask, float *__restrict__ pair_grad,
            unsigned long long *__restrict__ counters, uint32_t spread) {
    constexpr int NT = TW * TH;
    static_assert(64 % TW == 0 && 64 % TH == 0, "a tile lies inside one 64x64-aligned block");
    constexpr int NW = NT / 64;           // waves
    constexpr int BB = 48;                // splats per LDS batch (26 KB of LDS per 16x16 block: 6 per CU)
    constexpr bool CULL = NW > 1;
    static_assert(BB % 8 == 0, "a sub-batch's eight list entries are one 16-byte LDS read");
    __shared__ float4 sa[BB], sb[BB], sc[BB];
    __shared__ uint32_t smask[BB];
    __shared__ __align__(16) uint16_t slist[CULL ? NW : 1][CULL ? BB : 1];   // rows of 96 B
    __shared__ uint32_t sslot[BB];        // gradient row of each batch pair
    __shared__ float part[BB][NW][kTerm];
    __shared__ float2 pbuf[NW][kSub][kPitch];   // phase A -> B: (w, m') per (sub-batch splat, pixel)
    __shared__ uint32_t swlast[NW];
    __shared__ unsigned long long cnt_evals;
    // after a pair overflow some of the listed pairs' rows lie past the
    // capacity: nothing is stored (the reduce then writes zero gradients)
    if (pair_count[1] != 0) return;
    // neighbouring tiles share an XCD's L2; a window of uneven views is
    // spread over the XCDs in chunks of tiles
    const uint32_t lt_idx = xcd_spread(xcd_order(blockIdx.x, gridDim.x), gridDim.x, spread);
    const uint32_t tile = tile_lo + lt_idx;
    const ViewDev &V = views[view_of_tile(views, n_views, tile)];
    const uint32_t lt = tile - V.tile_base;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    int lx, ly;
    lane_pixel<TW, TH>(threadIdx.x, lx, ly);
    const int x = tx * TW + lx, y = ty * TH + ly;
    const bool inside = x < V.width && y < V.height;
    const float lxf = (float)(x & 63), lyf = (float)(y & 63);
    const uint2 rg = ranges[tile];

    float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
    uint32_t lst = 0;
    if (inside) {
        // per-view and per-channel bases (64-bit, wave-uniform), in-view
        // offsets in 32 bits (a view holds fewer than 2^31 pixels; the
        // channel planes are reached through their own bases, so 3 HW may
        // exceed 2^32)
        const size_t HW = (size_t)V.width * (size_t)V.height;
        const uint32_t o = (uint32_t)y * (uint32_t)V.width + (uint32_t)x;
        const float *dl0 = dLdC + 3 * V.pix_base;
        const float *dl1 = dl0 + HW, *dl2 = dl1 + HW;
        T = (T_final + V.pix_base)[o];
        lst = (last_in + V.pix_base)[o];
        g0 = dl0[o];
        g1 = dl1[o];
        g2 = dl2[o];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // a wave never needs splats at or beyond its pixels' largest `last`;
    // the tile's largest is the largest of its waves'
    const uint32_t wlast = wave_max_u32(lst);
    if (threadIdx.x == 0) cnt_evals = 0;
    if ((threadIdx.x & 63) == 0) swlast[threadIdx.x >> 6] = wlast;
    __syncthreads();
    if (COUNT) {   // counted build only (timing flag SWGS_TIMING_COUNT)
        atomicAdd(&cnt_evals, (unsigned long long)lst);
        __syncthreads();
    }
    uint32_t nmax = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) nmax = max(nmax, swlast[w]);
    if (COUNT && threadIdx.x == 0) atomicAdd(counters + 4 * (blockIdx.x % kCounterSlots) + 1, cnt_evals);
    // A pair's gradient row: the record's first row plus this tile's
    // row-major index inside the record's tile rect, from the record's
    // (base, rect width) = (first row - y0 w - x0, w) as base + ty w + tx
    // (modulo 2^32).
    auto slot_of = [&](uint32_t r) {
        const uint2 sb = slot_base[r];
        return sb.x + (uint32_t)ty * sb.y + (uint32_t)tx;
    };
    // pairs past every pixel's last contributor get zero terms
    for (uint32_t q = nmax + threadIdx.x; q < rg.y - rg.x; q += NT) {
        float *dst = pair_grad + 9 * (size_t)slot_of(pair_val[rg.x + q]);
#pragma unroll
        for (int t = 0; t < 9; ++t) dst[t] = 0.0f;
    }
    // W = what lies behind the current splat as seen through it: the colour
    // of the splats already walked (back to front) plus the background
    // through their transmittance.  It follows the blend recurrence
    // W <- c a + (1 - a) W from W = bg, and dL/da_k = T_k g.(c_k - W) with g
    // = dL/dC of the pixel; only gW = g.W is needed, and it follows the same
    // recurrence: gW <- gW + a (g.c - gW).
    float gW = g0 * V.bg[0] + g1 * V.bg[1] + g2 * V.bg[2];
    // phase B: lane (r, s) takes pixel row r of the wave's 8x8 block (pixels
    // r, columns 0-7: lanes 8 r .. 8 r + 7 of phase A) and sub-batch splat
    // s; (bx + i, byr) are the row's pixels inside the 64x64-aligned block
    const int sB = lane & 7, rB = lane >> 3;
    const float bx = (float)((tx * TW + (wave % (TW / 8)) * 8) & 63);
    const float byr = (float)(((ty * TH + (wave / (TW / 8)) * 8) & 63) + rB);

    // thread k stages entry k of a batch; its pair value (the record) is
    // read one batch ahead, so staging waits for one dependent load only
    static_assert(BB <= NT, "one staged entry per thread");
    auto batch_start = [&](uint32_t e) { return e > (uint32_t)BB ? e - BB : 0u; };
    uint32_t r_next = (uint32_t)threadIdx.x < nmax - batch_start(nmax)
                          ? pair_val[rg.x + batch_start(nmax) + threadIdx.x] : 0u;
    for (uint32_t b_end = nmax; b_end > 0;) {
        const uint32_t b_start = batch_start(b_end);
        const int m = (int)(b_end - b_start);
        if ((int)threadIdx.x < m) {
            const int k = threadIdx.x;
            const uint32_t r = r_next;
            sslot[k] = slot_of(r);
            sa[k] = block_offset(splat[3 * (size_t)r], tx * TW, ty * TH);
            sb[k] = splat[3 * (size_t)r + 1];
            sc[k] = splat[3 * (size_t)r + 2];
            // the forward's support test of this pair (the forward staged
            // every entry before the tile's largest last contributor)
            smask[k] = CULL ? (uint32_t)pair_mask[rg.x + b_start + k] : 1u;
        }
        __syncthreads();
        // the next batch's pair value (the loop below does not touch it)
        r_next = (uint32_t)threadIdx.x < b_start - batch_start(b_start)
                     ? pair_val[rg.x + batch_start(b_start) + threadIdx.x] : 0u;
        const int wm = (int)min((uint32_t)m, wlast > b_start ? wlast - b_start : 0u);
        // the wave's list length, wave-uniform (scalar loop control below)
        const int cnt = __builtin_amdgcn_readfirstlane(
            CULL ? wave_list<BB>(smask, wm, wave, lane, slist[CULL ? wave : 0]) : wm);
        // entries of this batch before the pixel's last contributor, as a
        // byte-offset bound (entry k is before it iff 16 k < lim)
        const int lim = 16 * ((int)min(lst, b_end) - (int)min(lst, b_start));
        wave_lds_sync();   // the list's stores before its 16-byte reads
        // sub-batches of list positions 8 m .. 8 m + 7, the top one first
        // (possibly partial), each walked back to front
        for (int top = cnt; top > 0;) {
            const int base8 = (top - 1) & ~(kSub - 1), nsb = top - base8;
            top = base8;
            // the sub-batch's eight list entries (one 16-byte read, kept in
            // scalar registers: position q's offset is a constant shift)
            uint32_t sw[4] = {0u, 0u, 0u, 0u};
            if (CULL) {
                const uint4 v = *reinterpret_cast<const uint4 *>(&slist[CULL ? wave : 0][base8]);
                sw[0] = __builtin_amdgcn_readfirstlane(v.x);
                sw[1] = __builtin_amdgcn_readfirstlane(v.y);
                sw[2] = __builtin_amdgcn_readfirstlane(v.z);
                sw[3] = __builtin_amdgcn_readfirstlane(v.w);
            }
            // phase B's splat: list position base8 + s (lanes past the
            // sub-batch take the last position and store nothing); read
            // before phase A
            const int ie = min(base8 + sB, cnt - 1);
            const int offs = CULL ? (int)slist[CULL ? wave : 0][ie] : 16 * ie;
            const float4 as = at16(sa, offs);
            const float os = at16(sb, offs).w;
            // phase A, lane = pixel, positions base8 + nsb - 1 down to base8
            // (back to front) into sub-batch slots q = position - base8:
            // the colour weight w = alpha T_k and m' = g dL/dalpha (g =
            // exp(-Q/2); zero where alpha is clamped), both zero where the
            // splat was not blended here
            auto phase_a = [&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if (q >= nsb) return;                            // wave-uniform
                const int off = CULL ? (int)((sw[q >> 1] >> (16 * (q & 1))) & 0xFFFFu) : 16 * (base8 + q);
                // contrib = the forward blended this splat here
                const Px e = eval_splat(lxf, lyf, at16(sa, off), at16(sb, off));
                // g.c, taken with the other reads of the entry (its LDS read
                // then overlaps the evaluation)
                const float4 c = at16(sc, off);
                const float gc = fmaf(g2, c.z, fmaf(g1, c.y, g0 * c.x));
                asm volatile("" : : "v"(gc));   // keeps the read and the product ahead of the branch
                const float alpha = fminf(0.99f, e.og);
                const bool contrib = off < lim && alpha >= (1.0f / 255.0f);
                // T and W change only where the splat was blended: a wave
                // with no such pixel skips the recurrence (branch-free inside)
                float wv = 0.0f, mp = 0.0f;
                if (__ballot(contrib) != 0) {
                    const float ri = __builtin_amdgcn_rcpf(1.0f - alpha);
                    const float Tk = T * ri;                                 // transmittance in front of k
                    const float diff = gc - gW;
                    const float ac = contrib ? alpha : 0.0f;
                    wv = ac * Tk;
                    // alpha = o g: dL/do = g dL/dalpha, dL/dQ = -o g dL/dalpha / 2
                    mp = (contrib && e.og < 0.99f) ? e.g * (Tk * diff) : 0.0f;
                    T = contrib ? Tk : T;
                    gW = fmaf(ac, diff, gW);                                 // a = 0 keeps gW
                }
                pbuf[wave][q][lane] = make_float2(wv, mp);
            };
            phase_a(std::integral_constant<int, 7>{});
            phase_a(std::integral_constant<int, 6>{});
            phase_a(std::integral_constant<int, 5>{});
            phase_a(std::integral_constant<int, 4>{});
            phase_a(std::integral_constant<int, 3>{});
            phase_a(std::integral_constant<int, 2>{});
            phase_a(std::integral_constant<int, 1>{});
            phase_a(std::integral_constant<int, 0>{});
            wave_lds_sync();
            // phase B: row sums of g.w (colour) and of m', i' m', i'^2 m'
            // (i' = i - 3.5, the column's offset from the row centre); with
            // dx = d0 + i' and dy constant along the row, the partials of
            // q = o m' (= -2 dL/dQ) follow: sum q dx = o (d0 S0 + S1), sum q
            // dx^2 = o (d0^2 S0 + 2 d0 S1 + S2), and dy factors out
            float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;
            const float2 *prow = &pbuf[CULL ? wave : 0][sB][8 * rB];
            row_step<0>(prow, g0, g1, g2, C0, C1, C2, S0, S1, S2);
            row_step<1>(prow, g0, g1, g2, C0, C1, C2, S0, S1, S2);
            row_step<2>(prow, g0, g1, g2, C0, C1, C2, S0, S1, S2);
            row_step<3>(prow, g0, g1, g2, C0, C1, C2, S0, S1, S2);
            row_step<4>(prow, g0, g1, g2, C0, C1, C2, S0, S1, S2);
            row_step<5>(prow, g0, g1, g2, C0, C1, C2, S0, S1, S2);
            row_step<6>(prow, g0, g1, g2, C0, C1, C2, S0, S1, S2);
            row_step<7>(prow, g0, g1, g2, C0, C1, C2, S0, S1, S2);
            wave_lds_sync();
            const float d0 = (bx + 3.5f) + as.x, dy = byr + as.y;
            const float Q0 = os * S0, Qx = os * fmaf(d0, S0, S1);
            const float Qxx = os * fmaf(d0, fmaf(d0, S0, 2.0f * S1), S2);
            const float Qy = Q0 * dy;
            // the eight rows of each splat added: lane swaps across halves
            // and row pairs, then a DPP exchange inside rows; lane (r, s)
            // ends with term brev3(r) of splat s and every lane with the
            // offset-y term
            const float b0 = xswap32(C0, C1), b1 = xswap32(C2, S0), b2 = xswap32(Qxx, Qx * dy);
            const float b3 = xswap32(Qy * dy, Qx), b4 = xswap32(Qy, Qy);
            const float c0 = xswap16(b0, b1), c1 = xswap16(b2, b3), c2 = xswap16(b4, b4);
            const float d = xstep<0x128>(c0, c1, (lane >> 3) & 1);
            const float d8 = c2 + dpp_f<0x128, 0xf>(c2);
            if (sB < nsb) {
                float *pd = part[offs >> 4][wave];
                pd[brev3(rB)] = d;
                if (rB == 0) pd[8] = d8;
            }
        }
        __syncthreads();
        // flush: one thread per (splat, term group) sums the group's row
        // partials over the waves whose block the splat reaches (in wave
        // order) and stores its terms of the pair's 36-byte gradient row
        // d/d(u, v, A, B, C, o, r, g, b), conic
        // unscaled (A = -2 A' ln2, B = -B' ln2, C = -2 C' ln2): no atomics,
        // and a fixed summation order.  Groups: 0 colour 3 + opacity,
        // 1 conic terms 3 (+ offset x), 2 offset y with offset x.
        auto flush = [&](int k, int j) {
            const uint32_t hit = smask[k];
            float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            float sx = 0.0f;
            for (int q = 0; q < NW; ++q) {
                // wave q wrote this partial only if the splat reaches its
                // block and lies before its pixels' largest `last`
                if (!((hit >> q) & 1u) || b_start + (uint32_t)k >= swlast[q]) continue;
                const float *a = part[k][q];
                if (j == 2) {
                    acc.x += a[8];
                    sx += a[7];
                } else {
                    acc.x += a[4 * j]; acc.y += a[4 * j + 1]; acc.z += a[4 * j + 2]; acc.w += a[4 * j + 3];
                }
            }
            float *row = pair_grad + 9 * (size_t)sslot[k];
            if (j == 0) {
                row[5] = acc.w;
                row[6] = acc.x;
                row[7] = acc.y;
                row[8] = acc.z;
            } else if (j == 1) {
                // conic terms dx^2, 2 dx dy, dy^2 times dL/dQ = -q/2
                row[2] = -0.5f * acc.x;
                row[3] = -acc.y;
                row[4] = -0.5f * acc.z;
            } else {
                // dQ/ddx = 2(A dx + B dy), ddx/du = -1; partials hold -2 dL/dQ
                const float4 b = sb[k];
                const float A = -2.0f * kLn2 * b.x, B = -kLn2 * b.y, C = -2.0f * kLn2 * b.z;
                const float sy = acc.x;
                row[0] = A * sx + B * sy;
                row[1] = B * sx + C * sy;
            }
        };
        static_assert(BB <= 64, "one lane per batch splat in the flush");
        if constexpr (NT >= 3 * 64) {
            // wave j takes term group j, lane k Gaussian k (the group's
            // branch is wave-uniform)
            if (threadIdx.x < 3 * 64 && (int)(threadIdx.x & 63) < m) flush((int)(threadIdx.x & 63), (int)(threadIdx.x >> 6));
        } else {
            for (int t = threadIdx.x; t < 3 * m; t += NT) flush(t % m, t / m);
        }
        __syncthreads();
        b_end = b_start;
    }
}

// Window L1 sum: per-tile partials (written by the forward epilogue) are
// reduced in two fixed-order levels, kLossBlocks contiguous chunks and then
// their kLossBlocks sums, so the result does not depend on scheduling.
constexpr int kLossBlocks = 256;

__device__ __forceinline__ void block_sum2(double &a, double &b) {
    __shared__ double sa[256], sb[256];
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
    a = sa[0];
    b = sb[0];
}

__global__ void __launch_bounds__(256)
k_loss_partial(const double *__restrict__ part, int nparts, double *__restrict__ sums) {
    const int chunk = (nparts + kLossBlocks - 1) / kLossBlocks;
    const int lo = blockIdx.x * chunk, hi = min(nparts, lo + chunk);
    double a = 0.0, b = 0.0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += 256) {
        a += part[2 * (size_t)i];
        b += part[2 * (size_t)i + 1];
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        sums[2 * blockIdx.x] = a;
        sums[2 * blockIdx.x + 1] = b;
    }
}

__global__ void __launch_bounds__(256)
k_loss_final(const double *__restrict__ sums, double inv_3p, double *__restrict__ stats) {
    double a = sums[2 * threadIdx.x], b = sums[2 * threadIdx.x + 1];
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        stats[0] = a;
        stats[1] = b * inv_3p;
    }
}

// Record gradients: each record's nine terms summed over its gradient rows
// in row order (deterministic).  A record's rows are consecutive and the
// records' rows follow record order, so the kReduceRecs consecutive records
// of a block own one contiguous stretch of rows: it is staged through LDS
// with 16-byte loads (kReduceChunk rows at a time, from the 16-byte boundary
// at or below its start), then nine lanes per record (lane t summing term t)
// add their record's rows, seven records per wave and round, and store each
// record's sums as one 36-byte row (the block's records: one contiguous
// stretch of sums).  After a pair overflow the rows are incomplete, and
// every record's sums are zero.
constexpr int kReduceRounds = 8;
constexpr int kReduceRecs = 4 * 7 * kReduceRounds;   // 4 waves
constexpr int kReduceChunk = 512;                    // rows per LDS stage (18 KB: 8 blocks per CU)
constexpr int kReduceVec = (9 * kReduceChunk + 3) / 4 + 1;

__global__ void __launch_bounds__(256, 8)
k_pair_grad_reduce(const uint32_t *__restrict__ first_row, const uint32_t *__restrict__ pair_count,
                   const float *__restrict__ pair_grad, uint32_t cap, uint32_t n, float *__restrict__ rec_grad) {
    __shared__ float4 buf4[kReduceVec];
    __shared__ uint32_t bound[kReduceRecs + 1];
    const float *buf = reinterpret_cast<const float *>(buf4);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane / 9, t = lane - 9 * g;
    const uint32_t j0 = blockIdx.x * kReduceRecs;
    const uint32_t nb = min((uint32_t)kReduceRecs, n - j0);
    const uint32_t total = pair_count[0];
    const bool overflow = pair_count[1] != 0;
    // record boundaries (all empty after an overflow)
    for (uint32_t x = threadIdx.x; x <= nb; x += 256)
        bound[x] = overflow ? 0u : min(j0 + x < n ? first_row[j0 + x] : total, cap);
    __syncthreads();
    const uint32_t lo = bound[0], hi = bound[nb];
    float acc[kReduceRounds];
#pragma unroll
    for (int q = 0; q < kReduceRounds; ++q) acc[q] = 0.0f;
    for (uint32_t base = lo; base < hi; base += kReduceChunk) {
        const uint32_t cnt = min((uint32_t)kReduceChunk, hi - base);
        const size_t f0 = 9 * (size_t)base, a0 = f0 & ~(size_t)3;
        const uint32_t shift = (uint32_t)(f0 - a0);
        const uint32_t n4 = (shift + 9 * cnt + 3) / 4;
        const float4 *src = reinterpret_cast<const float4 *>(pair_grad + a0);
        for (uint32_t x0 = threadIdx.x; x0 < n4; x0 += 8 * 256) {
            float4 v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                v[k] = x0 + 256 * k < n4 ? src[x0 + 256 * k] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (x0 + 256 * k < n4) buf4[x0 + 256 * k] = v[k];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kReduceRounds; ++q) {
            const uint32_t jj = (uint32_t)(7 * (kReduceRounds * wave + q) + g);
            if (g < 7 && jj < nb) {
                const uint32_t s0 = max(bound[jj], base), s1 = min(bound[jj + 1], base + cnt);
                // rows added in row order, four reads in flight at a time
                const float *row = buf + shift + 9 * (s0 - base) + t;
                uint32_t i = s0;
                for (; i + 4 <= s1; i += 4, row += 36) {
                    const float v0 = row[0], v1 = row[9], v2 = row[18], v3 = row[27];
                    acc[q] = (((acc[q] + v0) + v1) + v2) + v3;
                }
                for (; i < s1; ++i, row += 9) acc[q] += row[0];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kReduceRounds; ++q) {
        const uint32_t jj = (uint32_t)(7 * (kReduceRounds * wave + q) + g);
        if (g < 7 && jj < nb) rec_grad[9 * (size_t)(j0 + jj) + t] = acc[q];
    }
}

template <int TW, int TH, int BATCH>
void fwd_launch(hipStream_t s, const swgs_plan &p, uint8_t *ws, float *images, const float *targets,
                uint32_t tile_lo, uint32_t tile_hi, unsigned long long *counters, float l1_weight,
                bool write_dldc) {
    auto kern = counters ? k_blend_fwd<TW, TH, BATCH, true> : k_blend_fwd<TW, TH, BATCH, false>;
    hipLaunchKernelGGL(kern, dim3(tile_hi - tile_lo), dim3(TW * TH), 0, s,
                       wsp<uint2>(ws, p, WB_TILE_RANGE), wsp<uint32_t>(ws, p, WB_PAIR_VAL),
                       wsp<float4>(ws, p, WB_SPLAT), wsp<ViewDev>(ws, p, WB_VIEWS),
                       (int)p.views.size(), tile_lo, images, wsp<float>(ws, p, WB_T_FINAL),
                       wsp<uint32_t>(ws, p, WB_LAST), targets, write_dldc ? wsp<float>(ws, p, WB_DLDC) : nullptr,
                       wsp<double>(ws, p, WB_LOSS_PART) + 2 * (size_t)tile_lo, counters, l1_weight,
                       p.forward_only ? nullptr : wsp<uint8_t>(ws, p, WB_PAIR_MASK),
                       p.uneven && tile_hi - tile_lo == (uint32_t)p.T ? spread_multiplier(tile_hi - tile_lo) : 0u);
}

template <int TW, int TH, int BATCH>
void bwd_launch(hipStream_t s, const swgs_plan &p, uint8_t *ws, const float *dLdC, uint32_t tile_lo,
                uint32_t tile_hi, unsigned long long *counters) {
    auto kern = counters ? k_blend_bwd<TW, TH, BATCH, true> : k_blend_bwd<TW, TH, BATCH, false>;
    hipLaunchKernelGGL(kern, dim3(tile_hi - tile_lo), dim3(TW * TH), 0, s,
                       wsp<uint2>(ws, p, WB_TILE_RANGE), wsp<uint32_t>(ws, p, WB_PAIR_VAL),
                       wsp<float4>(ws, p, WB_SPLAT), wsp<ViewDev>(ws, p, WB_VIEWS),
                       (int)p.views.size(), tile_lo, wsp<float>(ws, p, WB_T_FINAL),
                       wsp<uint32_t>(ws, p, WB_LAST), dLdC, wsp<uint2>(ws, p, WB_PAIR_BASE),
                       wsp<uint32_t>(ws, p, WB_PAIR_COUNT), wsp<uint8_t>(ws, p, WB_PAIR_MASK),
                       wsp<float>(ws, p, WB_PAIR_GRAD), counters,
                       p.uneven && tile_hi - tile_lo == (uint32_t)p.T ? spread_multiplier(tile_hi - tile_lo) : 0u);
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
                          unsigned long long *counters, float l1_weight, bool write_dldc) {
    if (tile_hi <= tile_lo) return;
    SWGS_DISPATCH_TILE(fwd_launch, s, p, ws, images, targets, tile_lo, tile_hi, counters, l1_weight, write_dldc);
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
    double *part = wsp<double>(ws, p, WB_LOSS_PART);
    double *sums = part + 2 * (size_t)p.T;
    hipLaunchKernelGGL(k_loss_partial, dim3(kLossBlocks), dim3(256), 0, s, part, (int)p.T, sums);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, sums, 1.0 / (3.0 * (double)p.P),
                       wsp<double>(ws, p, WB_STATS));
}

void launch_pair_grad_reduce(hipStream_t s, const swgs_plan &p, uint8_t *ws, uint32_t rec_lo, uint32_t rec_hi) {
    // records [rec_lo, rec_hi), their first gradient rows and the pair
    // total of the same range
    if (rec_hi <= rec_lo) return;
    const uint32_t n = rec_hi - rec_lo;
    hipLaunchKernelGGL(k_pair_grad_reduce, dim3((n + kReduceRecs - 1) / kReduceRecs), dim3(256), 0, s,
                       wsp<uint32_t>(ws, p, WB_ROW_OFFSET) + rec_lo, wsp<uint32_t>(ws, p, WB_PAIR_COUNT),
                       wsp<float>(ws, p, WB_PAIR_GRAD), (uint32_t)p.pair_cap, n,
                       wsp<float>(ws, p, WB_REC_GRAD) + 9 * (size_t)rec_lo);
}

}  // namespace swgs

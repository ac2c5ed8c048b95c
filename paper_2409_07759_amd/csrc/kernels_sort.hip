// Per-tile depth sort and the device-wide exclusive scan, hand-written for
// gfx950 (wave64).
//
// Sorting puts the Gaussians of each tile in depth order, "close to far"
// (Sec. 2.1).  After binning, a tile's pairs sit contiguously in an
// arbitrary order; each tile is sorted by the unique 64-bit key
// (FP32 depth bits << 32 | record), so the result is deterministic and ties
// in depth go by record (= by slot within a view).  FP32 depths of visible
// Gaussians are positive, so their bit patterns order like the values.
//
// k_tile_sort: one workgroup per tile, bitonic sort in LDS of up to
// kTileSortCap keys (the paper-scale window has at most ~600 pairs per
// 16x16 tile).  Larger tiles are listed and sorted by k_tile_sort_big:
// bitonic-sorted runs of kTileSortCap in LDS, then merge passes in global
// memory between the pair buffers and their alternates, each merge split
// over the workgroup's threads by merge-path diagonals.
#include "swgs_internal.h"

namespace swgs {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr uint32_t kTileSortCap = 4096;

__device__ __forceinline__ uint64_t pair_key64(uint32_t key, uint32_t val) {
    return ((uint64_t)key << 32) | (uint64_t)val;
}

// ascending bitonic sort of s[0, P), P a power of two; every thread of the
// block calls it
__device__ void block_bitonic(uint64_t *s, uint32_t P) {
    for (uint32_t k = 2; k <= P; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < P; i += kBlock) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint64_t a = s[i], b = s[l];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        s[i] = b;
                        s[l] = a;
                    }
                }
            }
            __syncthreads();
        }
}

// load n <= kTileSortCap pairs into LDS (padded with the largest key),
// sort, store back in place
__device__ void sort_run(uint64_t *s, uint32_t *keys, uint32_t *vals, uint32_t n) {
    uint32_t P = 1;
    while (P < n) P <<= 1;
    for (uint32_t i = threadIdx.x; i < P; i += kBlock) s[i] = i < n ? pair_key64(keys[i], vals[i]) : ~0ull;
    __syncthreads();
    block_bitonic(s, P);
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
        keys[i] = (uint32_t)(s[i] >> 32);
        vals[i] = (uint32_t)s[i];
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kBlock)
k_tile_sort(const uint2 *__restrict__ ranges, uint32_t tile_lo, uint32_t *__restrict__ keys,
            uint32_t *__restrict__ vals, uint32_t *__restrict__ big_list, uint32_t *__restrict__ big_count) {
    __shared__ uint64_t s[kTileSortCap];
    const uint32_t tile = tile_lo + blockIdx.x;
    const uint2 rg = ranges[tile];
    const uint32_t n = rg.y - rg.x;
    if (n <= 1) return;
    if (n > kTileSortCap) {
        if (threadIdx.x == 0) big_list[atomicAdd(big_count, 1u)] = tile;
        return;
    }
    sort_run(s, keys + rg.x, vals + rg.x, n);
}

// merge sorted runs a[0, la) and b[0, lb) into o[0, la + lb); thread t
// produces a contiguous share of the output from the merge-path split at
// its first output diagonal
__device__ void merge_runs(const uint32_t *ak, const uint32_t *av, uint32_t la, const uint32_t *bk,
                           const uint32_t *bv, uint32_t lb, uint32_t *ok, uint32_t *ov) {
    const uint32_t L = la + lb;
    const uint32_t per = (L + kBlock - 1) / kBlock;
    const uint32_t d0 = min(L, threadIdx.x * per), d1 = min(L, d0 + per);
    if (d0 >= d1) return;
    uint32_t lo = d0 > lb ? d0 - lb : 0, hi = min(d0, la);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pair_key64(ak[mid], av[mid]) < pair_key64(bk[d0 - mid - 1], bv[d0 - mid - 1])) lo = mid + 1;
        else hi = mid;
    }
    uint32_t i = lo, j = d0 - lo;
    for (uint32_t d = d0; d < d1; ++d) {
        const bool take_a = j >= lb || (i < la && pair_key64(ak[i], av[i]) < pair_key64(bk[j], bv[j]));
        if (take_a) {
            ok[d] = ak[i];
            ov[d] = av[i];
            ++i;
        } else {
            ok[d] = bk[j];
            ov[d] = bv[j];
            ++j;
        }
    }
}

// tiles with more than kTileSortCap pairs; a fixed grid walks the list
// whose length is known only on the device
__global__ void __launch_bounds__(kBlock)
k_tile_sort_big(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ big_list,
                const uint32_t *__restrict__ big_count, uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                uint32_t *__restrict__ keys_alt, uint32_t *__restrict__ vals_alt) {
    __shared__ uint64_t s[kTileSortCap];
    const uint32_t nb = *big_count;
    for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const uint2 rg = ranges[big_list[b]];
        const uint32_t lo = rg.x, n = rg.y - rg.x;
        for (uint32_t c0 = 0; c0 < n; c0 += kTileSortCap)
            sort_run(s, keys + lo + c0, vals + lo + c0, min(kTileSortCap, n - c0));
        uint32_t *sk = keys + lo, *sv = vals + lo, *dk = keys_alt + lo, *dv = vals_alt + lo;
        for (uint32_t w = kTileSortCap; w < n; w <<= 1) {
            for (uint32_t a0 = 0; a0 < n; a0 += 2 * w) {
                const uint32_t la = min(w, n - a0);
                const uint32_t lb = a0 + w < n ? min(w, n - a0 - w) : 0;
                merge_runs(sk + a0, sv + a0, la, sk + a0 + la, sv + a0 + la, lb, dk + a0, dv + a0);
            }
            __syncthreads();
            uint32_t *t = sk; sk = dk; dk = t;
            t = sv; sv = dv; dv = t;
        }
        if (sk != keys + lo)
            for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
                keys[lo + i] = sk[i];
                vals[lo + i] = sv[i];
            }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- scan
constexpr int kScanChunk = 4096;

__device__ __forceinline__ uint32_t scan_in(const uint32_t *in, const uint32_t *idx, uint32_t i) {
    return idx ? in[idx[i]] : in[i];
}

__global__ void __launch_bounds__(kBlock)
k_scan_reduce(const uint32_t *__restrict__ in, const uint32_t *__restrict__ idx, uint32_t n,
              uint32_t *__restrict__ sums) {
    __shared__ uint32_t wsum[kWaves];
    const uint32_t lo = blockIdx.x * kScanChunk;
    uint32_t s = 0;
    for (uint32_t i = lo + threadIdx.x; i < min(n, lo + kScanChunk); i += kBlock) s += scan_in(in, idx, i);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) sums[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ void __launch_bounds__(kBlock)
k_scan_sums(uint32_t *__restrict__ sums, uint32_t nb, uint32_t *__restrict__ total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nb; b0 += kBlock) {
        uint32_t i = b0 + threadIdx.x;
        uint32_t v = i < nb ? sums[i] : 0;
        uint32_t x = v;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (i < nb) sums[i] = before + x - v;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) carry = before + x;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void __launch_bounds__(kBlock)
k_scan_write(const uint32_t *__restrict__ in, const uint32_t *__restrict__ idx, uint32_t n,
             const uint32_t *__restrict__ sums, uint32_t *__restrict__ out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ uint32_t wsum[kWaves];
    uint32_t carry = sums[blockIdx.x];
    const uint32_t lo = blockIdx.x * kScanChunk;
    for (uint32_t t0 = lo; t0 < min(n, lo + kScanChunk); t0 += kBlock) {
        uint32_t i = t0 + threadIdx.x;
        uint32_t v = i < n ? scan_in(in, idx, i) : 0;
        uint32_t x = v;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (i < n) out[i] = before + x - v;
        uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
        carry += tot;
    }
}

}  // namespace

void launch_tile_sort(hipStream_t s, const swgs_plan &p, uint8_t *ws, uint32_t tile_lo, uint32_t tile_hi) {
    if (tile_hi <= tile_lo) return;
    uint32_t *big = wsp<uint32_t>(ws, p, WB_BIG_TILES);
    uint32_t *big_count = big + (p.T + 1);
    launch_fill_u32(s, big_count, 0, 1);
    hipLaunchKernelGGL(k_tile_sort, dim3(tile_hi - tile_lo), dim3(kBlock), 0, s, wsp<uint2>(ws, p, WB_TILE_RANGE),
                       tile_lo, wsp<uint32_t>(ws, p, WB_PAIR_KEY), wsp<uint32_t>(ws, p, WB_PAIR_VAL), big, big_count);
    hipLaunchKernelGGL(k_tile_sort_big, dim3(64), dim3(kBlock), 0, s, wsp<uint2>(ws, p, WB_TILE_RANGE), big,
                       big_count, wsp<uint32_t>(ws, p, WB_PAIR_KEY), wsp<uint32_t>(ws, p, WB_PAIR_VAL),
                       wsp<uint32_t>(ws, p, WB_PAIR_KEY_ALT), wsp<uint32_t>(ws, p, WB_PAIR_VAL_ALT));
}

void exclusive_scan_u32(hipStream_t s, const uint32_t *in, uint32_t *out, uint32_t n,
                        uint32_t *total_out, uint32_t *scratch) {
    // scratch: at least ceil(n / kScanChunk) + 1 words; idx via the
    // gather variant below
    const uint32_t nb = (n + kScanChunk - 1) / kScanChunk;
    if (nb == 0) {
        launch_fill_u32(s, total_out, 0, 1);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, in, (const uint32_t *)nullptr, n, scratch);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, scratch, nb, total_out);
    hipLaunchKernelGGL(k_scan_write, dim3(nb), dim3(kBlock), 0, s, in, (const uint32_t *)nullptr, n, scratch,
                       out);
}

void exclusive_scan_gather_u32(hipStream_t s, const uint32_t *in, const uint32_t *idx, uint32_t *out,
                               uint32_t n, uint32_t *total_out, uint32_t *scratch) {
    const uint32_t nb = (n + kScanChunk - 1) / kScanChunk;
    if (nb == 0) {
        launch_fill_u32(s, total_out, 0, 1);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, in, idx, n, scratch);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, scratch, nb, total_out);
    hipLaunchKernelGGL(k_scan_write, dim3(nb), dim3(kBlock), 0, s, in, idx, n, scratch, out);
}

}  // namespace swgs

// Device-wide stable LSD radix sort of (uint32 key, uint32 value) pairs and
// an exclusive scan, hand-written for gfx950 (wave64).
//
// Sorting puts the splats of each tile in depth order, "close to far"
// (Sec. 2.1): the records are first sorted by FP32 depth bits, then the
// (tile, record) pairs emitted in that order are stably sorted by tile.
//
// One pass = histogram (LDS atomics per block) -> per-digit scan of the
// block counts -> stable scatter.  The grid is a fixed kSortBlocks blocks;
// block b owns the contiguous range [b L, (b+1) L) with L = ceil(n / B), so
// the element count may live on the device (graph-friendly).  Inside a block
// the stable rank of an element among equal digits comes from ballot-based
// match masks within the wave and per-wave digit counts in LDS.
// Keys take the fewest passes of at most 8-bit digits; with an odd pass
// count the caller places the input in the alternate buffers, so that the
// sorted data always ends in the primary ones.
#include "swgs_internal.h"

namespace swgs {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxDigitBits = 8;
constexpr int kMaxBins = 1 << kMaxDigitBits;
constexpr int kChunkRounds = 8;                   // rounds of kBlock elements per LDS chunk
constexpr int kChunk = kBlock * kChunkRounds;

// the scatter's count rows are cleared as 32-bit words and written as 16-bit
// counts: both through may_alias types, so neither store can be reordered
// across the other
typedef uint16_t __attribute__((may_alias)) u16_alias;
typedef uint32_t __attribute__((may_alias)) u32_alias;

__device__ __forceinline__ uint32_t resolve_n(const uint32_t *d_n, uint32_t n_fixed, uint32_t cap) {
    uint32_t n = d_n ? *d_n : n_fixed;
    return n < cap ? n : cap;
}

__global__ void __launch_bounds__(kBlock)
k_hist(const uint32_t *__restrict__ keys, const uint32_t *d_n, uint32_t n_fixed, uint32_t cap,
       int shift, int bins, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[kMaxBins];
    for (int i = threadIdx.x; i < bins; i += kBlock) h[i] = 0;
    __syncthreads();
    const uint32_t n = resolve_n(d_n, n_fixed, cap);
    const uint32_t L = (n + gridDim.x - 1) / gridDim.x;
    const uint32_t lo = blockIdx.x * L;
    const uint32_t hi = min(n, lo + L);
    const uint32_t mask = (uint32_t)bins - 1;
    constexpr int U = 8;   // loads in flight per thread
    for (uint32_t i0 = lo; i0 < hi; i0 += U * kBlock) {
        uint32_t kk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = i0 + (uint32_t)(u * kBlock) + threadIdx.x;
            kk[u] = i < hi ? keys[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + (uint32_t)(u * kBlock) + threadIdx.x < hi) atomicAdd(&h[(kk[u] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < bins; d += kBlock) hist[(size_t)d * gridDim.x + blockIdx.x] = h[d];
}

// one block per digit: exclusive scan over the kSortBlocks block counts
__global__ void __launch_bounds__(kBlock)
k_digit_scan(uint32_t *__restrict__ hist, int nblocks, uint32_t *__restrict__ totals) {
    const int d = blockIdx.x;
    uint32_t *c = hist + (size_t)d * nblocks;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nblocks; b0 += kBlock) {
        int i = b0 + threadIdx.x;
        uint32_t v = i < nblocks ? c[i] : 0;
        uint32_t x = v;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (i < nblocks) c[i] = before + x - v;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) carry = before + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[d] = carry;
}

// Stable scatter of one pass.  The block walks its range in chunks of
// kChunk elements, element r kBlock + t of a chunk held by thread t in
// round r (so stable order is (round, wave, lane)).  Per chunk:
//   1. every wave ranks its elements of each round among equal digits by
//      ballot match masks and records the round's per-digit counts;
//   2. one thread per digit turns its counts, in (round, wave) order, into
//      exclusive prefixes, and a block scan of the digit totals gives each
//      digit's run inside the chunk;
//   3. every element goes to run start + prefix + rank in an LDS copy of the
//      chunk ordered by digit, which is then written out run by run, so
//      consecutive threads write consecutive addresses of one digit's run.
__global__ void __launch_bounds__(kBlock, 4)   // 4 blocks per CU: the whole grid resident at once
k_scatter(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals, const uint32_t *d_n,
          uint32_t n_fixed, uint32_t cap, int shift, int dbits, const uint32_t *__restrict__ hist,
          const uint32_t *__restrict__ totals, uint32_t *__restrict__ keys_out,
          uint32_t *__restrict__ vals_out, const uint2 *__restrict__ grect, uint2 *__restrict__ rect_out,
          uint32_t *__restrict__ count_out) {
    const int bins = 1 << dbits;
    __shared__ uint32_t gbase[kMaxBins];          // next global position of each digit for this block
    __shared__ uint32_t coff[kMaxBins];           // start of each digit's run inside the chunk
    __shared__ uint32_t ctot[kMaxBins];           // elements of each digit in the chunk
    // per (round, wave, digit): count, then exclusive prefix inside the digit's run
    __shared__ __align__(8) uint16_t wcnt[kChunkRounds][kWaves][kMaxBins];
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t skey[kChunk], sval[kChunk];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    // exclusive scan of x over threads 0..kBlock-1 (x = 0 past the digits)
    auto block_exclusive = [&](uint32_t v) {
        uint32_t x = v;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        __syncthreads();   // wsum is reused by the next scan
        return before + x - v;
    };

    // digit bases: exclusive prefix of the digit totals + this block's offset
    {
        const uint32_t v = (int)threadIdx.x < bins ? totals[threadIdx.x] : 0;
        const uint32_t ex = block_exclusive(v);
        if ((int)threadIdx.x < bins) gbase[threadIdx.x] = ex + hist[(size_t)threadIdx.x * gridDim.x + blockIdx.x];
    }

    const uint32_t n = resolve_n(d_n, n_fixed, cap);
    const uint32_t L = (n + gridDim.x - 1) / gridDim.x;
    const uint32_t lo = blockIdx.x * L;
    const uint32_t hi = min(n, lo + L);
    const uint32_t mask = (uint32_t)bins - 1;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int words = (bins + 1) / 2;             // 32-bit words of one count row
    // the next chunk's keys and values are loaded while this one is placed
    uint32_t kn[kChunkRounds], vn[kChunkRounds];
    auto load_chunk = [&](uint32_t c0) {
#pragma unroll
        for (int r = 0; r < kChunkRounds; ++r) {
            const uint32_t i = c0 + (uint32_t)(r * kBlock) + threadIdx.x;
            kn[r] = i < hi ? keys[i] : 0u;
            vn[r] = i < hi ? vals[i] : 0u;
        }
    };
    if (lo < hi) load_chunk(lo);
    for (uint32_t c0 = lo; c0 < hi; c0 += kChunk) {
        const uint32_t cn = min((uint32_t)kChunk, hi - c0);
        uint32_t k[kChunkRounds], v[kChunkRounds], dg[kChunkRounds], rk[kChunkRounds];
#pragma unroll
        for (int r = 0; r < kChunkRounds; ++r) {
            const uint32_t i = (uint32_t)(r * kBlock) + threadIdx.x;
            const bool ok = i < cn;
            k[r] = kn[r];
            v[r] = vn[r];
            dg[r] = ok ? (k[r] >> shift) & mask : (uint32_t)bins;   // bins = no element
        }
        if (c0 + kChunk < hi) load_chunk(c0 + kChunk);
        // 1. per-wave ranks and counts (a wave's LDS operations take effect
        // in program order, so clearing its own rows needs no barrier)
#pragma unroll
        for (int r = 0; r < kChunkRounds; ++r) {
            u32_alias *row = reinterpret_cast<u32_alias *>(&wcnt[r][wave][0]);
            for (int w = lane; w < words; w += 64) row[w] = 0u;
            const uint32_t d = dg[r];
            const bool ok = d < (uint32_t)bins;
            uint64_t peers = __ballot(ok);
            for (int b = 0; b < dbits; ++b) {
                const uint64_t m = __ballot(ok && ((d >> b) & 1u));
                peers &= ((d >> b) & 1u) ? m : ~m;
            }
            rk[r] = (uint32_t)__popcll(peers & lt);
            if (ok && (peers & lt) == 0) reinterpret_cast<u16_alias *>(&wcnt[r][wave][0])[d] = (uint16_t)__popcll(peers);
        }
        __syncthreads();
        // 2. exclusive prefixes per digit in (round, wave) order, and the
        // digits' runs inside the chunk
        uint32_t tot = 0;
        if ((int)threadIdx.x < bins) {
            uint16_t c[kChunkRounds * kWaves];
#pragma unroll
            for (int q = 0; q < kChunkRounds * kWaves; ++q) c[q] = wcnt[q / kWaves][q % kWaves][threadIdx.x];
#pragma unroll
            for (int q = 0; q < kChunkRounds * kWaves; ++q) {
                wcnt[q / kWaves][q % kWaves][threadIdx.x] = (uint16_t)tot;
                tot += c[q];
            }
            ctot[threadIdx.x] = tot;
        }
        const uint32_t ex = block_exclusive(tot);
        if ((int)threadIdx.x < bins) coff[threadIdx.x] = ex;
        __syncthreads();
        // 3. placement in digit order, then the write-out run by run
#pragma unroll
        for (int r = 0; r < kChunkRounds; ++r) {
            const uint32_t d = dg[r];
            if (d < (uint32_t)bins) {
                const uint32_t pos = coff[d] + wcnt[r][wave][d] + rk[r];
                skey[pos] = k[r];
                sval[pos] = v[r];
            }
        }
        __syncthreads();
        for (uint32_t p = threadIdx.x; p < cn; p += kBlock) {
            const uint32_t key = skey[p];
            const uint32_t d = (key >> shift) & mask;
            const uint32_t o = gbase[d] + (p - coff[d]);
            keys_out[o] = key;
            vals_out[o] = sval[p];
            if (grect) {
                // the record's tile rectangle and tile count, in sorted order
                const uint2 rc = grect[sval[p]];
                rect_out[o] = rc;
                count_out[o] = ((rc.y & 0xFFFFu) - (rc.x & 0xFFFFu)) * ((rc.y >> 16) - (rc.x >> 16));
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < bins) gbase[threadIdx.x] += ctot[threadIdx.x];
        // the next chunk's first barrier orders this update before any read
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

// with slot_base, element i is a record's tile count: its first row r goes
// to out[i] and (r - y0 w - x0, w) of its rect (rect[i]) to slot_base[i]
__global__ void __launch_bounds__(kBlock)
k_scan_write(const uint32_t *in, const uint32_t *__restrict__ idx, uint32_t n,
             const uint32_t *__restrict__ sums, uint32_t *out,   // in may equal out (in-place scan)
             const uint2 *__restrict__ rect, uint2 *__restrict__ slot_base) {
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
        if (slot_base && i < n) {
            const uint2 rc = rect[i];
            const uint32_t w = max((rc.y & 0xFFFFu) - (rc.x & 0xFFFFu), 1u);
            slot_base[i] = make_uint2(before + x - v - (rc.x >> 16) * w - (rc.x & 0xFFFFu), w);
        }
        uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
        carry += tot;
    }
}

}  // namespace

int radix_passes(int bits) {
    if (bits < 1) bits = 1;
    if (bits > 32) bits = 32;
    return (bits + kMaxDigitBits - 1) / kMaxDigitBits;   // fewest passes whose digits fit
}

bool radix_input_in_alt(int bits) { return radix_passes(bits) & 1; }

void radix_sort_pairs(hipStream_t s, uint32_t *keys, uint32_t *vals, uint32_t *keys_alt,
                      uint32_t *vals_alt, const uint32_t *d_n, uint32_t n_fixed, uint32_t cap,
                      int bits, uint32_t *hist, uint32_t *totals, const uint2 *gather_rect,
                      uint2 *rect_out, uint32_t *count_out) {
    if (bits < 1) bits = 1;
    if (bits > 32) bits = 32;
    const int passes = radix_passes(bits);
    const int dbits = (bits + passes - 1) / passes;
    // an odd pass count starts from the alternate buffers, so that the
    // last pass writes (keys, vals)
    const bool odd = passes & 1;
    uint32_t *ki = odd ? keys_alt : keys, *vi = odd ? vals_alt : vals;
    uint32_t *ko = odd ? keys : keys_alt, *vo = odd ? vals : vals_alt;
    int shift = 0;
    for (int p = 0; p < passes; ++p) {
        int w = dbits;
        if (shift + w > 32) w = 32 - shift;
        if (w < 1) w = 1;
        const int bins = 1 << w;
        hipLaunchKernelGGL(k_hist, dim3(kSortBlocks), dim3(kBlock), 0, s, ki, d_n, n_fixed, cap, shift, bins,
                           hist);
        hipLaunchKernelGGL(k_digit_scan, dim3(bins), dim3(kBlock), 0, s, hist, kSortBlocks, totals);
        const bool last = p + 1 == passes;
        hipLaunchKernelGGL(k_scatter, dim3(kSortBlocks), dim3(kBlock), 0, s, ki, vi, d_n, n_fixed, cap, shift,
                           w, hist, totals, ko, vo, last ? gather_rect : nullptr, rect_out, count_out);
        shift += w;
        uint32_t *t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
}

void exclusive_scan_u32(hipStream_t s, const uint32_t *in, uint32_t *out, uint32_t n,
                        uint32_t *total_out, uint32_t *scratch) {
    // scratch: at least ceil(n / kScanChunk) + 1 words; in may equal out
    const uint32_t nb = (n + kScanChunk - 1) / kScanChunk;
    if (nb == 0) {
        launch_fill_u32(s, total_out, 0, 1);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, in, (const uint32_t *)nullptr, n, scratch);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, scratch, nb, total_out);
    hipLaunchKernelGGL(k_scan_write, dim3(nb), dim3(kBlock), 0, s, in, (const uint32_t *)nullptr, n, scratch,
                       out, (const uint2 *)nullptr, (uint2 *)nullptr);
}

void exclusive_scan_rows(hipStream_t s, const uint32_t *count, const uint2 *rect, uint32_t n, uint32_t *first,
                         uint2 *slot_base, uint32_t *scratch) {
    const uint32_t nb = (n + kScanChunk - 1) / kScanChunk;
    if (nb == 0) return;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, count, (const uint32_t *)nullptr, n, scratch);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, scratch, nb, (uint32_t *)nullptr);
    hipLaunchKernelGGL(k_scan_write, dim3(nb), dim3(kBlock), 0, s, count, (const uint32_t *)nullptr, n, scratch,
                       first, rect, slot_base);
}


}  // namespace swgs

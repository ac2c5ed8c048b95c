// Lifespan gating and compaction (Sec. 4.2: a Gaussian takes part in a
// frame only if start <= frame < expire; Algorithm 1 applies the filter to
// the optimisable and the frozen set alike).
//
// For every distinct frame g of a plan the live slots are compacted, in
// ascending slot order, into a list; one more list holds the window set A
// (optimisable slots live in at least one frame of the plan).  Three
// launches over a fixed chunking of the slots: count per chunk, scan of
// the chunk counts per group, stable write (wave ballots + LDS prefix).
// All integer work, bit-exact and deterministic.
#include "swgs_internal.h"

namespace swgs {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kPerThread = kGateChunk / kBlock;

__device__ __forceinline__ bool live_at(int32_t s, int32_t e, int32_t f) { return s <= f && f < e; }

// predicate of group g (g == n_groups: the window set A)
__device__ __forceinline__ bool gate_pred(const int32_t *__restrict__ start,
                                          const int32_t *__restrict__ expire,
                                          const GroupDev *__restrict__ groups, int n_groups,
                                          int num_gs, int g, int slot) {
    int32_t s = start[slot], e = expire[slot];
    if (g < n_groups) return live_at(s, e, groups[g].frame);
    if (slot >= num_gs) return false;
    bool any = false;
    for (int k = 0; k < n_groups; ++k) any |= live_at(s, e, groups[k].frame);
    return any;
}

__global__ void __launch_bounds__(kBlock)
k_gate_count(const int32_t *__restrict__ start, const int32_t *__restrict__ expire,
             const GroupDev *__restrict__ groups, int n_groups, int num_gs, int n_slots,
             int nblk, uint32_t *__restrict__ blk_count, uint32_t *__restrict__ stale) {
    const int g = blockIdx.y;
    const int base = blockIdx.x * kGateChunk;
    __shared__ uint32_t wsum[kWaves];
    if (stale && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *stale = 0u;   // set by k_gate_scan
    uint32_t c = 0;
    for (int k = 0; k < kPerThread; ++k) {
        int slot = base + k * kBlock + threadIdx.x;
        if (slot < n_slots && gate_pred(start, expire, groups, n_groups, num_gs, g, slot)) ++c;
    }
    // wave sum then block sum
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWaves; ++w) t += wsum[w];
        blk_count[(size_t)g * nblk + blockIdx.x] = t;
    }
}

// one block per group: exclusive scan of the chunk counts in place
__global__ void __launch_bounds__(kBlock)
k_gate_scan(uint32_t *__restrict__ blk_count, int nblk, uint32_t *__restrict__ totals,
            const GroupDev *__restrict__ groups, int n_groups, uint32_t nA_cap, uint32_t *__restrict__ stale) {
    const int g = blockIdx.x;
    uint32_t *c = blk_count + (size_t)g * nblk;
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int b0 = 0; b0 < nblk; b0 += kBlock) {
        int i = b0 + threadIdx.x;
        uint32_t v = i < nblk ? c[i] : 0;
        // inclusive wave scan
        uint32_t x = v;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (i < nblk) c[i] = before + x - v;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) carry = before + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        totals[g] = carry;
        // a live count that differs from the plan's means the lifespans
        // changed after the plan was made: its lists are stale
        if (stale && carry != (g < n_groups ? groups[g].n_live : nA_cap)) atomicOr(stale, 1u);
    }
}

__global__ void __launch_bounds__(kBlock)
k_gate_write(const int32_t *__restrict__ start, const int32_t *__restrict__ expire,
             const GroupDev *__restrict__ groups, int n_groups, int num_gs, int n_slots, int nblk,
             const uint32_t *__restrict__ blk_offset, uint32_t list_A_base, uint32_t nA_cap,
             uint32_t *__restrict__ lists, int32_t *__restrict__ pos_of) {
    const int g = blockIdx.y;
    const int base = blockIdx.x * kGateChunk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ uint32_t wcount[kWaves];
    uint32_t running = blk_offset[(size_t)g * nblk + blockIdx.x];
    const uint32_t list_base = g < n_groups ? groups[g].list_base : list_A_base;
    // capacity fixed at plan time: a plan used after the lifespans changed
    // never writes outside its own list
    const uint32_t list_cap = g < n_groups ? groups[g].n_live : nA_cap;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int k = 0; k < kPerThread; ++k) {
        int slot = base + k * kBlock + threadIdx.x;
        bool f = slot < n_slots && gate_pred(start, expire, groups, n_groups, num_gs, g, slot);
        uint64_t m = __ballot(f);
        if (lane == 0) wcount[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = running;
        for (int w = 0; w < wave; ++w) before += wcount[w];
        uint32_t pos = before + (uint32_t)__popcll(m & lt);
        const bool fits = f && pos < list_cap;
        if (fits) lists[list_base + pos] = (uint32_t)slot;
        if (g < n_groups && slot < num_gs) pos_of[(size_t)g * num_gs + slot] = fits ? (int32_t)pos : -1;
        uint32_t tot = 0;
        for (int w = 0; w < kWaves; ++w) tot += wcount[w];
        __syncthreads();
        running += tot;
    }
}

__global__ void __launch_bounds__(kBlock)
k_count_live(const int32_t *__restrict__ start, const int32_t *__restrict__ expire, int n_slots,
             int num_gs, const int32_t *__restrict__ frames, int n_frames,
             uint32_t *__restrict__ out) {
    const int g = blockIdx.y;
    __shared__ uint32_t wsum[kWaves];
    uint32_t c = 0;
    for (int slot = blockIdx.x * kBlock + threadIdx.x; slot < n_slots; slot += gridDim.x * kBlock) {
        int32_t s = start[slot], e = expire[slot];
        bool f;
        if (g < n_frames) {
            f = live_at(s, e, frames[g]);
        } else {
            f = false;
            if (slot < num_gs)
                for (int k = 0; k < n_frames; ++k) f |= live_at(s, e, frames[k]);
        }
        c += f ? 1u : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWaves; ++w) t += wsum[w];
        if (t) atomicAdd(out + g, t);
    }
}

}  // namespace

void launch_gate(hipStream_t s, const swgs_plan &p, uint8_t *ws) {
    const int S = p.pool.n_slots;
    const int G = (int)p.groups.size();
    const int nblk = (S + kGateChunk - 1) / kGateChunk;
    auto *blk = wsp<uint32_t>(ws, p, WB_GATE_BLK);
    auto *groups = wsp<GroupDev>(ws, p, WB_GROUPS);
    dim3 grid(nblk, G + 1);
    // word 3 of the pair-count block: set when a live count differs from the plan's
    uint32_t *stale = wsp<uint32_t>(ws, p, WB_PAIR_COUNT) + 3;
    hipLaunchKernelGGL(k_gate_count, grid, dim3(kBlock), 0, s, p.pool.start, p.pool.expire, groups, G,
                       p.pool.num_gs, S, nblk, blk, stale);
    hipLaunchKernelGGL(k_gate_scan, dim3(G + 1), dim3(kBlock), 0, s, blk, nblk,
                       wsp<uint32_t>(ws, p, WB_ACTIVE_COUNT), groups, G, p.n_A, stale);
    hipLaunchKernelGGL(k_gate_write, grid, dim3(kBlock), 0, s, p.pool.start, p.pool.expire, groups, G,
                       p.pool.num_gs, S, nblk, blk, p.list_A_base, p.n_A, wsp<uint32_t>(ws, p, WB_ACTIVE_LIST),
                       wsp<int32_t>(ws, p, WB_POS_OF));
}

void launch_frame_lists(hipStream_t s, const int32_t *start, const int32_t *expire, int n_slots,
                        const GroupDev *groups, int n_groups, uint32_t *blk, uint32_t *totals, uint32_t *lists) {
    // the gating kernels with no optimisable slots (num_gs = 0): the extra
    // group row (window set) stays empty and pos_of is never written
    const int nblk = (n_slots + kGateChunk - 1) / kGateChunk;
    dim3 grid(nblk, n_groups + 1);
    hipLaunchKernelGGL(k_gate_count, grid, dim3(kBlock), 0, s, start, expire, groups, n_groups, 0, n_slots, nblk,
                       blk, nullptr);
    hipLaunchKernelGGL(k_gate_scan, dim3(n_groups + 1), dim3(kBlock), 0, s, blk, nblk, totals, groups, n_groups,
                       0u, nullptr);
    hipLaunchKernelGGL(k_gate_write, grid, dim3(kBlock), 0, s, start, expire, groups, n_groups, 0, n_slots, nblk,
                       blk, 0u, 0u, lists, nullptr);
}

void launch_count_live(hipStream_t s, const int32_t *start, const int32_t *expire, int n_slots,
                       int num_gs, const int32_t *frames, int n_frames, uint32_t *out_counts) {
    int nb = (n_slots + kBlock - 1) / kBlock;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_count_live, dim3(nb, n_frames + 1), dim3(kBlock), 0, s, start, expire, n_slots,
                       num_gs, frames, n_frames, out_counts);
}

}  // namespace swgs

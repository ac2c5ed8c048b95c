// Compact per-frame update record: encoding of a mature record and its
// decoding on the client.
//
// What a frame streams follows Sec. 5.2 (Eq. 4), Sec. 5.6.2 and Table 6:
// per Gaussian its mean, scale, rotation, opacity and the DC term of its
// spherical harmonics, either in FP32 (56 bytes) or at Table 6's precisions
// (FP16 mean and scale, 8-bit rotation and opacity, FP32 DC: 29 bytes).
// Sec. 5.5's bandwidth adaptation keeps a slice's most opaque Gaussians and
// marks the rest empty.  The record layout and the rounding rules are
// documented with swgs_encode_update in swgs.h; every rounding decision is
// taken with IEEE-exact FP32 operations (FMA contraction off, correctly
// rounded square root and division) so that it can be reproduced exactly.
#include <cmath>

#include "swgs_internal.h"

namespace swgs {
namespace {

constexpr int kBlock = 256;
constexpr int32_t kMagic = 0x53475753;
constexpr int kEncFp32 = 1, kEncQ = 2;
constexpr int kFlagLifespans = 1, kFlagMask = 2;
constexpr float kHalfMax = 65504.0f;

__host__ __device__ inline size_t align16(size_t n) { return (n + 15) / 16 * 16; }

// 255 opacity thresholds (logit of (k - 1/2) / 255) and 256 decoded logits
struct OpacityThresholds {
    float t[255];
};
struct OpacityDecode {
    float v[256];
};

// v1 record views
struct V1 {
    const uint32_t *slot;
    const int32_t *birth, *start, *expire;
    const float *params;
};
inline V1 v1_view(const uint8_t *rec, uint32_t n) {
    V1 v;
    v.slot = reinterpret_cast<const uint32_t *>(rec + 32);
    v.birth = reinterpret_cast<const int32_t *>(rec + 32 + 4 * (size_t)n);
    v.start = reinterpret_cast<const int32_t *>(rec + 32 + 8 * (size_t)n);
    v.expire = reinterpret_cast<const int32_t *>(rec + 32 + 12 * (size_t)n);
    v.params = reinterpret_cast<const float *>(rec + 32 + 16 * (size_t)n);
    return v;
}

// byte offsets of the v2 sections
struct Sections {
    size_t life = 0, mask = 0, mean = 0, scale = 0, quat = 0, opac = 0, dc = 0, total = 0;
};
Sections sections(uint32_t n, uint32_t m, int enc, bool uniform, bool masked) {
    Sections s;
    size_t o = 64;
    if (!uniform) {
        s.life = o;
        o += 4 * align16(4 * (size_t)n);
    }
    if (masked) {
        s.mask = o;
        o += align16(4 * (((size_t)n + 31) / 32));
    }
    const size_t b[5] = {enc == kEncFp32 ? 12u : 6u, enc == kEncFp32 ? 12u : 6u, enc == kEncFp32 ? 16u : 4u,
                         enc == kEncFp32 ? 4u : 1u, 12u};
    size_t *dst[5] = {&s.mean, &s.scale, &s.quat, &s.opac, &s.dc};
    for (int i = 0; i < 5; ++i) {
        *dst[i] = o;
        o += align16(b[i] * m);
    }
    s.total = o;
    return s;
}

__global__ void __launch_bounds__(kBlock)
k_enc_uniform(const uint32_t *__restrict__ slot, const int32_t *__restrict__ birth, const int32_t *__restrict__ start,
              const int32_t *__restrict__ expire, uint32_t n, uint32_t *__restrict__ flag) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const bool diff = birth[k] != birth[0] || start[k] != start[0] || expire[k] != expire[0] ||
                      slot[k] != slot[0] + k;
    if (diff) atomicOr(flag, 1u);
}

// descending order of the opacity logit as an ascending uint32 key
__global__ void __launch_bounds__(kBlock)
k_enc_keys(const float *__restrict__ logit, uint32_t n, uint32_t *__restrict__ key, uint32_t *__restrict__ val) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const uint32_t u = __float_as_uint(logit[k]);
    const uint32_t asc = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    key[k] = ~asc;
    val[k] = k;
}

__global__ void __launch_bounds__(kBlock)
k_enc_mark(const uint32_t *__restrict__ sorted_idx, uint32_t keep, uint32_t *__restrict__ mask,
           uint32_t *__restrict__ kept) {
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= keep) return;
    const uint32_t e = sorted_idx[r];
    atomicOr(&mask[e >> 5], 1u << (e & 31));
    kept[e] = 1u;
}

__device__ __forceinline__ uint16_t to_half_bits(float x) {
    x = fminf(fmaxf(x, -kHalfMax), kHalfMax);
    return __builtin_bit_cast(uint16_t, static_cast<_Float16>(x));
}

#pragma clang fp contract(off)
__device__ __forceinline__ void quat_codes(float q0, float q1, float q2, float q3, uint8_t c[4]) {
    const float n2 = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
    float u[4] = {1.0f, 0.0f, 0.0f, 0.0f};
    if (n2 != 0.0f) {
        const float n = sqrtf(n2);   // correctly rounded (HIP's default for FP32 sqrt and division)
        u[0] = q0 / n;
        u[1] = q1 / n;
        u[2] = q2 / n;
        u[3] = q3 / n;
    }
    for (int i = 0; i < 4; ++i) {
        float t = u[i] * 127.5f;
        t = t + 127.5f;
        c[i] = (uint8_t)fminf(fmaxf(rintf(t), 0.0f), 255.0f);
    }
}

__device__ __forceinline__ float quat_decode(uint8_t c) { return ((float)c - 127.5f) / 127.5f; }
#pragma clang fp contract(fast)

__device__ __forceinline__ uint8_t opacity_code(float logit, const OpacityThresholds &T) {
    // number of thresholds at or below the logit (thresholds ascending)
    int lo = 0, hi = 255;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (T.t[mid] <= logit) lo = mid + 1; else hi = mid;
    }
    return (uint8_t)lo;
}

__global__ void __launch_bounds__(kBlock)
k_encode(const float *__restrict__ P, uint32_t n, int enc, const uint32_t *__restrict__ kept,
         const uint32_t *__restrict__ pos, uint32_t m, uint8_t *__restrict__ out, Sections sec,
         OpacityThresholds T) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    if (kept && !kept[k]) return;
    const uint32_t o = pos ? pos[k] : k;
    float v[14];
#pragma unroll
    for (int r = 0; r < 14; ++r) v[r] = P[(size_t)r * n + k];
    float *dc = reinterpret_cast<float *>(out + sec.dc);
    for (int c = 0; c < 3; ++c) dc[(size_t)c * m + o] = v[11 + c];
    if (enc == kEncFp32) {
        float *mean = reinterpret_cast<float *>(out + sec.mean), *scale = reinterpret_cast<float *>(out + sec.scale);
        float *quat = reinterpret_cast<float *>(out + sec.quat), *opac = reinterpret_cast<float *>(out + sec.opac);
        for (int c = 0; c < 3; ++c) {
            mean[(size_t)c * m + o] = v[c];
            scale[(size_t)c * m + o] = v[3 + c];
        }
        for (int c = 0; c < 4; ++c) quat[(size_t)c * m + o] = v[6 + c];
        opac[o] = v[10];
    } else {
        uint16_t *mean = reinterpret_cast<uint16_t *>(out + sec.mean), *scale = reinterpret_cast<uint16_t *>(out + sec.scale);
        uint8_t *quat = out + sec.quat, *opac = out + sec.opac;
        for (int c = 0; c < 3; ++c) {
            mean[(size_t)c * m + o] = to_half_bits(v[c]);
            scale[(size_t)c * m + o] = to_half_bits(v[3 + c]);
        }
        uint8_t qc[4];
        quat_codes(v[6], v[7], v[8], v[9], qc);
        for (int c = 0; c < 4; ++c) quat[(size_t)c * m + o] = qc[c];
        opac[o] = opacity_code(v[10], T);
    }
}

__global__ void __launch_bounds__(kBlock)
k_mask_popc(const uint32_t *__restrict__ mask, uint32_t words, uint32_t *__restrict__ cnt) {
    const uint32_t w = blockIdx.x * kBlock + threadIdx.x;
    if (w < words) cnt[w] = (uint32_t)__popc(mask[w]);
}

struct V2Head {
    uint32_t n, m;
    int enc, flags;
    int32_t slot0, birth0, start0, expire0;
};

__global__ void __launch_bounds__(kBlock)
k_decode(const uint8_t *__restrict__ rec, V2Head h, Sections sec, const uint32_t *__restrict__ word_rank,
         int64_t slot_base, float *__restrict__ params, int n_slots, int F, int32_t *__restrict__ birth,
         int32_t *__restrict__ start, int32_t *__restrict__ expire, OpacityDecode D, uint32_t *__restrict__ bad) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= h.n) return;
    int64_t slot;
    int32_t b, s, e;
    if (h.flags & kFlagLifespans) {
        const uint32_t *sl = reinterpret_cast<const uint32_t *>(rec + sec.life);
        const size_t stride = align16(4 * (size_t)h.n) / 4;
        slot = sl[k];
        b = (int32_t)sl[stride + k];
        s = (int32_t)sl[2 * stride + k];
        e = (int32_t)sl[3 * stride + k];
    } else {
        slot = (int64_t)h.slot0 + k;
        b = h.birth0;
        s = h.start0;
        e = h.expire0;
    }
    if (slot_base >= 0) slot = slot_base + (int64_t)k;
    if (slot < 0 || slot >= n_slots) {
        atomicAdd(bad, 1u);
        return;
    }
    uint32_t o = k;
    if (h.flags & kFlagMask) {
        const uint32_t *mask = reinterpret_cast<const uint32_t *>(rec + sec.mask);
        const uint32_t w = mask[k >> 5], bit = 1u << (k & 31);
        if (!(w & bit)) {
            // dropped by the tail-drop: an empty lifespan, never drawn
            if (birth) birth[slot] = b;
            start[slot] = b;
            expire[slot] = b;
            return;
        }
        o = word_rank[k >> 5] + (uint32_t)__popc(w & (bit - 1u));
    }
    const size_t S = (size_t)n_slots, m = h.m;
    float v[14];
    const float *dc = reinterpret_cast<const float *>(rec + sec.dc);
    for (int c = 0; c < 3; ++c) v[11 + c] = dc[c * m + o];
    if (h.enc == kEncFp32) {
        const float *mean = reinterpret_cast<const float *>(rec + sec.mean);
        const float *scale = reinterpret_cast<const float *>(rec + sec.scale);
        const float *quat = reinterpret_cast<const float *>(rec + sec.quat);
        for (int c = 0; c < 3; ++c) {
            v[c] = mean[c * m + o];
            v[3 + c] = scale[c * m + o];
        }
        for (int c = 0; c < 4; ++c) v[6 + c] = quat[c * m + o];
        v[10] = reinterpret_cast<const float *>(rec + sec.opac)[o];
    } else {
        const _Float16 *mean = reinterpret_cast<const _Float16 *>(rec + sec.mean);
        const _Float16 *scale = reinterpret_cast<const _Float16 *>(rec + sec.scale);
        for (int c = 0; c < 3; ++c) {
            v[c] = (float)mean[c * m + o];
            v[3 + c] = (float)scale[c * m + o];
        }
        for (int c = 0; c < 4; ++c) v[6 + c] = quat_decode(rec[sec.quat + c * m + o]);
        v[10] = D.v[rec[sec.opac + o]];
    }
    for (int r = 0; r < 14; ++r) params[(size_t)r * S + (size_t)slot] = v[r];
    for (int r = 14; r < F; ++r) params[(size_t)r * S + (size_t)slot] = 0.0f;   // higher SH bands not streamed
    if (birth) birth[slot] = b;
    start[slot] = s;
    expire[slot] = e;
}

OpacityThresholds opacity_thresholds() {
    OpacityThresholds T;
    for (int k = 1; k <= 255; ++k) {
        const double p = (k - 0.5) / 255.0;
        T.t[k - 1] = (float)std::log(p / (1.0 - p));
    }
    return T;
}

OpacityDecode opacity_decode() {
    OpacityDecode D;
    for (int c = 0; c < 256; ++c) {
        double p = c / 255.0;
        p = p < 1.0 / 510.0 ? 1.0 / 510.0 : (p > 1.0 - 1.0 / 510.0 ? 1.0 - 1.0 / 510.0 : p);
        D.v[c] = (float)std::log(p / (1.0 - p));
    }
    return D;
}

inline int grid_of(size_t n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

size_t encoded_bytes(uint32_t n, uint32_t m, int enc, bool uniform, bool masked) {
    return sections(n, m, enc, uniform, masked).total;
}

// Encode: src (v1, n entries, F rows) -> out (v2).  scratch holds at least
// encode_scratch_words(n) words.  `uniform` comes from encode_uniform().
size_t encode_scratch_words(uint32_t n) {
    return 8 + 6 * ((size_t)n + 8) + (size_t)256 * kSortBlocks + 512 + (size_t)n / 4096 + 16;
}

void launch_encode_uniform(hipStream_t s, const uint8_t *src, uint32_t n, uint32_t *flag) {
    launch_fill_u32(s, flag, 0, 1);
    if (!n) return;
    const V1 v = v1_view(src, n);
    hipLaunchKernelGGL(k_enc_uniform, dim3(grid_of(n)), dim3(kBlock), 0, s, v.slot, v.birth, v.start, v.expire, n,
                       flag);
}

void launch_encode(hipStream_t s, const uint8_t *src, uint32_t n, int F, int enc, uint32_t keep, bool uniform,
                   const int32_t header[16], uint8_t *out, uint32_t *scratch) {
    const bool masked = keep < n;
    const uint32_t m = masked ? keep : n;
    const Sections sec = sections(n, m, enc, uniform, masked);
    (void)F;
    // padding between the 16-byte aligned arrays is zero: the record is
    // fully determined by its contents
    launch_fill_u32(s, reinterpret_cast<uint32_t *>(out), 0, sec.total / 4);
    (void)hipMemcpyAsync(out, header, 64, hipMemcpyHostToDevice, s);
    const V1 v = v1_view(src, n);
    if (!uniform && n) {
        const size_t a = align16(4 * (size_t)n);
        (void)hipMemcpyAsync(out + sec.life, v.slot, 4 * (size_t)n, hipMemcpyDeviceToDevice, s);
        (void)hipMemcpyAsync(out + sec.life + a, v.birth, 4 * (size_t)n, hipMemcpyDeviceToDevice, s);
        (void)hipMemcpyAsync(out + sec.life + 2 * a, v.start, 4 * (size_t)n, hipMemcpyDeviceToDevice, s);
        (void)hipMemcpyAsync(out + sec.life + 3 * a, v.expire, 4 * (size_t)n, hipMemcpyDeviceToDevice, s);
    }
    uint32_t *kept = nullptr, *pos = nullptr;
    if (masked) {
        // scratch: keys, vals, alt keys, alt vals, kept flags, positions, histogram, totals, scan partials
        const size_t nn = (size_t)n + 8;
        uint32_t *key = scratch, *val = key + nn, *key_alt = val + nn, *val_alt = key_alt + nn;
        kept = val_alt + nn;
        pos = kept + nn;
        uint32_t *hist = pos + nn, *totals = hist + (size_t)256 * kSortBlocks, *part = totals + 512;
        const uint32_t words = (n + 31) / 32;
        uint32_t *mask = reinterpret_cast<uint32_t *>(out + sec.mask);
        launch_fill_u32(s, mask, 0, words);
        launch_fill_u32(s, kept, 0, n);
        hipLaunchKernelGGL(k_enc_keys, dim3(grid_of(n)), dim3(kBlock), 0, s, v.params + (size_t)10 * n, n, key, val);
        radix_sort_pairs(s, key, val, key_alt, val_alt, nullptr, n, n, 32, hist, totals);
        if (keep) hipLaunchKernelGGL(k_enc_mark, dim3(grid_of(keep)), dim3(kBlock), 0, s, val, keep, mask, kept);
        exclusive_scan_u32(s, kept, pos, n, part + (size_t)n / 4096 + 8, part);
    }
    if (m)
        hipLaunchKernelGGL(k_encode, dim3(grid_of(n)), dim3(kBlock), 0, s, v.params, n, enc, kept, pos, m, out, sec,
                           opacity_thresholds());
}

bool decode_layout(const int32_t h[16], size_t *need) {
    const uint32_t n = (uint32_t)h[3], m = (uint32_t)h[4];
    *need = sections(n, m, h[5], !(h[7] & kFlagLifespans), (h[7] & kFlagMask) != 0).total;
    return true;
}

void launch_decode(hipStream_t s, const swgs_pool &pool, int F, const uint8_t *rec, const int32_t h[16],
                   int64_t slot_base, uint32_t *scratch, uint32_t *bad) {
    V2Head hd;
    hd.n = (uint32_t)h[3];
    hd.m = (uint32_t)h[4];
    hd.enc = h[5];
    hd.flags = h[7];
    hd.slot0 = h[8];
    hd.birth0 = h[9];
    hd.start0 = h[10];
    hd.expire0 = h[11];
    if (!hd.n) return;
    const Sections sec = sections(hd.n, hd.m, hd.enc, !(hd.flags & kFlagLifespans), (hd.flags & kFlagMask) != 0);
    uint32_t *rank = nullptr;
    if (hd.flags & kFlagMask) {
        const uint32_t words = (hd.n + 31) / 32;
        rank = scratch;
        uint32_t *part = rank + words + 8;
        hipLaunchKernelGGL(k_mask_popc, dim3(grid_of(words)), dim3(kBlock), 0, s,
                           reinterpret_cast<const uint32_t *>(rec + sec.mask), words, rank);
        exclusive_scan_u32(s, rank, rank, words, part + words / 4096 + 8, part);
    }
    hipLaunchKernelGGL(k_decode, dim3(grid_of(hd.n)), dim3(kBlock), 0, s, rec, hd, sec, rank, slot_base,
                       pool.params, pool.n_slots, F, pool.birth, pool.start, pool.expire, opacity_decode(), bad);
}

}  // namespace swgs

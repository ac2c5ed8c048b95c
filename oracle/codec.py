"""Oracle of the compact per-frame update record (test infrastructure only:
tests, the smoke check and the benchmark's CPU baseline use it; the product
path never does).

What is streamed per frame follows Sec. 5.2 (Eq. 4: bytes per Gaussian times
the slice size), Sec. 5.6.2 and Table 6: a Gaussian is sent as its mean,
scale, rotation, opacity and the DC term of its spherical harmonics only (the
higher SH bands are not streamed), either in FP32 (14 floats, 56 bytes) or at
Table 6's precisions -- FP16 means and scales, 8-bit rotation and opacity,
the SH DC kept in FP32 -- 29 bytes.  Sec. 5.5's bandwidth adaptation keeps a
slice's highest-opacity Gaussians and marks the rest as empty padding.

Readings where the paper is silent (each side of the codec implements them
from these definitions; nothing is shared with the GPU code):
  * FP16: IEEE binary16, round to nearest even, finite values saturated to
    +-65504 first.  The scale attribute is the stored log-scale.
  * 8-bit rotation: each component of the unit quaternion q/|q| mapped from
    [-1, 1] to round(c 127.5 + 127.5), round half to even; FP32 arithmetic
    with |q|^2 = ((q0^2 + q1^2) + q2^2) + q3^2, a correctly rounded square
    root and division, then a product and a sum, each rounded; the zero
    quaternion is sent as the identity.  Decoded c = (code - 127.5) / 127.5
    (the renderer normalises).
  * 8-bit opacity: code = round(sigma 255) for sigma = sigmoid(logit),
    decided on the logit: code = the number of thresholds
    L_k = fl32(logit((k - 1/2) / 255)), k = 1..255, at or below the FP32
    logit.  Decoded logit = fl32(logit(p)) with p = code / 255 kept inside
    [1/510, 1 - 1/510] so that it is finite.
  * Tail-drop: keep the `keep` entries of largest opacity logit, ties to the
    lower entry index; a dropped entry's slot gets the empty lifespan
    [birth, birth) on the client and is never drawn.

Record, version 2 (little endian): int32 header[16] = {magic 'SWGS',
2, st, n (entries of the source record), n_kept, enc (1 = FP32, 2 = Table 6),
swin, flags (1: per-entry slots and lifespans present, 2: keep mask
present), slot0, birth0, start0, expire0, source SH degree, 0, 0, 0};
then, each array starting at a 16-byte boundary: [flags & 1] uint32
slot[n], int32 birth[n], start[n], expire[n]; [flags & 2] uint32
mask[ceil(n / 32)] (bit k & 31 of word k >> 5 = entry k kept); the kept
entries' attributes, planar: mean[3][m], scale[3][m], quat[4][m],
opacity[m], dc[3][m] (FP32, or FP16 / FP16 / uint8 / uint8 / FP32).  Without
flag 1 every entry shares (birth0, start0, expire0) and entry k is slot
slot0 + k.
"""
import math

import numpy as np

MAGIC = 0x53475753
ENC_FP32, ENC_Q = 1, 2
F_LIFESPANS, F_MASK = 1, 2
HALF_MAX = 65504.0


def _align16(n: int) -> int:
    return (n + 15) // 16 * 16


def opacity_thresholds():
    """L_k = fl32(logit((k - 1/2) / 255)), k = 1..255 (FP64, then rounded)."""
    out = np.empty(255, np.float32)
    for k in range(1, 256):
        p = (k - 0.5) / 255.0
        out[k - 1] = np.float32(math.log(p / (1.0 - p)))
    return out


def opacity_decode_table():
    """Decoded logit of each opacity code."""
    out = np.empty(256, np.float32)
    for c in range(256):
        p = min(max(c / 255.0, 1.0 / 510.0), 1.0 - 1.0 / 510.0)
        out[c] = np.float32(math.log(p / (1.0 - p)))
    return out


def to_half(x):
    x = np.asarray(x, np.float32)
    return np.clip(x, np.float32(-HALF_MAX), np.float32(HALF_MAX)).astype(np.float16)


def quat_codes(q):
    """q: float32 [4][m] -> uint8 codes [4][m]."""
    q = np.asarray(q, np.float32)
    n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]
    zero = n2 == np.float32(0.0)
    n = np.sqrt(np.where(zero, np.float32(1.0), n2))
    c = q / n
    c[:, zero] = np.array([1.0, 0.0, 0.0, 0.0], np.float32)[:, None]
    t = c * np.float32(127.5)
    t = t + np.float32(127.5)
    return np.clip(np.rint(t), 0, 255).astype(np.uint8)


def quat_decode(codes):
    return (codes.astype(np.float32) - np.float32(127.5)) / np.float32(127.5)


def opacity_codes(logit):
    L = opacity_thresholds()
    return np.searchsorted(L, np.asarray(logit, np.float32), side="right").astype(np.uint8)


def keep_mask(logit, keep):
    """Entries kept by the tail-drop (bool [n])."""
    n = len(logit)
    if keep < 0 or keep >= n:
        return np.ones(n, bool)
    order = sorted(range(n), key=lambda k: (-float(logit[k]), k))
    m = np.zeros(n, bool)
    m[order[:keep]] = True
    return m


def encode(rec, st: int, swin: int, sh_degree: int, enc: int, keep: int = -1) -> bytes:
    """rec: dict(slots, birth, start, expire, params [F][n]) as swgs_mature
    emits it (oracle.mature's return value)."""
    slots = np.asarray(rec["slots"], np.int64)
    birth, start, expire = (np.asarray(rec[k], np.int32) for k in ("birth", "start", "expire"))
    P = np.asarray(rec["params"], np.float32)
    n = len(slots)
    uniform = n == 0 or (np.all(birth == birth[0]) and np.all(start == start[0]) and
                         np.all(expire == expire[0]) and np.all(slots == slots[0] + np.arange(n)))
    kept = keep_mask(P[10], keep)
    m = int(kept.sum())
    flags = (0 if uniform else F_LIFESPANS) | (0 if m == n else F_MASK)
    h = np.zeros(16, np.int32)
    h[:8] = [MAGIC, 2, st, n, m, enc, swin, flags]
    if n and uniform:
        h[8:12] = [slots[0], birth[0], start[0], expire[0]]
    h[12] = sh_degree
    parts = [h.tobytes()]

    def put(arr):
        b = np.ascontiguousarray(arr).tobytes()
        parts.append(b + bytes(_align16(len(b)) - len(b)))

    if flags & F_LIFESPANS:
        put(slots.astype(np.uint32))
        put(birth)
        put(start)
        put(expire)
    if flags & F_MASK:
        words = np.zeros((n + 31) // 32, np.uint32)
        for k in np.nonzero(kept)[0]:
            words[k >> 5] |= np.uint32(1 << (k & 31))
        put(words)
    K = P[:, kept]
    if enc == ENC_FP32:
        for a in (K[0:3], K[3:6], K[6:10], K[10:11], K[11:14]):
            put(a.astype(np.float32))
    elif enc == ENC_Q:
        put(to_half(K[0:3]))
        put(to_half(K[3:6]))
        put(quat_codes(K[6:10]))
        put(opacity_codes(K[10]))
        put(K[11:14].astype(np.float32))
    else:
        raise ValueError("unknown encoding")
    return b"".join(parts)


def encoded_bytes(n: int, m: int, enc: int, uniform: bool, masked: bool) -> int:
    per = [12, 12, 16, 4, 12] if enc == ENC_FP32 else [6, 6, 4, 1, 12]
    size = 64
    if not uniform:
        size += 4 * _align16(4 * n)
    if masked:
        size += _align16(4 * ((n + 31) // 32))
    return size + sum(_align16(b * m) for b in per)


def decode(buf: bytes, F: int):
    """-> dict(slots, birth, start, expire, kept, params [F][n]) for all n
    entries of the record (dropped entries: lifespan [birth, birth), params
    NaN as 'not written')."""
    h = np.frombuffer(buf[:64], np.int32)
    assert h[0] == MAGIC and h[1] == 2
    n, m, enc, flags = int(h[3]), int(h[4]), int(h[5]), int(h[7])
    off = 64

    def take(dtype, count):
        nonlocal off
        a = np.frombuffer(buf, dtype, count, off)
        off += _align16(a.nbytes)
        return a

    if flags & F_LIFESPANS:
        slots = take(np.uint32, n).astype(np.int64)
        birth, start, expire = take(np.int32, n), take(np.int32, n), take(np.int32, n)
    else:
        slots = int(h[8]) + np.arange(n, dtype=np.int64)
        birth, start, expire = (np.full(n, h[i], np.int32) for i in (9, 10, 11))
    if flags & F_MASK:
        words = take(np.uint32, (n + 31) // 32)
        kept = np.array([(words[k >> 5] >> np.uint32(k & 31)) & 1 for k in range(n)], bool)
    else:
        kept = np.ones(n, bool)
    K = np.zeros((F, m), np.float32)
    if enc == ENC_FP32:
        K[0:3] = take(np.float32, 3 * m).reshape(3, m)
        K[3:6] = take(np.float32, 3 * m).reshape(3, m)
        K[6:10] = take(np.float32, 4 * m).reshape(4, m)
        K[10] = take(np.float32, m)
        K[11:14] = take(np.float32, 3 * m).reshape(3, m)
    else:
        K[0:3] = take(np.float16, 3 * m).reshape(3, m).astype(np.float32)
        K[3:6] = take(np.float16, 3 * m).reshape(3, m).astype(np.float32)
        K[6:10] = quat_decode(take(np.uint8, 4 * m).reshape(4, m))
        K[10] = opacity_decode_table()[take(np.uint8, m)]
        K[11:14] = take(np.float32, 3 * m).reshape(3, m)
    params = np.full((F, n), np.nan, np.float32)
    params[:, kept] = K
    start = np.where(kept, start, birth).astype(np.int32)
    expire = np.where(kept, expire, birth).astype(np.int32)
    return dict(slots=slots, birth=np.array(birth), start=start, expire=expire, kept=kept, params=params,
                st=int(h[2]), enc=enc, flags=flags, n=n, m=m)

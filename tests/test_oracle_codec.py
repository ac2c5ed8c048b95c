"""Pins of the oracle's compact update record (Eq. 4 sizes, Table 6
precisions, DC-only SH of Sec. 5.6.2, Sec. 5.5's tail-drop).  CPU only."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import codec as C


def slice_record(n, F=59, seed=0, uniform=True):
    rng = np.random.default_rng(seed)
    P = rng.normal(size=(F, n)).astype(np.float32)
    P[0:3] *= 3.0
    P[3:6] = rng.uniform(-5, -1, size=(3, n))
    slots = np.arange(40, 40 + n)
    b = np.full(n, 7, np.int32)
    rec = dict(slots=slots, birth=b, start=b.copy(), expire=b + 5, params=P)
    if not uniform:
        rec["expire"] = b + 1 + (np.arange(n) % 5).astype(np.int32)
    return rec


def test_sizes_match_eq4_and_the_paper_figures():
    """56 bytes per Gaussian (mean, scale, quaternion, opacity, SH DC in FP32)
    and 29 at Table 6's precisions; 40K Gaussians per frame (200K, swin 5)
    give 2.24e6 bytes = 2.14 MiB ("2.1MB") and 1.16e6 bytes ("1.2MB")."""
    n = 40_000
    rec = slice_record(n)
    full = C.encode(rec, 7, 5, 3, C.ENC_FP32)
    q = C.encode(rec, 7, 5, 3, C.ENC_Q)
    assert len(full) == 64 + 56 * n and len(q) == 64 + 29 * n
    assert round((len(full) - 64) / 2 ** 20, 1) == 2.1 and round((len(q) - 64) / 1e6, 1) == 1.2
    assert len(full) == C.encoded_bytes(n, n, C.ENC_FP32, True, False)
    assert len(q) == C.encoded_bytes(n, n, C.ENC_Q, True, False)
    # Eq. 4 at 30 fps: bandwidth = fps x slice size x bytes per Gaussian
    assert 30 * n * 29 * 8 / 1e6 == pytest.approx(278.4)


def test_half_precision_rounds_to_nearest_even_and_saturates():
    x = np.array([0.5, -3.25, 2048.0, 1 + 2 ** -11, 1 + 3 * 2 ** -11, 65504.0, 7e4, -1e9, 2 ** -24, 2 ** -26],
                 np.float32)
    h = C.to_half(x).astype(np.float64)
    want = [0.5, -3.25, 2048.0, 1.0, 1 + 2 ** -9, 65504.0, 65504.0, -65504.0, 2 ** -24, 0.0]
    assert h.tolist() == want


def test_quaternion_codes_by_hand():
    q = np.array([[1, 0, 0, 0], [-1, 0, 0, 0], [2, 0, 0, 0], [0.5, 0.5, 0.5, 0.5], [0, 0, 0, 0],
                  [0, 0, 0, -3]], np.float32).T
    codes = C.quat_codes(q).T.tolist()
    # 1 -> 255, 0 -> 127.5 -> 128 (half to even), -1 -> 0, 0.5 -> 191.25 -> 191
    assert codes == [[255, 128, 128, 128], [0, 128, 128, 128], [255, 128, 128, 128], [191, 191, 191, 191],
                     [255, 128, 128, 128], [128, 128, 128, 0]]
    rng = np.random.default_rng(1)
    r = rng.normal(size=(4, 20000)).astype(np.float32)
    u = r / np.linalg.norm(r.astype(np.float64), axis=0)
    err = np.abs(C.quat_decode(C.quat_codes(r)) - u)
    assert err.max() <= 1 / 255 + 1e-6


def test_opacity_codes_are_rounded_sigmoid():
    rng = np.random.default_rng(2)
    z = rng.uniform(-9, 9, 100000).astype(np.float32)
    s = 1 / (1 + np.exp(-z.astype(np.float64)))
    t = s * 255
    away = np.abs(t - np.floor(t) - 0.5) > 1e-4
    assert np.array_equal(C.opacity_codes(z)[away], np.floor(t[away] + 0.5).astype(np.uint8))
    assert C.opacity_codes(np.float32([0.0, -40.0, 40.0])).tolist() == [128, 0, 255]
    D = C.opacity_decode_table()
    assert D[0] == np.float32(math.log((1 / 510) / (1 - 1 / 510))) and D[255] == -D[0]
    sig = 1 / (1 + np.exp(-D.astype(np.float64)))
    assert np.allclose(sig[1:255], np.arange(1, 255) / 255, atol=1e-6)
    dec = 1 / (1 + np.exp(-D[C.opacity_codes(z)].astype(np.float64)))
    assert np.abs(dec - s).max() <= 1 / 510 + 1e-6


def test_tail_drop_keeps_the_most_opaque_ties_to_lower_index():
    logit = np.float32([0.5, 2.0, 0.5, -1.0, 2.0, 0.5])
    assert C.keep_mask(logit, 3).tolist() == [True, True, False, False, True, False]
    assert C.keep_mask(logit, 4).tolist() == [True, True, True, False, True, False]
    assert C.keep_mask(logit, 0).sum() == 0 and C.keep_mask(logit, 6).all() and C.keep_mask(logit, -1).all()


@pytest.mark.parametrize("enc", [C.ENC_FP32, C.ENC_Q])
@pytest.mark.parametrize("uniform", [True, False])
def test_round_trip(enc, uniform):
    n, F = 300, 59
    rec = slice_record(n, F, seed=3, uniform=uniform)
    buf = C.encode(rec, 9, 5, 3, enc, keep=200)
    d = C.decode(buf, F)
    assert d["n"] == n and d["m"] == 200 and d["flags"] == (0 if uniform else C.F_LIFESPANS) | C.F_MASK
    assert len(buf) == C.encoded_bytes(n, 200, enc, uniform, True)
    k = d["kept"]
    assert np.array_equal(k, C.keep_mask(rec["params"][10], 200))
    assert np.array_equal(d["slots"], rec["slots"]) and np.array_equal(d["birth"], rec["birth"])
    assert np.array_equal(d["start"][k], rec["start"][k]) and np.array_equal(d["expire"][k], rec["expire"][k])
    assert np.all(d["start"][~k] == d["birth"][~k]) and np.all(d["expire"][~k] == d["birth"][~k])
    P, Q = rec["params"][:, k], d["params"][:, k]
    assert np.all(Q[14:] == 0)                               # higher SH bands are not streamed
    assert np.array_equal(Q[11:14], P[11:14])                # DC in full precision
    if enc == C.ENC_FP32:
        assert np.array_equal(Q[:11], P[:11])
    else:
        assert np.all(np.abs(Q[0:6] - P[0:6]) <= np.abs(P[0:6]) * 2 ** -11 + 2 ** -24)
        u = P[6:10] / np.linalg.norm(P[6:10], axis=0)
        assert np.abs(Q[6:10] - u).max() <= 1 / 255 + 1e-6
        so = 1 / (1 + np.exp(-P[10].astype(np.float64)))
        sq = 1 / (1 + np.exp(-Q[10].astype(np.float64)))
        assert np.abs(sq - so).max() <= 1 / 510 + 1e-6


def test_schedule_records_after_genesis_are_uniform_slices():
    """Algorithm 1's records: the first (the genesis window) has per-slot
    expiries; every later one is one slice -- contiguous slots, one lifespan
    -- so it needs no per-entry slots or lifespans."""
    num_gs, swin, F = 50, 5, 14
    params = np.random.default_rng(4).normal(size=(F, 2 * num_gs)).astype(np.float32)
    birth, start, expire = O.genesis(num_gs, swin)
    O.schedule_expire(num_gs, swin, expire)
    for st in range(1, 9):
        rec = O.mature(st, num_gs, swin, params, birth, start, expire)
        d = C.decode(C.encode(rec, st, swin, 0, C.ENC_Q), F)
        assert (d["flags"] & C.F_LIFESPANS) == (C.F_LIFESPANS if st == 1 else 0), st
        assert np.array_equal(d["slots"], rec["slots"])
        if st > 1:
            assert len(rec["slots"]) == num_gs // swin

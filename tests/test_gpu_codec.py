"""GPU parity of the compact per-frame update record (encode after mature,
decode in apply_update) against the oracle's codec: the encoded bytes are
compared bit for bit, and so are the decoded client parameters and
lifespans.  Records come from Algorithm 1's schedule (the genesis window's
record with per-slot expiries, then one slice per frame), with and without
the tail-drop, at SH degree 3, and at the paper's slice size (40K)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from oracle import codec as C
from paper_2409_07759_amd import synth as S

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def sw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_07759_amd import swgs
    return swgs


@pytest.fixture(scope="module")
def ctx(sw):
    c = sw.Context(0)
    yield c
    c.close()


def genesis_pool(num_gs, swin, deg, seed):
    F = 11 + 3 * (deg + 1) ** 2
    rng = np.random.default_rng(seed)
    P = rng.normal(size=(F, 2 * num_gs)).astype(np.float32)
    P[0:3] *= 2.0
    P[3:6] = rng.uniform(-5, -1, size=(3, 2 * num_gs)).astype(np.float32)
    P[10] = rng.uniform(-6, 6, size=2 * num_gs).astype(np.float32)
    P[6:10, :7] = 0.0                                    # zero quaternions are sent as the identity
    P[0, 7] = 7e4                                        # FP16 saturation
    b, s, e = O.genesis(num_gs, swin)
    O.schedule_expire(num_gs, swin, e)
    return P, b, s, e


def client(sw, num_gs, deg, fill=5.0):
    F = 11 + 3 * (deg + 1) ** 2
    return sw.Pool(np.full((F, num_gs), fill, np.float32), np.full(num_gs, -9, np.int32),
                   np.full(num_gs, -9, np.int32), np.full(num_gs, -9, np.int32), 0, 5, deg, "cuda", train=False)


def check_decoded(sw, ctx, rec_gpu, buf, cl, F_client):
    """apply_update of the encoded record == the oracle's decode."""
    before = host(cl.params).copy()
    n = sw.apply_update(ctx, cl, rec_gpu)
    d = C.decode(buf, F_client)
    assert n == d["n"]
    P = host(cl.params)
    sl = d["slots"]
    k = d["kept"]
    assert np.array_equal(P[:, sl[k]], d["params"][:, k])
    assert np.array_equal(P[:, sl[~k]], before[:, sl[~k]])   # dropped: parameters untouched
    for name in ("birth", "start", "expire"):
        assert np.array_equal(host(getattr(cl, name))[sl], d[name]), name


@pytest.mark.parametrize("enc", [1, 2])
def test_schedule_records_encode_and_decode_bit_exact(sw, ctx, enc):
    num_gs, swin, deg = 3000, 5, 3
    P, b, s, e = genesis_pool(num_gs, swin, deg, 1)
    dp = sw.Pool(P.copy(), b.copy(), s.copy(), e.copy(), num_gs, swin, deg, "cuda")
    F = P.shape[0]
    for st in (1, 2, 3, 4):
        rec, cnt = sw.mature(ctx, dp, st)
        ref = O.mature(st, num_gs, swin, P, b, s, e)
        for keep in (-1, cnt // 3, 0, cnt):
            say("st", st, "enc", enc, "keep", keep, "entries", cnt)
            out = sw.encode_update(ctx, rec, enc, keep)
            want = C.encode(ref, st, swin, deg, enc, keep)
            got = host(out).tobytes()
            assert len(got) == len(want), (len(got), len(want))
            assert got == want
            for cdeg in (3, 0):
                check_decoded(sw, ctx, out, want, client(sw, num_gs, cdeg), 11 + 3 * (cdeg + 1) ** 2)
        if st == 1:
            assert C.decode(want, F)["flags"] & C.F_LIFESPANS
        else:
            assert cnt == num_gs // swin and not (C.decode(want, F)["flags"] & C.F_LIFESPANS)


def test_paper_slice_size_bytes_and_bits(sw, ctx):
    """200K Gaussians, swin 5: a 40K slice is 2.24 MB in FP32 and 1.16 MB at
    Table 6's precisions (the paper's 2.1 MB and 1.2 MB per frame)."""
    num_gs, swin, deg = 200_000, 5, 3
    pool = S.steady_window_pool(num_gs, swin, deg, 7, 3)
    dp = sw.Pool.from_synth(pool)
    P, b, s, e = pool.params.copy(), pool.birth.copy(), pool.start.copy(), pool.expire.copy()
    rec, cnt = sw.mature(ctx, dp, 8)
    ref = O.mature(8, num_gs, swin, P, b, s, e)
    assert cnt == 40_000
    sizes = {}
    for enc in (1, 2):
        out = sw.encode_update(ctx, rec, enc)
        want = C.encode(ref, 8, swin, deg, enc)
        assert host(out).tobytes() == want
        sizes[enc] = out.numel()
        check_decoded(sw, ctx, out, want, client(sw, num_gs, deg), P.shape[0])
    say("bytes per frame", sizes, "full record", rec.numel())
    assert sizes[1] == 64 + 56 * 40_000 and sizes[2] == 64 + 29 * 40_000
    assert rec.numel() > 4 * sizes[1]


def test_codec_rejects_bad_input(sw, ctx):
    num_gs, swin, deg = 100, 5, 1
    P, b, s, e = genesis_pool(num_gs, swin, deg, 2)
    dp = sw.Pool(P.copy(), b.copy(), s.copy(), e.copy(), num_gs, swin, deg, "cuda")
    rec, cnt = sw.mature(ctx, dp, 1)
    with pytest.raises(sw.SwgsError):
        sw.encode_update(ctx, rec, 3)
    out = sw.encode_update(ctx, rec, 2, keep=10)
    with pytest.raises(sw.SwgsError):
        sw.encode_update(ctx, rec[:40], 2)                    # shorter than its entries
    bad = out.clone()
    bad[28:32] = torch.tensor([4, 0, 0, 0], dtype=torch.uint8, device="cuda")   # unknown flag bit
    with pytest.raises(sw.SwgsError):
        sw.apply_update(ctx, client(sw, num_gs, deg), bad)
    with pytest.raises(sw.SwgsError):
        sw.apply_update(ctx, client(sw, num_gs, deg), out[:100])
    # an empty record (nothing matures before frame 0) round-trips as a no-op
    rec0, cnt0 = sw.mature(ctx, dp, 0)
    assert cnt0 == 0
    out0 = sw.encode_update(ctx, rec0, 2)
    assert out0.numel() == C.encoded_bytes(0, 0, 2, True, False)
    assert sw.apply_update(ctx, client(sw, num_gs, deg), out0) == 0

"""Client playback (Algorithm 2) on the GPU: the player's buffer after every
frame equals the oracle's replay of the same update stream (bit for bit),
and renders issued right after advance(), with no host synchronisation,
see the new slices.  Streams: Table 6 records with and without the
tail-drop, and full version-1 records."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from oracle import codec as C
from paper_2409_07759_amd import synth as S

pytestmark = pytest.mark.gpu

NUM_GS, SWIN, DEG = 2000, 5, 3
F = 11 + 3 * (DEG + 1) ** 2


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


def trainer_stream(sw, ctx, n_frames, enc, keep_frac):
    """Algorithm 1's records for frames 1..n_frames from a genesis pool:
    (device-encoded host bytes, oracle record) per frame."""
    rng = np.random.default_rng(3)
    P = S.make_gaussians(2 * NUM_GS, DEG, 4).astype(np.float32)
    b, s, e = O.genesis(NUM_GS, SWIN)
    O.schedule_expire(NUM_GS, SWIN, e)
    dp = sw.Pool(P.copy(), b.copy(), s.copy(), e.copy(), NUM_GS, SWIN, DEG, "cuda")
    out = []
    for st in range(1, n_frames + 1):
        rec, cnt = sw.mature(ctx, dp, st)
        ref = O.mature(st, NUM_GS, SWIN, P, b, s, e)
        keep = -1 if keep_frac is None else int(cnt * keep_frac)
        if enc is None:
            data = host(rec).tobytes()
        else:
            data = host(sw.encode_update(ctx, rec, enc, keep)).tobytes()
            assert data == C.encode(ref, st, SWIN, DEG, enc, keep)
        out.append((data, ref, keep))
        # the window trains between frames: move the optimisable slots
        dp.params[:, :NUM_GS] += 0.01
        P[:, :NUM_GS] += np.float32(0.01)
        assert np.array_equal(host(dp.params), P)
    return out


def replay(buf, record, enc, keep):
    """Algorithm 2's buffer update by the oracle (decode + scatter)."""
    if enc is None:
        d = dict(slots=record["slots"], birth=record["birth"], start=record["start"], expire=record["expire"],
                 kept=np.ones(len(record["slots"]), bool), params=record["params"].astype(np.float32))
    else:
        d = C.decode(C.encode(record, 0, SWIN, DEG, enc, keep), F)
    sl = d["slots"]
    k = d["kept"]
    buf["params"][:, sl[k]] = d["params"][:, k]
    for name in ("birth", "start", "expire"):
        buf[name][sl] = d[name]


def target(record):
    return int(record["birth"][0])


@pytest.mark.parametrize("enc,keep_frac", [(2, None), (2, 0.6), (None, None)])
def test_player_replays_the_stream(sw, ctx, enc, keep_frac):
    stream = trainer_stream(sw, ctx, 10, enc, keep_frac)
    view = S.ring_views([0], 1, 96, 72)[0]
    buf_pool = sw.Pool(np.zeros((F, NUM_GS), np.float32), np.full(NUM_GS, -1, np.int32),
                       np.full(NUM_GS, -1, np.int32), np.full(NUM_GS, -1, np.int32), 0, SWIN, DEG, "cuda",
                       train=False)
    ref = dict(params=np.zeros((F, NUM_GS), np.float32), birth=np.full(NUM_GS, -1, np.int32),
               start=np.full(NUM_GS, -1, np.int32), expire=np.full(NUM_GS, -1, np.int32))
    player = sw.Player(ctx, buf_pool, queue_depth=3, max_record_bytes=max(len(d) for d, _, _ in stream))
    next_push, applied = 0, set()
    for frame in range(0, 9):
        # the stream runs ahead of playback by up to the queue depth
        while next_push < len(stream) and player.queued()[0] < 3:
            player.push(stream[next_push][0])
            next_push += 1
        n = player.advance(frame)
        due = [i for i in range(next_push) if target(stream[i][1]) <= frame and i not in applied]
        for i in due:
            replay(ref, stream[i][1], enc, stream[i][2])
            applied.add(i)
        assert n == len(due), (frame, n, len(due))
        # render on the context stream right after advance (no sync in between)
        vf = S.ring_views([frame], 1, 96, 72)[0]
        pl = sw.Plan(ctx, buf_pool, [vf])
        img = host(pl.forward()).copy()
        pl.close()
        say("frame", frame, "applied", n, "live", int(((ref["start"] <= frame) & (frame < ref["expire"])).sum()))
        assert np.array_equal(host(buf_pool.params), ref["params"]), frame
        for name in ("birth", "start", "expire"):
            assert np.array_equal(host(getattr(buf_pool, name)), ref[name]), (frame, name)
        rp = sw.Pool(ref["params"], ref["birth"], ref["start"], ref["expire"], 0, SWIN, DEG, "cuda", train=False)
        pl2 = sw.Plan(ctx, rp, [vf])
        assert np.array_equal(host(pl2.forward()), img), frame
        pl2.close()
        live = (ref["start"] <= frame) & (frame < ref["expire"])
        if keep_frac is None and frame >= 1:
            assert live.sum() == NUM_GS            # Algorithm 2: num_gs live Gaussians every frame
        elif frame >= 1:
            assert live.sum() < NUM_GS             # tail-dropped slots are empty
    player.close()


def test_player_queue_limits_and_late_records(sw, ctx):
    stream = trainer_stream(sw, ctx, 5, 2, None)
    buf_pool = sw.Pool(np.zeros((F, NUM_GS), np.float32), np.full(NUM_GS, -1, np.int32),
                       np.full(NUM_GS, -1, np.int32), np.full(NUM_GS, -1, np.int32), 0, SWIN, DEG, "cuda",
                       train=False)
    player = sw.Player(ctx, buf_pool, queue_depth=2, max_record_bytes=max(len(d) for d, _, _ in stream))
    player.push(stream[0][0])
    player.push(stream[1][0])
    with pytest.raises(sw.SwgsError) as e:
        player.push(stream[2][0])
    assert e.value.status == sw.SWGS_ERR_CAPACITY
    assert player.advance(0) == 1                  # the genesis record (birth 0)
    assert player.advance(5) == 1                  # frame 1's slice, applied late
    player.push(stream[2][0])
    assert player.queued() == (1, 2)
    assert player.advance(1) == 0 and player.advance(2) == 1
    with pytest.raises(sw.SwgsError):
        player.push(b"\x00" * 64)                  # not a record
    small = sw.Pool(np.zeros((F, 10), np.float32), np.zeros(10, np.int32), np.zeros(10, np.int32),
                    np.zeros(10, np.int32), 0, SWIN, DEG, "cuda", train=False)
    p2 = sw.Player(ctx, small, queue_depth=1, max_record_bytes=len(stream[3][0]))
    with pytest.raises(sw.SwgsError):
        p2.push(stream[3][0])                       # slots outside a 10-slot buffer
    p2.close()
    player.close()

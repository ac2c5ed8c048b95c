"""GPU tests of the serving side, through the C ABI: Algorithm 2's update
(swgs_apply_update) against the oracle's mature records and client replay,
and the render server (swgs_server_*): served images against the FP64
oracle (1e-5 absolute), each image identical alone and in a mixed batch (bit
for bit), admission by memory budget, pair-overflow recovery, invalid
requests, real-time arrivals and the submit/progress interface."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2409_07759_amd import synth as S
from scenes import IMG_TOL, MARGIN_PIX

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


SIZES = [(64, 48), (96, 72), (40, 30), (33, 17), (128, 96), (17, 64)]


def requests(n, n_frames, seed, sizes=SIZES):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        v = S.random_pose_view(rng, int(rng.integers(0, n_frames)), W, H)
        if i % 3 == 1:
            v.bg = (0.2, 0.1, 0.05)
        out.append(v)
    return out


def out_images(views):
    return [torch.full((3, v.height, v.width), float("nan"), device="cuda") for v in views]


@pytest.fixture(scope="module")
def serving(sw):
    pool = S.serving_pool(1500, 6, 1, 4)
    return pool, sw.Pool.from_synth(pool, train=False)


# ------------------------------------------------------- Algorithm 2 update
def test_apply_update_replays_algorithm2(sw, ctx):
    """Training side: genesis, schedule_expire and mature(st) for st = 1..10
    on the device (parameters re-drawn between matures as training would);
    client side: each record applied into a num_gs-slot buffer at the slots
    it came from, at its birth frame.  The client's buffer equals the
    oracle's replay bit for bit, and its live set at every frame equals the
    server's snapshots; appending the records instead (slot_base) gives a
    resident pool with the same per-frame content."""
    say("apply_update replay")
    num_gs, swin, deg = 40, 4, 1
    F = 11 + 3 * (deg + 1) ** 2
    rng = np.random.default_rng(21)
    P = np.zeros((F, 2 * num_gs), np.float32)
    P[:, :num_gs] = S.make_gaussians(num_gs, deg, 5)
    b, s_, e = O.genesis(num_gs, swin)
    e = O.schedule_expire(num_gs, swin, e)
    dp = sw.Pool(P, b, s_, e, num_gs, swin, deg, "cuda", train=True)
    # the client buffer (forward-only pool of num_gs slots)
    client = sw.Pool(np.zeros((F, num_gs), np.float32), np.zeros(num_gs, np.int32), np.zeros(num_gs, np.int32),
                     np.zeros(num_gs, np.int32), 0, swin, deg, "cuda", train=False)
    resident_n = num_gs + 10 * (num_gs // swin)
    resident = sw.Pool(np.zeros((F, resident_n), np.float32), np.zeros(resident_n, np.int32),
                       np.zeros(resident_n, np.int32), np.zeros(resident_n, np.int32), 0, swin, deg, "cuda",
                       train=False)
    cur = 0
    ref_buf = {}
    records = []
    Ph, bh, sh_, eh = P.astype(np.float64), b.copy(), s_.copy(), e.copy()
    for st in range(1, 11):
        rec, cnt = sw.mature(ctx, dp, st)
        ref = O.mature(st, num_gs, swin, Ph, bh, sh_, eh)
        r = sw.parse_record(host(rec))
        assert cnt == len(ref["slots"]) and np.array_equal(r["slots"], ref["slots"].astype(np.uint32))
        assert np.array_equal(r["params"], ref["params"].astype(np.float32))
        records.append(r)
        # Algorithm 2: slice birth mod swin of the client buffer is replaced
        if st > 1:
            assert np.all(r["slots"] // (num_gs // swin) == r["birth"][0] % swin)
        assert sw.apply_update(ctx, client, rec) == cnt
        assert sw.apply_update(ctx, resident, rec, slot_base=cur) == cnt
        cur += cnt
        for j, slot in enumerate(r["slots"]):
            ref_buf[int(slot)] = (r["params"][:, j], r["birth"][j], r["start"][j], r["expire"][j])
        # training continues: new values for the optimisable slots
        newp = rng.normal(size=(F, num_gs)).astype(np.float32) * 0.1 + P[:, :num_gs]
        Ph[:, :num_gs] = newp
        dp.params[:, :num_gs] = torch.as_tensor(newp, device="cuda")
    cp, cb, cs, ce = host(client.params), host(client.birth), host(client.start), host(client.expire)
    for slot, (pp, bb, ss, ee) in ref_buf.items():
        assert np.array_equal(cp[:, slot], pp) and cb[slot] == bb and cs[slot] == ss and ce[slot] == ee
    rp, rs, re_ = host(resident.params), host(resident.start), host(resident.expire)
    for frame in range(1, 9):
        # server side: the latest snapshot of every slot covering the frame
        snaps = {}
        for r in records:
            for j, slot in enumerate(r["slots"]):
                if r["start"][j] <= frame < r["expire"][j]:
                    snaps[int(slot)] = r["params"][:, j]
        assert len(snaps) == num_gs
        live_res = np.nonzero((rs[:cur] <= frame) & (frame < re_[:cur]))[0]
        got = sorted(map(tuple, rp[:, live_res].T.tolist()))
        want = sorted(map(tuple, np.stack(list(snaps.values()), 1).T.tolist()))
        assert got == want, frame


def test_apply_update_rejects_bad_records(sw, ctx):
    say("apply_update errors")
    num_gs, swin = 20, 4
    pool = S.steady_window_pool(num_gs, swin, 0, 6, 1)
    dp = sw.Pool.from_synth(pool)
    rec, cnt = sw.mature(ctx, dp, 7)
    small = sw.Pool(np.zeros((14, 8), np.float32), np.zeros(8, np.int32), np.zeros(8, np.int32),
                    np.zeros(8, np.int32), 0, swin, 0, "cuda", train=False)
    with pytest.raises(sw.SwgsError) as ei:
        sw.apply_update(ctx, small, rec, slot_base=4)          # 4 + 5 > 8 slots
    assert ei.value.status == sw.SWGS_ERR_INVALID_ARG
    with pytest.raises(sw.SwgsError) as ei:
        sw.apply_update(ctx, small, rec)                       # record slots up to 19 > 8
    assert ei.value.status == sw.SWGS_ERR_INVALID_ARG and "outside" in str(ei.value)
    bad = rec.clone()
    bad[0] = 0
    with pytest.raises(sw.SwgsError):
        sw.apply_update(ctx, dp, bad)
    deg1 = sw.Pool(np.zeros((23, 40), np.float32), np.zeros(40, np.int32), np.zeros(40, np.int32),
                   np.zeros(40, np.int32), 0, swin, 1, "cuda", train=False)
    with pytest.raises(sw.SwgsError):
        sw.apply_update(ctx, deg1, rec)                        # SH degree differs
    with pytest.raises(sw.SwgsError):
        sw.apply_update(ctx, dp, rec[:40])                     # truncated


# ----------------------------------------------------------------- server
def check_against_oracle(pool, views, imgs):
    for v, im in zip(views, imgs):
        n = v.width * v.height
        rgb, To, cnt, dm, cm = O.render_view(pool.params, pool.sh_degree, pool.start, pool.expire, v)
        keep = dm >= MARGIN_PIX
        got = host(im).reshape(3, n)
        assert np.isfinite(got).all()
        assert np.abs(got - rgb)[:, keep].max(initial=0) <= IMG_TOL, (v.frame, v.width, v.height)
        assert (~keep).sum() <= max(2, n // 100)


def test_server_images_match_oracle(sw, ctx, serving):
    pool, dp = serving
    views = requests(14, 6, 31)
    say("server vs oracle", len(views))
    srv = sw.Server(ctx, dp, 6, 256 << 20, lanes=2, max_batch=4)
    imgs = out_images(views)
    (arr, ready, status, batch), st = srv.run(views, images=imgs)
    srv.close()
    assert (status == sw.SWGS_OK).all() and st["completed"] == len(views) and st["failed"] == 0
    assert st["batches"] >= 4 and st["mean_batch"] <= 4
    check_against_oracle(pool, views, imgs)


def test_served_image_is_the_same_alone_and_in_the_mix(sw, ctx, serving):
    pool, dp = serving
    views = requests(24, 6, 32)
    say("alone vs mix", len(views))
    mixed = out_images(views)
    srv = sw.Server(ctx, dp, 6, 256 << 20, lanes=3, max_batch=8)
    (_, _, status, batch), st = srv.run(views, images=mixed)
    assert (status == sw.SWGS_OK).all() and st["batches"] >= 3 and st["mean_batch"] > 1
    srv.close()
    alone = out_images(views)
    one = sw.Server(ctx, dp, 6, 256 << 20, lanes=1, max_batch=1)
    (_, _, status1, batch1), st1 = one.run(views, images=alone)
    one.close()
    assert (status1 == sw.SWGS_OK).all() and st1["batches"] == len(views)
    for i, v in enumerate(views):
        a, b = host(mixed[i]), host(alone[i])
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), i
    # and equal to a training plan's forward of the same view
    for i in (0, 5, 11):
        pl = sw.Plan(ctx, dp, [views[i]])
        im = host(pl.forward())
        pl.close()
        assert np.array_equal(im.view(np.uint32), host(mixed[i]).reshape(-1).view(np.uint32)), i


def test_server_admission_by_memory_budget(sw, ctx, serving):
    """A budget that holds one large request at a time: everything still
    completes, in more batches, never above the budget; a request larger than
    the whole budget fails alone."""
    pool, dp = serving
    views = requests(6, 6, 33, sizes=[(640, 480), (48, 32)])
    huge = S.random_pose_view(np.random.default_rng(1), 2, 2048, 2048)
    views.insert(3, huge)
    say("admission", [(v.width, v.height) for v in views])
    ref = out_images(views)
    big = sw.Server(ctx, dp, 6, 512 << 20, lanes=1, max_batch=1)
    (_, _, s_ref, _), _ = big.run(views, images=ref)
    big.close()
    assert (s_ref == sw.SWGS_OK).all()
    got = out_images(views)
    srv = sw.Server(ctx, dp, 6, 40 << 20, lanes=3, max_batch=8)
    (_, _, status, batch), st = srv.run(views, images=got)
    srv.close()
    say("admission stats", st)
    assert status[3] == sw.SWGS_ERR_WORKSPACE_TOO_SMALL
    ok = [i for i in range(len(views)) if i != 3]
    assert (status[ok] == sw.SWGS_OK).all() and st["completed"] == len(ok) and st["failed"] == 1
    assert st["peak_bytes"] <= st["budget_bytes"]
    for i in ok:
        assert np.array_equal(host(got[i]).view(np.uint32), host(ref[i]).view(np.uint32)), i


def test_server_recovers_from_pair_overflow(sw, ctx, serving):
    pool, dp = serving
    views = requests(10, 6, 34)
    say("overflow redo")
    ref = out_images(views)
    a = sw.Server(ctx, dp, 6, 256 << 20, lanes=1, max_batch=1)
    a.run(views, images=ref)
    a.close()
    got = out_images(views)
    srv = sw.Server(ctx, dp, 6, 256 << 20, lanes=2, max_batch=5, pair_ratio=1e-4)
    (_, _, status, _), st = srv.run(views, images=got)
    srv.close()
    assert (status == sw.SWGS_OK).all() and st["redone"] >= 1
    for i in range(len(views)):
        assert np.array_equal(host(got[i]).view(np.uint32), host(ref[i]).view(np.uint32)), i


def test_server_rejects_invalid_requests_only(sw, ctx, serving):
    pool, dp = serving
    views = requests(5, 6, 35)
    views[1].frame = 6            # outside the clip
    views[3].width = 0
    say("invalid requests")
    srv = sw.Server(ctx, dp, 6, 128 << 20, lanes=2, max_batch=4)
    imgs = [None if i in (1, 3) else torch.zeros((3, v.height, v.width), device="cuda")
            for i, v in enumerate(views)]
    (_, _, status, _), st = srv.run(views, images=imgs)
    srv.close()
    assert status[1] == sw.SWGS_ERR_INVALID_ARG and status[3] == sw.SWGS_ERR_INVALID_ARG
    assert (status[[0, 2, 4]] == sw.SWGS_OK).all() and st["failed"] == 2
    with pytest.raises(sw.SwgsError):
        sw.Server(ctx, dp, 6, 128 << 20, lanes=9)
    with pytest.raises(sw.SwgsError):
        sw.Server(ctx, dp, 6, 128 << 20, tile=(16, 8))
    with pytest.raises(sw.SwgsError):
        sw.Server(ctx, dp, 6, 4096)   # arena cannot hold the live lists


def test_server_realtime_poisson_arrivals(sw, ctx, serving):
    """Arrivals replayed on the clock: every request is ready after it
    arrived, and the images equal the all-at-once renders."""
    pool, dp = serving
    rng = np.random.default_rng(36)
    n = 80
    arrivals = np.cumsum(rng.exponential(1.0 / 400.0, size=n))
    views = requests(n, 6, 37)
    say("realtime", n, "over", float(arrivals[-1]), "s")
    got = out_images(views)
    srv = sw.Server(ctx, dp, 6, 256 << 20, lanes=3, max_batch=8)
    (arr, ready, status, batch), st = srv.run(views, arrivals=arrivals, images=got, realtime=True)
    assert (status == sw.SWGS_OK).all()
    assert np.allclose(arr, arrivals) and (ready >= arr).all()
    assert st["wall_s"] >= arrivals[-1] - arrivals[0]
    ref = out_images(views)
    srv.run(views, images=ref)
    srv.close()
    for i in range(n):
        assert np.array_equal(host(got[i]).view(np.uint32), host(ref[i]).view(np.uint32)), i


def test_server_submit_and_progress(sw, ctx, serving):
    pool, dp = serving
    views = requests(9, 6, 38)
    say("submit/progress")
    srv = sw.Server(ctx, dp, 6, 256 << 20, lanes=2, max_batch=3)
    imgs = out_images(views)
    reqs = srv.submit(views[:5], images=imgs[:5])
    reqs2 = srv.submit(views[5:], images=imgs[5:])
    for _ in range(100000):
        if srv.progress(wait=True) == 0:
            break
    assert all(r.status == sw.SWGS_OK for r in list(reqs) + list(reqs2))
    assert all(r.ready >= r.arrival for r in list(reqs) + list(reqs2))
    srv.close()
    check_against_oracle(pool, views[:4], imgs[:4])


# ---------------------------------------------------- standalone batch render
def test_render_batch_matches_server_and_oracle(sw, ctx, serving):
    """swgs_render_batch (no server: gating in its own workspace) renders a
    batch of mixed frames and resolutions bit-identical to the server's
    images of the same requests, and within 1e-5 of the oracle."""
    pool, dp = serving
    views = requests(10, 6, 41)
    say("render_batch", len(views))
    got = out_images(views)
    status, ws_bytes = sw.render_batch(ctx, dp, views, images=got)
    assert (status == sw.SWGS_OK).all() and ws_bytes > 0
    ref = out_images(views)
    srv = sw.Server(ctx, dp, 6, 256 << 20, lanes=2, max_batch=4)
    (_, _, st2, _), _ = srv.run(views, images=ref)
    srv.close()
    assert (st2 == sw.SWGS_OK).all()
    for a, b in zip(got, ref):
        assert np.array_equal(host(a).view(np.uint32), host(b).view(np.uint32))
    check_against_oracle(pool, views, got)


def test_render_batch_reports_capacity_and_bad_workspace(sw, ctx, serving):
    pool, dp = serving
    views = requests(4, 6, 42)
    say("render_batch capacity")
    with pytest.raises(sw.SwgsError) as e:
        sw.render_batch(ctx, dp, views, images=out_images(views), pair_capacity=64)
    assert e.value.status == sw.SWGS_ERR_CAPACITY and "needs" in str(e.value)
    import ctypes
    reqs = sw.c_requests(views)
    cp = dp.c()
    opts = sw.SwgsPlanOpts(ctypes.sizeof(sw.SwgsPlanOpts), 16, 16, 0, 0, 1 << 20)
    nb = ctypes.c_size_t()
    ctx.check(sw.swgs_query_workspace_batch(ctx.h, ctypes.byref(cp), reqs, len(views), ctypes.byref(opts),
                                            ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    assert sw.swgs_render_batch(ctx.h, ctypes.byref(cp), reqs, len(views), ctypes.byref(opts), sw.ptr(ws),
                                nb.value - 256) == sw.SWGS_ERR_WORKSPACE_TOO_SMALL


def test_pool_bind_checks_device_pointers(sw, ctx, serving):
    """swgs_pool_bind keeps the checked descriptor; a host pointer in it is
    refused; a plan made from the bound descriptor renders."""
    import ctypes
    pool, dp = serving
    b = sw.BoundPool(ctx, dp)
    d = ctypes.cast(b.desc(), ctypes.POINTER(sw.SwgsPool)).contents
    assert d.params == dp.params.data_ptr() and d.n_slots == dp.params.shape[1]
    pl = sw.Plan(ctx, dp, requests(2, 6, 43))
    assert np.isfinite(host(pl.forward())).all()
    pl.close()
    b.close()
    host_params = np.zeros(16, np.float32)
    bad = dp.c()
    bad.params = host_params.ctypes.data
    h = ctypes.c_void_p()
    assert sw.swgs_pool_bind(ctx.h, ctypes.byref(bad), ctypes.byref(h)) == sw.SWGS_ERR_INVALID_ARG
    assert b"params" in sw.swgs_last_error(ctx.h)

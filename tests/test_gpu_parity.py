"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bit-exact: active lists, tile ranges (rects), tile counts, FP32 depth keys,
depth order, sorted (tile, record) pairs, tile ranges, relocation indices,
mature records.  Images within 1e-5 absolute (pixels whose skip/stop decision
is within 1e-4 of its threshold are excluded and counted); gradients within
1e-3 relative with a 1e-2 * max floor per tensor."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2409_07759_amd import synth as S
from scenes import IMG_TOL, MARGIN_INT, MARGIN_PIX, grad_close, steady, tiny

pytestmark = pytest.mark.gpu

TILES = [(16, 16), (8, 8), (32, 8)]


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


def plan_for(sw, ctx, pool, views, tile=(16, 16), lds=0, train=True, cap=None):
    dp = sw.Pool.from_synth(pool, train=train)
    return dp, sw.Plan(ctx, dp, views, tile=tile, lds_batch=lds, pair_capacity=cap)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ----------------------------------------------------------------- a1 gating
def test_gating_lists_bit_exact(sw, ctx):
    say("gating tiny")
    pool, views = tiny()
    dp, pl = plan_for(sw, ctx, pool, views)
    pl.forward()
    counts = host(pl.buffer(sw.SWGS_BUF_ACTIVE_COUNT))
    lists = host(pl.buffer(sw.SWGS_BUF_ACTIVE_LIST))
    o = 0
    for g, f in enumerate([0, 1, 2]):
        ref = np.nonzero(O.active(pool.start, pool.expire, f))[0]
        assert counts[g] == len(ref)
        assert np.array_equal(lists[o:o + len(ref)], ref.astype(np.uint32))
        o += len(ref)
    A = np.nonzero(O.window_set(pool.start, pool.expire, pool.num_gs, [0, 1, 2]))[0]
    assert counts[3] == len(A) and np.array_equal(lists[o:o + len(A)], A.astype(np.uint32))


def test_gating_steady_pool_with_frozen_store(sw, ctx):
    say("gating steady")
    pool, views = steady()
    dp, pl = plan_for(sw, ctx, pool, views)
    pl.forward()
    counts = host(pl.buffer(sw.SWGS_BUF_ACTIVE_COUNT))
    lists = host(pl.buffer(sw.SWGS_BUF_ACTIVE_LIST))
    frames = sorted(set(v.frame for v in views), key=[v.frame for v in views].index)
    o = 0
    for g, f in enumerate(frames):
        ref = np.nonzero(O.active(pool.start, pool.expire, f))[0]
        assert counts[g] == len(ref) == pool.num_gs
        assert np.array_equal(lists[o:o + len(ref)], ref)
        o += len(ref)


# ------------------------------------------------------- a2 preprocess records
def records_of(sw, pl, pool, views):
    lists = host(pl.buffer(sw.SWGS_BUF_ACTIVE_LIST))
    rvb = host(pl.buffer(sw.SWGS_BUF_RECORD_VIEW_BASE))
    tc = host(pl.buffer(sw.SWGS_BUF_TILE_COUNT))
    rect = host(pl.buffer(sw.SWGS_BUF_RECT)).reshape(-1, 2)
    splat = host(pl.buffer(sw.SWGS_BUF_SPLAT, torch.float32)).reshape(-1, 12)
    frames = []
    for v in views:
        if v.frame not in frames:
            frames.append(v.frame)
    counts = host(pl.buffer(sw.SWGS_BUF_ACTIVE_COUNT))
    base = np.concatenate([[0], np.cumsum(counts[:len(frames)].astype(np.int64))]).astype(np.int64)
    out = []
    for vi, v in enumerate(views):
        g = frames.index(v.frame)
        slots = lists[base[g]:base[g + 1]]
        r0 = int(rvb[vi])
        out.append((slots, tc[r0:r0 + len(slots)], rect[r0:r0 + len(slots)], splat[r0:r0 + len(slots)]))
    return out


@pytest.mark.parametrize("tile", TILES)
def test_preprocess_records_bit_exact_decisions(sw, ctx, tile):
    say("preprocess tiny", tile)
    pool, views = tiny()
    dp, pl = plan_for(sw, ctx, pool, views, tile=tile)
    pl.forward()
    recs = records_of(sw, pl, pool, views)
    flagged = mism = 0
    for v, (slots, tc, rect, splat) in zip(views, recs):
        vis, rec, orect = O.preprocess(pool.params, 0, pool.start, pool.expire, v, *tile)
        m = rec[slots, O.R_MARGIN]
        ok = m >= MARGIN_INT
        flagged += int((~ok).sum())
        ovis = vis[slots] == 1
        gvis = tc > 0
        gx0, gy0 = rect[:, 0] & 0xFFFF, rect[:, 0] >> 16
        gx1, gy1 = rect[:, 1] & 0xFFFF, rect[:, 1] >> 16
        orc = orect[slots]
        same = (ovis == gvis)
        same &= ~ovis | ((gx0 == orc[:, 0]) & (gy0 == orc[:, 1]) & (gx1 == orc[:, 2]) & (gy1 == orc[:, 3]))
        same &= ~ovis | (tc == (orc[:, 2] - orc[:, 0]) * (orc[:, 3] - orc[:, 1]))
        # FP32 depth key: bit-exact
        od = rec[slots, O.R_DEPTH].astype(np.float32)
        same &= ~ovis | (splat[:, 11].view(np.uint32) == od.view(np.uint32))
        mism += int((~same & ok).sum())
        assert np.all(same | ~ok)
        # values
        w = ovis & ok
        u = splat[w, 0].astype(np.float64) + 0.5 - splat[w, 2]
        vv = splat[w, 1].astype(np.float64) + 0.5 - splat[w, 3]
        assert np.allclose(u, rec[slots[w], O.R_U], atol=2e-6, rtol=0)
        assert np.allclose(vv, rec[slots[w], O.R_V], atol=2e-6, rtol=0)
        l2e = 1.4426950408889634
        assert np.allclose(-2 * splat[w, 4] / l2e, rec[slots[w], O.R_A], rtol=3e-7, atol=1e-12)
        assert np.allclose(-splat[w, 5] / l2e, rec[slots[w], O.R_B], rtol=3e-7, atol=1e-7 * np.abs(rec[slots[w], O.R_A]).max())
        assert np.allclose(-2 * splat[w, 6] / l2e, rec[slots[w], O.R_C], rtol=3e-7, atol=1e-12)
        assert np.allclose(splat[w, 7], rec[slots[w], O.R_OPA], rtol=1e-7)
        assert np.allclose(splat[w, 8:11], rec[slots[w], O.R_RGB:O.R_RGB + 3], rtol=1e-7, atol=1e-7)
    say("flagged records", flagged)
    assert mism == 0 and flagged <= 0.01 * pl.n_records


# ------------------------------------------------------- a3/a4 binning + sort
@pytest.mark.parametrize("tile", TILES)
def test_sorted_pairs_and_ranges_bit_exact(sw, ctx, tile):
    say("sort tiny", tile)
    pool, views = tiny()
    dp, pl = plan_for(sw, ctx, pool, views, tile=tile)
    pl.forward()
    recs = records_of(sw, pl, pool, views)
    K = int(host(pl.buffer(sw.SWGS_BUF_PAIR_COUNT))[0])
    keys = host(pl.buffer(sw.SWGS_BUF_PAIR_KEY))[:K]
    vals = host(pl.buffer(sw.SWGS_BUF_PAIR_VAL))[:K]
    ranges = host(pl.buffer(sw.SWGS_BUF_TILE_RANGE)).reshape(-1, 2)
    rvb = host(pl.buffer(sw.SWGS_BUF_RECORD_VIEW_BASE))
    # record -> slot
    rec_slot = np.zeros(pl.n_records, np.int64)
    for vi, (slots, *_r) in enumerate(recs):
        rec_slot[rvb[vi]:rvb[vi] + len(slots)] = slots
    ref_tiles, ref_slots = [], []
    tbase = 0
    flagged = 0
    for v in views:
        vis, rec, rect = O.preprocess(pool.params, 0, pool.start, pool.expire, v, *tile)
        act = O.active(pool.start, pool.expire, v.frame)
        flagged += int(((rec[:, O.R_MARGIN] < MARGIN_INT) & act).sum())
        t, s_, rg = O.tile_pairs(vis, rec, rect, v, *tile)
        ref_tiles.append(t + tbase)
        ref_slots.append(s_)
        nt = ((v.width + tile[0] - 1) // tile[0]) * ((v.height + tile[1] - 1) // tile[1])
        assert np.array_equal(ranges[tbase:tbase + nt, 1] - ranges[tbase:tbase + nt, 0], rg[:, 1] - rg[:, 0])
        tbase += nt
    ref_tiles = np.concatenate(ref_tiles)
    ref_slots = np.concatenate(ref_slots)
    say("pairs", K, "flagged", flagged)
    if flagged == 0:
        assert K == len(ref_tiles)
        assert np.array_equal(keys.astype(np.int64), ref_tiles)
        assert np.array_equal(rec_slot[vals], ref_slots)
    else:
        # flagged records may legitimately differ; everything else must not
        assert abs(K - len(ref_tiles)) <= 8 * flagged
    # depth order: records by (FP32 depth, record)
    order = host(pl.buffer(sw.SWGS_BUF_DEPTH_ORDER))[:pl.n_records]
    splat = host(pl.buffer(sw.SWGS_BUF_SPLAT, torch.float32)).reshape(-1, 12)
    tc = host(pl.buffer(sw.SWGS_BUF_TILE_COUNT))
    dk = np.where(tc > 0, splat[:, 11].view(np.uint32), np.uint32(0xFFFFFFFF)).astype(np.uint64)
    ref = np.lexsort((np.arange(pl.n_records), dk))
    assert np.array_equal(order, ref)


def test_dense_tiles_lists_and_pixels(sw, ctx):
    """Tiles holding many thousands of pairs (up to ~17k): their depth-ordered
    lists and pixels still match the oracle."""
    say("dense tiles")
    pool, views = tiny(n=60000, width=40, height=24, frames=(0,), cams=2)
    dp, pl = plan_for(sw, ctx, pool, views, tile=(16, 16))
    img = host(pl.forward())
    K = int(host(pl.buffer(sw.SWGS_BUF_PAIR_COUNT))[0])
    vals = host(pl.buffer(sw.SWGS_BUF_PAIR_VAL))[:K]
    ranges = host(pl.buffer(sw.SWGS_BUF_TILE_RANGE)).reshape(-1, 2)
    rvb = host(pl.buffer(sw.SWGS_BUF_RECORD_VIEW_BASE))
    recs = records_of(sw, pl, pool, views)
    counts = ranges[:, 1] - ranges[:, 0]
    say("largest tile", int(counts.max()))
    assert counts.max() > 3 * 4096
    rec_slot = np.zeros(pl.n_records, np.int64)
    for vi, (slots, *_r) in enumerate(recs):
        rec_slot[rvb[vi]:rvb[vi] + len(slots)] = slots
    tbase, o = 0, 0
    for v in views:
        vis, rec, rect = O.preprocess(pool.params, 0, pool.start, pool.expire, v, 16, 16)
        t, s_, rg = O.tile_pairs(vis, rec, rect, v, 16, 16)
        act = O.active(pool.start, pool.expire, v.frame)
        nt = len(rg)
        if not ((rec[:, O.R_MARGIN] < MARGIN_INT) & act).any():
            for k in range(nt):
                lo, hi = ranges[tbase + k]
                assert np.array_equal(rec_slot[vals[lo:hi]], s_[rg[k, 0]:rg[k, 1]]), k
        n = v.width * v.height
        rgb, To, cnt, dm, cm = O.render_view(pool.params, 0, pool.start, pool.expire, v)
        keep = dm >= MARGIN_PIX
        assert np.abs(img[o:o + 3 * n].reshape(3, n) - rgb)[:, keep].max(initial=0) <= IMG_TOL
        tbase += nt
        o += 3 * n


# ----------------------------------------------------------- a5 forward blend
def render_gpu(sw, ctx, pool, views, tile, lds=0):
    dp, pl = plan_for(sw, ctx, pool, views, tile=tile, lds=lds)
    img = pl.forward()
    return host(img), host(pl.buffer(sw.SWGS_BUF_T_FINAL, torch.float32)), pl


@pytest.mark.parametrize("tile", TILES)
def test_forward_images_match_oracle(sw, ctx, tile):
    say("forward tiny", tile)
    pool, views = tiny()
    for v in views[1::3]:
        v.bg = (0.25, 0.5, 1.0)
    img, T, pl = render_gpu(sw, ctx, pool, views, tile)
    o3 = o1 = 0
    excl = total = 0
    worst = 0.0
    for v in views:
        n = v.width * v.height
        rgb, To, cnt, dm, cm = O.render_view(pool.params, 0, pool.start, pool.expire, v)
        g = img[o3:o3 + 3 * n].reshape(3, n)
        keep = dm >= MARGIN_PIX
        excl += int((~keep).sum())
        total += n
        d = np.abs(g - rgb)[:, keep]
        worst = max(worst, float(d.max()))
        assert d.max() <= IMG_TOL
        assert np.abs(T[o1:o1 + n] - To)[keep].max() <= IMG_TOL
        o3 += 3 * n
        o1 += n
    say("worst", worst, "excluded", excl, "of", total)
    assert excl <= 1e-3 * total


def test_images_bit_identical_across_tile_shapes(sw, ctx):
    say("tile invariance")
    pool, views = tiny(width=100, height=75)      # ragged tails for every tile shape
    ref = None
    for tile, lds in [((16, 16), 256), ((16, 16), 128), ((8, 8), 64), ((8, 8), 128), ((32, 8), 256)]:
        img, T, _ = render_gpu(sw, ctx, pool, views, tile, lds)
        if ref is None:
            ref = (img, T)
        else:
            assert np.array_equal(img.view(np.uint32), ref[0].view(np.uint32)), (tile, lds)
            assert np.array_equal(T.view(np.uint32), ref[1].view(np.uint32)), (tile, lds)


def test_forward_ragged_sizes_and_sh_degrees(sw, ctx):
    for deg, (W, H) in [(1, (37, 23)), (2, (64, 1)), (3, (1, 1)), (3, (73, 50))]:
        say("forward deg", deg, W, H)
        pool, views = tiny(n=600, width=W, height=H, deg=deg, frames=(0, 2), cams=2)
        img, T, _ = render_gpu(sw, ctx, pool, views, (16, 16))
        o = 0
        for v in views:
            n = W * H
            rgb, To, cnt, dm, cm = O.render_view(pool.params, deg, pool.start, pool.expire, v)
            keep = dm >= MARGIN_PIX
            assert np.abs(img[o:o + 3 * n].reshape(3, n) - rgb)[:, keep].max(initial=0) <= IMG_TOL
            o += 3 * n


def test_empty_frame_and_culled_views(sw, ctx):
    say("empty frame")
    pool, _ = tiny(n=300)
    views = S.ring_views([7], 2, 32, 24)           # no Gaussian lives at frame 7
    views += S.ring_views([0], 1, 32, 24, radius=0.1)  # camera inside the cloud
    v_far = S.ring_views([0], 1, 32, 24)[0]
    v_far.t = v_far.t + np.array([0.0, 0.0, -50.0])  # everything behind the camera
    views.append(v_far)
    for v in views:
        v.bg = (0.1, 0.2, 0.3)
    img, T, pl = render_gpu(sw, ctx, pool, views, (16, 16))
    o = 0
    for v in views:
        n = v.width * v.height
        rgb, To, *_ = O.render_view(pool.params, 0, pool.start, pool.expire, v)
        assert np.abs(img[o:o + 3 * n].reshape(3, n) - rgb).max() <= IMG_TOL
        o += 3 * n
    assert np.allclose(img[:3 * 32 * 24].reshape(3, -1), np.array([0.1, 0.2, 0.3])[:, None])


# ------------------------------------------------------------- a7 backward
def masked_upstream(pool, views, seed):
    """Random dL/dimage, zeroed at pixels whose skip/stop/clamp decision lies
    within MARGIN_PIX of its threshold (there the two sides may blend a
    different set; with zero upstream gradient such a pixel contributes
    nothing to either gradient)."""
    rng = np.random.default_rng(seed)
    out = []
    for v in views:
        n = v.width * v.height
        rgb, To, cnt, dm, cm = O.render_view(pool.params, pool.sh_degree, pool.start, pool.expire, v)
        g = rng.uniform(-1, 1, size=(3, n))
        g[:, (dm < MARGIN_PIX) | (cm < MARGIN_PIX)] = 0.0
        out.append(g.reshape(-1))
    return np.concatenate(out)


@pytest.mark.parametrize("tile", TILES)
def test_backward_record_and_param_gradients(sw, ctx, tile):
    # every tile shape: one wave per 8x8 tile (no per-wave lists) and four
    # waves per 16x16 / 32x8 tile take different paths through the backward
    say(f"backward tiny {tile}")
    pool, views = tiny(n=1200, deg=1)
    dp, pl = plan_for(sw, ctx, pool, views, tile=tile)
    pl.forward()
    dL = masked_upstream(pool, views, 11)
    dp.grads.zero_()
    pl.backward(torch.as_tensor(dL, dtype=torch.float32, device="cuda"))
    recs = records_of(sw, pl, pool, views)
    rg = host(pl.buffer(sw.SWGS_BUF_RECORD_GRAD, torch.float32)).reshape(-1, 9).T
    rvb = host(pl.buffer(sw.SWGS_BUF_RECORD_VIEW_BASE))
    F = pool.params.shape[0]
    gsum = np.zeros((F, pool.slots))
    o = 0
    for vi, v in enumerate(views):
        n = 3 * v.width * v.height
        g, drec = O.view_backward(pool.params, 1, pool.start, pool.expire, v, pool.num_gs, dL[o:o + n])
        gsum += g
        slots = recs[vi][0]
        got = rg[:, rvb[vi]:rvb[vi] + len(slots)].T
        ref = drec[slots]
        for c in range(9):
            ok = grad_close(got[:, c], ref[:, c])
            assert ok.all(), (vi, c, np.nonzero(~ok)[0][:5], got[~ok, c][:5], ref[~ok, c][:5])
        o += n
    G = host(dp.grads)
    A = O.window_set(pool.start, pool.expire, pool.num_gs, [0, 1, 2])
    for r in range(F):
        ok = grad_close(G[r, A], gsum[r, A])
        assert ok.all(), (r, np.nonzero(~ok)[0][:5], G[r, A][~ok][:5], gsum[r, A][~ok][:5])


def test_frozen_slots_get_no_gradient(sw, ctx):
    say("frozen")
    pool, views = steady(num_gs=300, deg=0)
    dp, pl = plan_for(sw, ctx, pool, views)
    pl.forward()
    dL = masked_upstream(pool, views, 5)
    dp.grads.fill_(7.0)
    pl.backward(torch.as_tensor(dL, dtype=torch.float32, device="cuda"))
    G = host(dp.grads)
    gsum = np.zeros((pool.params.shape[0], pool.slots))
    o = 0
    for v in views:
        n = 3 * v.width * v.height
        g, _ = O.view_backward(pool.params, 0, pool.start, pool.expire, v, pool.num_gs, dL[o:o + n])
        gsum += g
        o += n
    assert np.all(gsum[:, pool.num_gs:] == 0)
    for r in range(pool.params.shape[0]):
        assert grad_close(G[r], gsum[r, :pool.num_gs]).all(), r


def test_autograd_function_matches_backward(sw, ctx):
    say("autograd")
    pool, views = tiny(n=500)
    dp, pl = plan_for(sw, ctx, pool, views)
    p = dp.params.requires_grad_(True)
    img = sw.render(p, pl)
    w = torch.randn_like(img)
    (img * w).sum().backward()
    g1 = p.grad.detach().clone()
    dp.grads.zero_()
    pl.forward()
    pl.backward(w)
    g2 = torch.zeros_like(g1)
    g2[:, :dp.num_gs] = dp.grads
    # same kernels and a fixed summation order: identical bits
    assert torch.equal(g1, g2)


def test_backward_is_deterministic(sw, ctx):
    """Record and parameter gradients come out bit-identical from repeated
    backward passes: every (tile, record) pair's terms land in their own
    slot and each record sums its slots in a fixed order (no float
    atomics).  Dense scene: most records cover several tiles."""
    say("deterministic backward")
    pool, views = tiny(n=4000, deg=2)
    dp, pl = plan_for(sw, ctx, pool, views, tile=(8, 8))
    pl.forward()
    n = sum(3 * v.width * v.height for v in views)
    dL = torch.as_tensor(np.random.default_rng(17).normal(size=n), dtype=torch.float32, device="cuda")
    outs = []
    for _ in range(3):
        dp.grads.fill_(3.0)
        pl.backward(dL)
        outs.append((host(pl.buffer(sw.SWGS_BUF_RECORD_GRAD, torch.float32)).copy(), host(dp.grads).copy()))
    tc = host(pl.buffer(sw.SWGS_BUF_TILE_COUNT))
    say("records", len(tc), "multi-tile", int((tc > 1).sum()), "max tiles", int(tc.max()))
    assert (tc > 1).sum() > 0.3 * (tc > 0).sum()
    for rg, g in outs[1:]:
        assert np.array_equal(rg.view(np.uint32), outs[0][0].view(np.uint32))
        assert np.array_equal(g.view(np.uint32), outs[0][1].view(np.uint32))


# ------------------------------------------------------------ a6 loss
def test_fused_l1_gradient_and_loss(sw, ctx):
    say("loss")
    pool, views = tiny(n=800)
    dp, pl = plan_for(sw, ctx, pool, views)
    tgt = S.random_images(views, 4)
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    img = pl.forward(targets=torch.as_tensor(tgt, device="cuda"), stats=stats)
    img_h = host(img)
    dldc = host(pl.buffer(sw.SWGS_BUF_DLDC, torch.float32))
    ref_img, _ = O.window_render(pool.params, 0, pool.start, pool.expire, views)
    L, l1, g, _ = O.loss_and_grad(ref_img, tgt, views, pool.params, np.zeros(pool.num_gs, bool))
    clear = np.abs(ref_img - tgt) > 1e-4
    assert np.array_equal(dldc[clear], g[clear].astype(np.float32))
    st = host(stats)
    assert st[0] == pytest.approx(l1, rel=1e-5)
    assert st[1] == pytest.approx(np.mean((ref_img - tgt) ** 2), rel=1e-5)


# ------------------------------------------------------------- a9 step
@pytest.mark.parametrize("use_eta", [True, False])
def test_adam_sgld_step_matches_oracle(sw, ctx, use_eta):
    say("step eta", use_eta)
    pool, views = tiny(n=700, deg=1)
    dp, pl = plan_for(sw, ctx, pool, views)
    rng = np.random.default_rng(2)
    F = pool.params.shape[0]
    g = rng.normal(0, 1e-3, size=(F, pool.num_gs)).astype(np.float32)
    m = rng.normal(0, 1e-4, size=(F, pool.num_gs)).astype(np.float32)
    v = rng.uniform(0, 1e-7, size=(F, pool.num_gs)).astype(np.float32)
    # a few very transparent Gaussians so the noise gate is open
    dp.params[10, :50] = -6.0
    P0 = host(dp.params).astype(np.float64)
    dp.grads.copy_(torch.as_tensor(g))
    dp.adam_m.copy_(torch.as_tensor(m))
    dp.adam_v.copy_(torch.as_tensor(v))
    A = O.window_set(pool.start, pool.expire, pool.num_gs, [0, 1, 2])
    eta = rng.normal(size=(3, pool.num_gs)).astype(np.float32) if use_eta else None
    cfg = sw.step_cfg(grad_scale_base=0.1, window_start=1)
    pl.step(cfg, adam_t=3, step=17, seed=99, eta=torch.as_tensor(eta, device="cuda") if use_eta else None)
    Pg = host(dp.params)
    # the oracle takes the hyper-parameters exactly as the kernel holds them (FP32 values)
    f32 = lambda x: float(np.float32(x))
    lr = {k: f32(v_) for k, v_ in O.DEFAULT_LR.items()}
    Pr, Mr, Vr = O.adam_sgld_step(P0[:, :pool.num_gs], g, m, v, A, 3, 1, seed=99, step=17, lr=lr,
                                  betas=(f32(cfg.beta1), f32(cfg.beta2)), eps=f32(cfg.eps),
                                  noise_lr=f32(cfg.noise_lr), k=f32(cfg.noise_k), t0=f32(cfg.noise_t0),
                                  eta=eta[:, A] if use_eta else None, grad_scale_base=f32(0.1), window_start=1,
                                  swin=3, start=pool.start[:pool.num_gs])
    assert np.allclose(Pg[:, :pool.num_gs], Pr, rtol=2e-6, atol=2e-7)
    # FP32 moments: cancellation in beta m + (1 - beta) g leaves ~ulp(1e-4) absolute error
    assert np.allclose(host(dp.adam_m), Mr, rtol=2e-6, atol=1e-10)
    assert np.allclose(host(dp.adam_v), Vr, rtol=2e-6, atol=1e-14)
    assert np.array_equal(Pg[:, ~A], P0[:, :pool.num_gs][:, ~A].astype(np.float32))
    # the noise actually moved the transparent means
    moved = np.abs(Pg[0:3, :50] - P0[0:3, :50]).max()
    assert moved > 1e-6


# -------------------------------------------------------- a10 relocation
def test_relocation_indices_bit_exact(sw, ctx):
    say("relocation")
    pool, views = tiny(n=1500, deg=1)
    rng = np.random.default_rng(6)
    dead = rng.uniform(size=pool.num_gs) < 0.25
    pool.params[10, dead] = rng.uniform(-12, -5.4, size=dead.sum()).astype(np.float32)
    dp, pl = plan_for(sw, ctx, pool, views)
    F = pool.params.shape[0]
    m = rng.normal(size=(F, pool.num_gs)).astype(np.float32)
    dp.adam_m.copy_(torch.as_tensor(m))
    dp.adam_v.copy_(torch.as_tensor(np.abs(m)))
    cfg = sw.step_cfg()
    dst, src = pl.relocate(cfg, step=(3 << 32) + 5, seed=1234)
    A = O.window_set(pool.start, pool.expire, pool.num_gs, [0, 1, 2])
    Pr, Mr, Vr, odst, osrc, wm = O.relocate(pool.params, m, np.abs(m), A, 1234, (3 << 32) + 5)
    # no alive weight sigmoid * 2^24 within FP64 rounding of an integer
    assert wm > 1e-13
    assert np.array_equal(host(dst), odst) and np.array_equal(host(src), osrc)
    assert len(odst) > 50
    Pg = host(dp.params)
    assert np.allclose(Pg, Pr, rtol=1e-6, atol=1e-6)
    assert np.array_equal(host(dp.adam_m) == 0, Mr == 0)


def test_relocation_many_chunks_and_cap_bit_exact(sw, ctx):
    """Relocation at the sizes a paper-scale window relocates at: a window set
    of 60,000 slots, so the alive-weight prefix spans 30 scan chunks of 2048
    with carries across every chunk boundary and the draws' upper-bound
    search runs over all of them; 40% of the slots are dead, and six opaque
    sources among faint ones draw far more copies than the cap N_max = 32.
    Indices bit-exact, parameters to 1e-6, Adam moments of sources and
    copies zeroed."""
    n = 60_000
    say("relocation many chunks", n)
    pool, views = tiny(n=n, deg=1)
    rng = np.random.default_rng(16)
    dead = rng.uniform(size=n) < 0.4
    lg = rng.uniform(-5.25, -4.6, size=n)                # alive and faint: sigma 0.0052 .. 0.0099
    lg[dead] = rng.uniform(-12.0, -5.4, size=int(dead.sum()))
    big = rng.choice(np.nonzero(~dead)[0], size=6, replace=False)
    lg[big] = rng.uniform(4.0, 6.0, size=6)
    pool.params[10] = lg.astype(np.float32)
    dp, pl = plan_for(sw, ctx, pool, views)
    F = pool.params.shape[0]
    m = rng.normal(size=(F, n)).astype(np.float32)
    dp.adam_m.copy_(torch.as_tensor(m))
    dp.adam_v.copy_(torch.as_tensor(np.abs(m)))
    cfg = sw.step_cfg()
    step, seed = (7 << 32) + 11, 98765
    dst, src = pl.relocate(cfg, step=step, seed=seed)
    A = O.window_set(pool.start, pool.expire, pool.num_gs, [0, 1, 2])
    assert A.all()
    Pr, Mr, Vr, odst, osrc, wm = O.relocate(pool.params, m, np.abs(m), A, seed, step)
    assert wm > 1e-13
    copies = np.bincount(osrc, minlength=n)
    say("dead", len(odst), "largest copy count", int(copies.max()), "sources", int((copies > 0).sum()))
    assert len(odst) == int(dead.sum()) and (n + 2047) // 2048 >= 30
    assert copies.max() + 1 > 32 and (copies > 0).sum() > 1000       # the cap applies; faint sources drawn too
    assert np.array_equal(host(dst), odst) and np.array_equal(host(src), osrc)
    Pg = host(dp.params)
    assert np.allclose(Pg, Pr, rtol=1e-6, atol=1e-6)
    assert np.array_equal(host(dp.adam_m) == 0, Mr == 0)
    assert np.array_equal(host(dp.adam_v) == 0, Vr == 0)


# ------------------------------------------------------------- a11 mature
def test_mature_record_and_pool_bit_exact(sw, ctx):
    say("mature")
    num_gs, swin = 250, 5
    pool = S.steady_window_pool(num_gs, swin, 1, 7, 2)
    dp = sw.Pool.from_synth(pool)
    P, b, s_, e = pool.params.copy(), pool.birth.copy(), pool.start.copy(), pool.expire.copy()
    for st in (8, 9):
        rec, cnt = sw.mature(ctx, dp, st)
        ref = O.mature(st, num_gs, swin, P, b, s_, e)
        r = sw.parse_record(host(rec))
        assert cnt == len(ref["slots"]) == num_gs // swin and r["count"] == cnt and r["st"] == st
        assert np.array_equal(r["slots"], ref["slots"].astype(np.uint32))
        for k in ("birth", "start", "expire"):
            assert np.array_equal(r[k], ref[k])
        assert np.array_equal(r["params"], ref["params"].astype(np.float32))
        assert np.array_equal(host(dp.params), P.astype(np.float32))
        assert np.array_equal(host(dp.birth), b) and np.array_equal(host(dp.start), s_)
        assert np.array_equal(host(dp.expire), e)


# ------------------------------------------------------------- window step
def test_window_step_modes_agree(sw, ctx):
    say("window step modes")
    pool, views = tiny(n=1500)
    tgt = torch.as_tensor(S.random_images(views, 8), device="cuda")
    outs = {}
    for mode in (sw.SWGS_MODE_PLAIN, sw.SWGS_MODE_BATCHED, sw.SWGS_MODE_GRAPH):
        dp, pl = plan_for(sw, ctx, pool, views)
        cfg = sw.step_cfg(mode=mode)
        img = pl.image_buffer()
        stats = torch.zeros(8, dtype=torch.float64, device="cuda")
        imgs = []
        for it in range(3):
            pl.window_step(cfg, tgt, adam_t=1 + it, step=it, seed=5, images=img, stats=stats)
            imgs.append(host(img).copy())
        outs[mode] = (imgs, host(dp.params), host(stats))
        say("mode", mode, "stats", host(stats))
    p_img, p_par, p_st = outs[sw.SWGS_MODE_PLAIN]
    for mode in (sw.SWGS_MODE_BATCHED, sw.SWGS_MODE_GRAPH):
        imgs, par, st = outs[mode]
        # first forward is identical math per pixel
        assert np.array_equal(imgs[0], p_img[0])
        assert np.allclose(par, p_par, rtol=1e-3, atol=1e-4)
        assert st[0] == pytest.approx(p_st[0], rel=1e-3)
    # the captured graph replays the batched kernel sequence, and no step
    # kernel depends on scheduling order: identical bits
    b_imgs, b_par, b_st = outs[sw.SWGS_MODE_BATCHED]
    g_imgs, g_par, g_st = outs[sw.SWGS_MODE_GRAPH]
    for a, b in zip(b_imgs, g_imgs):
        assert np.array_equal(a, b)
    assert np.array_equal(b_par, g_par) and np.array_equal(b_st, g_st)
    say("plain == batched params:", bool(np.array_equal(p_par, b_par)))


def test_window_step_end_to_end_loss_matches_oracle(sw, ctx):
    say("window step e2e")
    pool, views = tiny(n=1000)
    tgt_h = S.random_images(views, 9)
    dp, pl = plan_for(sw, ctx, pool, views)
    cfg = sw.step_cfg(mode=sw.SWGS_MODE_BATCHED, relocate_period=0)
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    pl.window_step(cfg, torch.as_tensor(tgt_h, device="cuda"), 1, 0, 3, stats=stats)
    st = host(stats)
    ref_img, _ = O.window_render(pool.params, 0, pool.start, pool.expire, views)
    A = O.window_set(pool.start, pool.expire, pool.num_gs, [0, 1, 2])
    L, l1, _, _ = O.loss_and_grad(ref_img, tgt_h, views, pool.params, A, lam_dssim=float(np.float32(cfg.lambda_dssim)))
    assert cfg.lambda_dssim == pytest.approx(0.2)
    assert st[0] == pytest.approx(l1, rel=1e-5)
    assert st[3] == pytest.approx(L, rel=1e-5)
    assert st[7] == A.sum()


@pytest.mark.parametrize("mode", ["batched", "plain", "graph"])
def test_dssim_term_and_image_gradient_match_oracle(sw, ctx, mode):
    """The D-SSIM image term (lambda 0.2) and the full dL/dC it leaves for the
    backward, on views of mixed and ragged sizes (down to smaller than the
    11x11 window; 100x75 has interior SSIM tiles whose halo reaches into
    neighbours on every side), in every launch structure."""
    say("dssim", mode)
    pool, _ = tiny(n=900)
    views = S.ring_views([0, 1], 3, 0, 0, sizes=[(64, 48), (37, 23), (100, 75)]) + S.ring_views([2], 1, 7, 5)
    tgt_h = S.random_images(views, 12)
    dp, pl = plan_for(sw, ctx, pool, views)
    m = {"batched": sw.SWGS_MODE_BATCHED, "plain": sw.SWGS_MODE_PLAIN, "graph": sw.SWGS_MODE_GRAPH}[mode]
    cfg = sw.step_cfg(mode=m, relocate_period=0)
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    img = pl.image_buffer()
    pl.window_step(cfg, torch.as_tensor(tgt_h, device="cuda"), 1, 0, 3, images=img, stats=stats)
    st = host(stats)
    dldc = host(pl.buffer(sw.SWGS_BUF_DLDC, torch.float32)).astype(np.float64)
    ref_img, _ = O.window_render(pool.params, 0, pool.start, pool.expire, views)
    lam = float(np.float32(cfg.lambda_dssim))
    A = O.window_set(pool.start, pool.expire, pool.num_gs, [0, 1, 2])
    L, part, g, _ = O.loss_and_grad(ref_img, tgt_h, views, pool.params, A, lam_dssim=lam)
    assert st[0] == pytest.approx(part, rel=1e-5)
    assert st[3] == pytest.approx(L, rel=1e-5)
    # element by element, per view: the whole dL/dC, and its D-SSIM part
    # alone (the kernel's total minus the oracle's L1 part), each within
    # 1e-3 relative with the 1e-2 * max floor of its view.  The L1 sign is
    # only defined away from zero residuals.
    clear = np.abs(ref_img - tgt_h) > 1e-4
    _, _, g1, _ = O.loss_and_grad(ref_img, tgt_h, views, pool.params, A)
    g_ssim = g - (1.0 - lam) * g1
    o = 0
    for v in views:
        n = 3 * v.width * v.height
        sl, c = slice(o, o + n), clear[o:o + n]
        ok = grad_close(dldc[sl][c], g[sl][c])
        assert ok.all(), (v.width, v.height, dldc[sl][c][~ok][:4], g[sl][c][~ok][:4])
        ok = grad_close((dldc[sl] - (1.0 - lam) * g1[sl])[c], g_ssim[sl][c])
        assert ok.all(), (v.width, v.height, "ssim part")
        o += n
    assert np.abs(g_ssim).max() > 0


def test_window_step_without_image_buffer_with_dssim(sw, ctx):
    """A window step given no image buffer renders into the workspace, where
    the D-SSIM term reads the images from: its loss matches the oracle's
    (a NULL image pointer once reached the D-SSIM kernel), in every launch
    structure."""
    say("window step images=None dssim")
    pool, views = tiny(n=1200)
    tgt_h = S.random_images(views, 13)
    ref_img, _ = O.window_render(pool.params, 0, pool.start, pool.expire, views)
    A = O.window_set(pool.start, pool.expire, pool.num_gs, [0, 1, 2])
    for mode in (sw.SWGS_MODE_BATCHED, sw.SWGS_MODE_PLAIN, sw.SWGS_MODE_GRAPH):
        dp, pl = plan_for(sw, ctx, pool, views)
        cfg = sw.step_cfg(mode=mode, relocate_period=0, lambda_dssim=0.2)
        stats = torch.zeros(8, dtype=torch.float64, device="cuda")
        pl.window_step(cfg, torch.as_tensor(tgt_h, device="cuda"), 1, 0, 3, images=None, stats=stats)
        st = host(stats)
        L, part, _, _ = O.loss_and_grad(ref_img, tgt_h, views, pool.params, A,
                                        lam_dssim=float(np.float32(cfg.lambda_dssim)))
        assert st[0] == pytest.approx(part, rel=1e-5), mode
        assert st[3] == pytest.approx(L, rel=1e-5), mode
        assert st[6] == 0
        pl.close()


def test_graph_replay_takes_each_calls_step_and_seed(sw, ctx):
    """A captured window step replays with the Adam t, step and seed of each
    call (resumed, rewound or re-seeded runs), bit-equal to the batched
    launches given the same numbers."""
    say("graph step numbers")
    pool, views = tiny(n=900)
    tgt = torch.as_tensor(S.random_images(views, 14), device="cuda")
    calls = [(1, 0, 5), (2, 1, 5), (7, 40, 5), (3, 2, 9), (3, 2, 9)]
    outs = []
    for mode in (sw.SWGS_MODE_BATCHED, sw.SWGS_MODE_GRAPH):
        dp, pl = plan_for(sw, ctx, pool, views)
        dp.params[10, :60] = -5.0          # faint Gaussians: noise gate open, some relocation
        cfg = sw.step_cfg(mode=mode, relocate_period=2)
        stats = torch.zeros(8, dtype=torch.float64, device="cuda")
        seq = []
        for (t, step, seed) in calls:
            pl.window_step(cfg, tgt, t, step, seed, stats=stats)
            seq.append((host(dp.params).copy(), host(stats).copy()))
        outs.append(seq)
        pl.close()
    for (pb, sb), (pg, sg) in zip(*outs):
        assert np.array_equal(pb, pg) and np.array_equal(sb, sg)


def test_stale_plan_is_flagged(sw, ctx):
    """A plan whose pool's lifespans changed after it was made (here by
    mature()) reports flag 2 in stats[6]; a fresh plan reports none."""
    say("stale plan flag")
    num_gs, swin, st = 250, 5, 8
    pool = S.steady_window_pool(num_gs, swin, 1, st, 2)
    views = S.ring_views(list(range(st, st + swin)), 2, 64, 48)
    dp = sw.Pool.from_synth(pool)
    pl = sw.Plan(ctx, dp, views)
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    pl.forward(stats=stats)
    assert host(stats)[6] == 0
    sw.mature(ctx, dp, st + 1)
    pl.forward(stats=stats)
    assert int(host(stats)[6]) & 2
    pl.close()
    pl2 = sw.Plan(ctx, dp, views)
    pl2.forward(stats=stats)
    assert host(stats)[6] == 0
    pl2.close()


def test_pair_capacity_overflow_is_reported(sw, ctx):
    say("overflow")
    pool, views = tiny(n=800)
    dp = sw.Pool.from_synth(pool)
    pl = sw.Plan(ctx, dp, views, pair_capacity=1000)
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    pl.forward(stats=stats)
    st = host(stats)
    assert st[6] == 1.0 and st[4] > 1000
    # the image term of an overflowed render contributes zero gradients
    # (the pairs past the capacity were never listed), never stale rows
    dp.grads.fill_(float("nan"))
    pl.backward(torch.ones(3 * pl.n_pixels, dtype=torch.float32, device="cuda"))
    g = dp.grads.cpu().numpy()
    written = ~np.isnan(g)
    assert written.any() and np.all(g[written] == 0.0)
    tgt = torch.as_tensor(S.random_images(views, 1), device="cuda")
    with pytest.raises(sw.SwgsError) as e:
        pl.window_step(sw.step_cfg(mode=sw.SWGS_MODE_PLAIN), tgt, 1, 0, 0)
    assert e.value.status == sw.SWGS_ERR_CAPACITY


def test_invalid_arguments_are_rejected(sw, ctx):
    say("invalid args")
    pool, views = tiny(n=100)
    dp = sw.Pool.from_synth(pool)
    pl = sw.Plan(ctx, dp, views)
    import ctypes
    with pytest.raises(sw.SwgsError) as e:
        with ctx:
            ctx.check(sw.swgs_render_forward(ctx.h, pl.h, sw.ptr(pl.ws), pl.ws_bytes - 256, None, None, None))
    assert e.value.status == sw.SWGS_ERR_WORKSPACE_TOO_SMALL
    dp.sh_degree = 4
    with pytest.raises(sw.SwgsError) as e:
        sw.Plan(ctx, dp, views)
    assert e.value.status == sw.SWGS_ERR_INVALID_ARG
    dp.sh_degree = 0
    with pytest.raises(sw.SwgsError) as e:
        sw.Plan(ctx, dp, views, tile=(4, 4))
    assert e.value.status == sw.SWGS_ERR_UNSUPPORTED
    with pytest.raises(sw.SwgsError) as e:
        pl.set_timing(4)
    assert e.value.status == sw.SWGS_ERR_INVALID_ARG
    # a view of 2^31 pixels or more (in-view pixel offsets are 32-bit) is
    # rejected before anything is allocated
    import copy
    big = copy.copy(views[0])
    big.width, big.height = 65536, 32768
    with pytest.raises(sw.SwgsError) as e:
        sw.Plan(ctx, dp, [big])
    assert e.value.status == sw.SWGS_ERR_INVALID_ARG


def test_counted_forward_matches_uncounted(sw, ctx):
    """The forward's counting build (timing flag COUNT) renders the same
    bits as the uncounted one; its blended-pair count matches the oracle's
    contributor counts (to 0.1%: a pixel whose skip/stop decision sits on a
    threshold may count differently in FP32 and FP64) and the evaluated
    count bounds it."""
    say("counted forward")
    pool, views = tiny(n=1500)
    dp, pl = plan_for(sw, ctx, pool, views)
    a = host(pl.forward()).copy()
    pl.set_timing(sw.SWGS_TIMING_COUNT)
    b = host(pl.forward()).copy()
    _, (ev_f, ev_b, n_bl) = pl.timing()
    pl.set_timing(0)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    P0 = pool.params.astype(np.float64)
    evals = blended = 0
    for v in views:
        vis, rec, rect = O.preprocess(P0, 0, pool.start, pool.expire, v, 16, 16)
        pix = np.arange(v.width * v.height)
        _, _, cnt, _, _ = O.render_records(vis, rec, v, pix)
        blended += int(cnt.sum())
    say("counts", ev_f, ev_b, n_bl, "oracle blended", blended)
    assert blended > 0 and abs(n_bl - blended) <= 1e-3 * blended and ev_f >= n_bl and ev_b == 0


def test_extreme_shapes_tile_invariant_and_match_oracle(sw, ctx):
    """Needle-like, huge and sub-pixel splats: the per-wave support test
    and the tile ranges must never drop a contribution."""
    say("extreme shapes")
    rng = np.random.default_rng(21)
    pool, views = tiny(n=400, width=90, height=70)
    p = pool.params
    k = np.arange(400)
    p[3, k % 4 == 0] = -0.5                          # needles: one long axis
    p[4:6, k % 4 == 0] = -6.5
    p[3:6, k % 4 == 1] = rng.uniform(-1.0, -0.3, size=(3, (k % 4 == 1).sum()))   # huge
    p[3:6, k % 4 == 2] = -7.5                        # far below a pixel
    p[10, k % 4 == 1] = -3.0                         # faint huge ones
    ref = None
    for tile in [(16, 16), (8, 8), (32, 8)]:
        img, T, _ = render_gpu(sw, ctx, pool, views, tile)
        if ref is None:
            ref = img
        else:
            assert np.array_equal(img.view(np.uint32), ref.view(np.uint32)), tile
    o = 0
    for v in views:
        n = v.width * v.height
        rgb, To, cnt, dm, cm = O.render_view(p, 0, pool.start, pool.expire, v)
        keep = dm >= MARGIN_PIX
        assert np.abs(ref[o:o + 3 * n].reshape(3, n) - rgb)[:, keep].max() <= IMG_TOL
        o += 3 * n

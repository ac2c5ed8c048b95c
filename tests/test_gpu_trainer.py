"""The paper's training loop (Algorithm 1) on the GPU.  train_swin: the
trainer equals, bit for bit, the single-view window steps it is made of
(each already checked against the oracle), iterating views sampled by the
published rule with Adam's t and the step following the global iteration,
relocation at its cadence; its first iteration's loss equals the oracle's.
schedule_expire equals the oracle's; Algorithm 1's main loop runs (genesis
window, schedule, one slice matured per frame)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2409_07759_amd import synth as S
from scenes import tiny

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


def test_trainer_equals_its_window_steps(sw, ctx):
    pool, views = tiny(n=1500, deg=1)
    tgts = [torch.as_tensor(S.random_images([v], 20 + i), device="cuda") for i, v in enumerate(views)]
    cfg = sw.step_cfg(mode=sw.SWGS_MODE_GRAPH, relocate_period=3, window_start=0)
    iters, iter0, seed = 10, 5, 11
    dp1 = sw.Pool.from_synth(pool)
    tr = sw.Trainer(ctx, dp1, views)
    stats1 = torch.zeros(8 * iters, dtype=torch.float64, device="cuda")
    order = tr.run(cfg, tgts, iters, iter0, seed, stats=stats1)
    tr.close()
    say("views", order.tolist())
    assert order.tolist() == [sw.trainer_view(seed, iter0 + i, len(views)) for i in range(iters)]
    assert len(set(order.tolist())) > 3
    dp2 = sw.Pool.from_synth(pool)
    plans = [sw.Plan(ctx, dp2, [v], pair_capacity=tr.pair_capacity) for v in views]
    cb = sw.step_cfg(mode=sw.SWGS_MODE_BATCHED, relocate_period=3, window_start=0)
    stats2 = torch.zeros(8 * iters, dtype=torch.float64, device="cuda")
    for i, v in enumerate(order.tolist()):
        it = iter0 + i
        plans[v].window_step(cb, tgts[v], it + 1, it, seed, stats=stats2[8 * i:8 * i + 8])
    for p in plans:
        p.close()
    for name in ("params", "adam_m", "adam_v", "start", "expire"):
        a, b = host(getattr(dp1, name)), host(getattr(dp2, name))
        assert np.array_equal(a.view(np.uint32) if a.dtype == np.float32 else a,
                              b.view(np.uint32) if b.dtype == np.float32 else b), name
    s1, s2 = host(stats1).reshape(iters, 8), host(stats2).reshape(iters, 8)
    assert np.array_equal(s1, s2)
    say("losses", s1[:, 3].round(5).tolist(), "relocated", s1[:, 5].tolist())
    # relocation only at iterations whose step is a multiple of the period
    assert all(s1[i, 5] == 0 for i in range(iters) if (iter0 + i) % 3)


def test_trainer_first_iteration_loss_matches_oracle(sw, ctx):
    pool, views = tiny(n=1200, deg=0)
    tg = [S.random_images([v], 40 + i) for i, v in enumerate(views)]
    dp = sw.Pool.from_synth(pool)
    tr = sw.Trainer(ctx, dp, views)
    cfg = sw.step_cfg(relocate_period=0)
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    order = tr.run(cfg, [torch.as_tensor(t, device="cuda") for t in tg], 1, 0, 3, stats=stats)
    tr.close()
    v = int(order[0])
    st = host(stats)
    ref_img, _ = O.window_render(pool.params, 0, pool.start, pool.expire, [views[v]])
    A = O.window_set(pool.start, pool.expire, pool.num_gs, [views[v].frame])
    L, img_term, _, _ = O.loss_and_grad(ref_img, tg[v], [views[v]], pool.params, A,
                                        lam_dssim=float(np.float32(cfg.lambda_dssim)))
    assert st[0] == pytest.approx(img_term, rel=1e-5)
    assert st[3] == pytest.approx(L, rel=1e-5)
    assert st[7] == A.sum()


@pytest.mark.parametrize("num_gs,swin", [(1000, 5), (1003, 4), (3, 5)])
def test_schedule_expire_matches_oracle(sw, ctx, num_gs, swin):
    b, s, e = O.genesis(num_gs, swin)
    P = np.zeros((14, 2 * num_gs), np.float32)
    dp = sw.Pool(P, b, s, e, num_gs, swin, 0, "cuda", train=False)
    sw.schedule_expire(ctx, dp)
    assert np.array_equal(host(dp.expire), O.schedule_expire(num_gs, swin, e.copy()))


def test_algorithm1_main_loop(sw, ctx):
    """Genesis window, schedule_expire, then mature + train one window per
    frame: the genesis record holds num_gs Gaussians, every later one a
    slice of num_gs / swin born at the previous frame."""
    num_gs, swin, deg, cams = 1000, 5, 1, 2
    P = S.make_gaussians(2 * num_gs, deg, 5)
    b, s, e = (np.zeros(2 * num_gs, np.int32) for _ in range(3))
    e[:num_gs] = swin                                # genesis: [0, swin)
    dp = sw.Pool(P, b, s, e, num_gs, swin, deg, "cuda")
    n_frames = 8
    allv = S.ring_views(list(range(n_frames + swin)), cams, 64, 48)
    tg = {(v.frame, k % cams): torch.as_tensor(S.random_images([v], 100 + k), device="cuda")
          for k, v in enumerate(allv)}
    cfg = sw.step_cfg(relocate_period=4)
    it = 0

    def train(st, n_it):
        nonlocal it
        vs = [v for v in allv if st <= v.frame < st + swin]
        tr = sw.Trainer(ctx, dp, vs)
        stats = torch.zeros(8 * n_it, dtype=torch.float64, device="cuda")
        tr.run(cfg, [tg[(v.frame, k % cams)] for k, v in enumerate(vs)], n_it, it, 9, stats=stats)
        tr.close()
        it += n_it
        return host(stats).reshape(n_it, 8)

    s0 = train(0, 20)
    assert np.all(np.isfinite(s0[:, 3]))
    sw.schedule_expire(ctx, dp)
    for st in range(1, 4):
        rec, cnt = sw.mature(ctx, dp, st)
        r = sw.parse_record(host(rec))
        if st == 1:
            assert cnt == num_gs and np.all(r["birth"] == 0)
        else:
            assert cnt == num_gs // swin and np.all(r["birth"] == st - 1)
        sx = train(st, 10)
        say("window", st, "loss", sx[:, 3].round(4).tolist())
        assert np.all(np.isfinite(sx[:, 3]))

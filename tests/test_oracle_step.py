"""Pins for the oracle optimiser step (Adam + adaptive mean-gradient scaling
+ SGLD noise, Algorithm 1 and Secs. 4.4-4.5.1) and relocation (Sec. 3.2,
Algorithm 1).  CPU only."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

import oracle as O
from paper_2409_07759_amd import synth as S


def rand_state(n, deg, seed):
    rng = np.random.default_rng(seed)
    p = S.make_gaussians(n, deg, seed).astype(np.float64)
    F = p.shape[0]
    g = rng.normal(0, 1e-3, size=(F, n))
    return p, g, np.zeros((F, n)), np.zeros((F, n))


def test_adam_equals_torch_adam_on_dense_active_set():
    n, deg = 50, 1
    p, g, m, v = rand_state(n, deg, 0)
    in_A = np.ones(n, bool)
    lrr = O.lr_rows(deg)
    groups = {}
    for r, lr in enumerate(lrr):
        groups.setdefault(lr, []).append(r)
    tp = [torch.nn.Parameter(torch.tensor(p[rows], dtype=torch.float64)) for rows in groups.values()]
    opt = torch.optim.Adam([{"params": [t], "lr": lr} for t, lr in zip(tp, groups.keys())],
                           betas=(0.9, 0.999), eps=1e-15)
    rng = np.random.default_rng(1)
    P = p
    for t in range(1, 4):
        gt = rng.normal(0, 1e-3, size=g.shape)
        P, m, v = O.adam_sgld_step(P, gt, m, v, in_A, t, deg, seed=0, step=t, noise_lr=0.0)
        for tt, rows in zip(tp, groups.values()):
            tt.grad = torch.tensor(gt[rows], dtype=torch.float64)
        opt.step()
    for tt, rows in zip(tp, groups.values()):
        assert np.allclose(P[rows], tt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_slots_outside_the_window_set_are_bit_unchanged():
    n, deg = 40, 0
    p, g, m, v = rand_state(n, deg, 2)
    in_A = np.arange(n) % 3 == 0
    P, M, V = O.adam_sgld_step(p, g, m, v, in_A, 1, deg, seed=5, step=1)
    assert np.array_equal(P[:, ~in_A], p[:, ~in_A])
    assert np.all(M[:, ~in_A] == 0) and np.all(V[:, ~in_A] == 0)
    assert np.all(P[:, in_A] != p[:, in_A])


def test_first_adam_step_moves_each_parameter_by_its_learning_rate():
    n, deg = 10, 0
    p, g, m, v = rand_state(n, deg, 3)
    P, _, _ = O.adam_sgld_step(p, g, m, v, np.ones(n, bool), 1, deg, 0, 1, noise_lr=0.0)
    lrr = O.lr_rows(deg)[:, None]
    assert np.allclose(P - p, -lrr * np.sign(g), rtol=1e-9)


def test_sgld_noise_isotropic_closed_form():
    """Isotropic scale s: Sigma = s^2 I, so the mean moves by
    noise_lr * lr_mean * sigmoid(-k (o - t0)) * s^2 * eta on top of Adam."""
    n, deg = 6, 0
    p, g, m, v = rand_state(n, deg, 4)
    s = np.array([0.01, 0.02, 0.05, 0.1, 0.03, 0.2])
    p[3:6] = np.log(s)[None, :]
    p[10] = [-6.0, -5.3, -4.0, 0.0, 2.0, -5.2933]
    g[:] = 0.0                               # Adam moves nothing
    eta = np.random.default_rng(0).normal(size=(3, n))
    P, _, _ = O.adam_sgld_step(p, g, m, v, np.ones(n, bool), 1, deg, 0, 1, eta=eta)
    o = 1 / (1 + np.exp(-p[10]))
    gate = 1 / (1 + np.exp(100 * (o - 0.005)))
    expect = 5e4 * 1.6e-4 * gate * s * s
    assert np.allclose(P[0:3] - p[0:3], expect[None, :] * eta, rtol=1e-9, atol=1e-15)
    # at o = t0 the gate is exactly one half
    assert 1 / (1 + math.exp(100 * 0.0)) == 0.5


def test_noise_uses_the_anisotropic_covariance():
    n, deg = 3, 0
    p, g, m, v = rand_state(n, deg, 6)
    g[:] = 0
    p[10] = -8.0
    eta = np.random.default_rng(2).normal(size=(3, n))
    P, _, _ = O.adam_sgld_step(p, g, m, v, np.ones(n, bool), 1, deg, 0, 1, eta=eta)
    o = 1 / (1 + np.exp(-p[10]))
    coef = 5e4 * 1.6e-4 / (1 + np.exp(100 * (o - 0.005)))
    for i in range(n):
        q = p[6:10, i] / np.linalg.norm(p[6:10, i])
        from scipy.spatial.transform import Rotation
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Sig = R @ np.diag(np.exp(2 * p[3:6, i])) @ R.T
        assert np.allclose(P[0:3, i] - p[0:3, i], coef[i] * Sig @ eta[:, i], rtol=1e-10)


def test_adaptive_gradient_scaling_of_the_mean():
    n, deg, swin, st = 8, 0, 4, 10
    p, g, m, v = rand_state(n, deg, 7)
    start = np.array([10, 11, 12, 13, 10, 11, 12, 13], np.int32)
    P, M, V = O.adam_sgld_step(p, g, m, v, np.ones(n, bool), 1, deg, 0, 1, noise_lr=0.0,
                               grad_scale_base=0.1, window_start=st, swin=swin, start=start)
    w = np.clip(st - start + swin - 1, 0, swin - 1)          # 3, 2, 1, 0, ...
    assert w.tolist() == [3, 2, 1, 0, 3, 2, 1, 0]
    assert np.allclose(M[0:3], 0.1 * g[0:3] * 0.1 ** (w / swin)[None, :], rtol=1e-12)
    assert np.allclose(M[3:], 0.1 * g[3:], rtol=1e-12)       # other rows unscaled


# ------------------------------------------------------------ relocation

@pytest.mark.parametrize("N", [1, 2, 3, 5, 8, 16, 32])
def test_SN_double_sum_equals_its_integral_form(N):
    for a in [0.005, 0.01, 0.1, 0.3, 0.5, 0.7, 0.9, 0.99]:
        I, _ = integrate.quad(lambda u: 1 - (1 - a * math.exp(-u * u)) ** N, 0, np.inf,
                              epsabs=1e-14, epsrel=1e-13, limit=200)
        # the alternating double sum loses ~C(N, N/2) ulps to cancellation
        assert O.reloc_SN(N, a) == pytest.approx(2 / math.sqrt(math.pi) * I, rel=1e-9 if N <= 16 else 1e-7)


def test_SN_of_one_copy_is_the_opacity():
    for a in [0.01, 0.4, 0.95]:
        assert O.reloc_SN(1, a) == pytest.approx(a, rel=1e-15)


def pool_for_reloc(n, seed, dead_frac=0.3):
    rng = np.random.default_rng(seed)
    p = S.make_gaussians(n, 0, seed).astype(np.float64)
    dead = rng.uniform(size=n) < dead_frac
    p[10, dead] = rng.uniform(-12, -5.4, size=dead.sum())
    p[10, ~dead] = rng.uniform(-5.0, 4.0, size=(~dead).sum())
    F = p.shape[0]
    return p, rng.normal(size=(F, n)), rng.uniform(size=(F, n))


def brute_force_sources(p, in_A, seed, step):
    """Independent re-statement of the sampler in plain Python integers."""
    Ls = float(np.float32(math.log(0.005 / 0.995)))
    alive, wts, dead = [], [], []
    for i in range(len(in_A)):
        if not in_A[i]:
            continue
        if p[10, i] < Ls:
            dead.append(i)
        else:
            alive.append(i)
            wts.append(math.floor(16777216.0 / (1.0 + math.exp(-p[10, i]))))
    W = sum(wts)
    out = []
    for j in range(len(dead)):
        x = O.philox4x32_10([j, step & 0xFFFFFFFF, step >> 32, 0x52454C4F], [seed & 0xFFFFFFFF, seed >> 32])
        r = int(x[0]) | (int(x[1]) << 32)
        u = (r * W) >> 64
        acc = 0
        for a, w in zip(alive, wts):
            acc += w
            if acc > u:
                out.append(a)
                break
    return dead, out


def test_relocation_indices_equal_brute_force():
    n = 300
    p, m, v = pool_for_reloc(n, 0)
    in_A = np.random.default_rng(1).uniform(size=n) < 0.8
    P, M, V, dst, src, _ = O.relocate(p, m, v, in_A, seed=77, step=(5 << 32) + 3)
    d, s = brute_force_sources(p, in_A, 77, (5 << 32) + 3)
    assert dst.tolist() == d and src.tolist() == s
    assert len(d) > 20


def test_relocation_draws_follow_the_weights():
    """Chi-square of 200k draws against the opacity weights."""
    n = 12
    p = np.zeros((14, n))
    p[10] = [-8.0, 0.0, 1.0, -1.0, 2.0, -7.0, 0.5, -2.0, 3.0, -0.5, 1.5, -3.0]
    Ls = float(np.float32(math.log(0.005 / 0.995)))
    alive = np.nonzero(p[10] >= Ls)[0]
    w = np.floor(2 ** 24 / (1 + np.exp(-p[10, alive])))
    counts = np.zeros(n)
    # many dead slots in one call -> many draws
    big = np.zeros((14, n + 200000))
    big[:, :n] = p
    big[10, n:] = -9.0
    mm = np.zeros((14, n + 200000))
    _, _, _, dst, src, _ = O.relocate(big, mm, mm.copy(), np.ones(n + 200000, bool), 3, 9)
    src = src[dst >= n]
    counts = np.bincount(src, minlength=n)[alive]
    expect = w / w.sum() * src.size
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2 < 40.0        # 9 dof; p ~ 1e-5


def test_relocated_parameters_closed_form_two_copies():
    """One dead, one alive slot: N = 2, o' = 1 - sqrt(1 - o), scale' = scale o / S_2(o')
    with S_2(a) = 2a - a^2/sqrt(2); mean, rotation and colour copied; Adam reset."""
    p = S.make_gaussians(2, 0, 4).astype(np.float64)
    p[10] = [-9.0, 0.7]
    m = np.ones((14, 2))
    v = np.ones((14, 2))
    P, M, V, dst, src, _ = O.relocate(p, m, v, np.ones(2, bool), 1, 1)
    assert dst.tolist() == [0] and src.tolist() == [1]
    o = 1 / (1 + math.exp(-0.7))
    on = 1 - math.sqrt(1 - o)
    s2 = 2 * on - on * on / math.sqrt(2)
    for i in (0, 1):
        assert 1 / (1 + math.exp(-P[10, i])) == pytest.approx(on, rel=1e-12)
        assert np.allclose(np.exp(P[3:6, i]), np.exp(p[3:6, 1]) * o / s2, rtol=1e-12)
        assert np.allclose(P[[0, 1, 2, 6, 7, 8, 9, 11, 12, 13], i], p[[0, 1, 2, 6, 7, 8, 9, 11, 12, 13], 1])
    assert np.all(M == 0) and np.all(V == 0)
    # total opacity of the two copies reproduces the source: 1-(1-o')^2 = o
    assert 1 - (1 - on) ** 2 == pytest.approx(o, rel=1e-12)


def test_copy_count_is_capped():
    n = 50
    p = np.zeros((14, n))
    p[10] = -9.0
    p[10, 7] = 1.0               # the only alive slot: 49 copies, N capped at 32
    P, _, _, dst, src, _ = O.relocate(p, np.zeros((14, n)), np.zeros((14, n)), np.ones(n, bool), 1, 1, n_max=32)
    assert np.all(src == 7) and len(dst) == 49
    o = 1 / (1 + math.exp(-1.0))
    on = 1 - (1 - o) ** (1 / 32)
    assert 1 / (1 + math.exp(-P[10, 7])) == pytest.approx(on, rel=1e-12)


def test_dead_threshold_is_strict_in_fp32_logit_space():
    Ls = np.float32(math.log(0.005 / 0.995))
    below = np.nextafter(Ls, np.float32(-np.inf))
    p = np.zeros((14, 3))
    p[10] = [float(Ls), float(below), 2.0]
    _, _, _, dst, src, _ = O.relocate(p, np.zeros((14, 3)), np.zeros((14, 3)), np.ones(3, bool), 0, 0)
    assert dst.tolist() == [1]


def test_relocation_noops():
    p = np.zeros((14, 4))
    p[10] = [1.0, 2.0, 3.0, 4.0]
    r = O.relocate(p, np.zeros((14, 4)), np.zeros((14, 4)), np.ones(4, bool), 0, 0)
    assert len(r[3]) == 0 and np.array_equal(r[0], p)
    p[10] = -9.0
    r = O.relocate(p, np.zeros((14, 4)), np.zeros((14, 4)), np.ones(4, bool), 0, 0)
    assert len(r[3]) == 0 and np.array_equal(r[0], p)

"""Pins of the oracle's SSIM / D-SSIM loss term (image term of the loss
after 3DGS-MCMC's practice, Sec. 4.4; SSIM per Wang et al. 2004 with an
11x11, sigma 1.5 Gaussian window, C1 = 0.01^2, C2 = 0.03^2).  CPU only."""
import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from paper_2409_07759_amd import synth as S


def test_window_is_the_normalised_separable_gaussian():
    w = O.ssim_window()
    assert w.shape == (11, 11)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1])
    # ratio of neighbouring taps of the 1D profile: exp((2k+1) / (2 sigma^2))
    g = w[5] / w[5, 5]
    assert np.isclose(g[5] / g[6], np.exp(1.0 / (2 * 1.5 ** 2)))
    assert np.isclose(g[6] / g[7], np.exp(3.0 / (2 * 1.5 ** 2)))
    assert np.linalg.matrix_rank(w) == 1


def test_window_sum_is_zero_padded_correlation():
    rng = np.random.default_rng(0)
    img = rng.uniform(size=(13, 17))
    w = O.ssim_window()
    ref = ndimage.correlate(img, w, mode="constant", cval=0.0)
    assert np.allclose(O.window_sum(img, w), ref, atol=1e-14)


def test_window_sum_adjoint_is_the_adjoint():
    rng = np.random.default_rng(1)
    w = O.ssim_window()
    a, b = rng.normal(size=(9, 14)), rng.normal(size=(9, 14))
    # <window_sum(a), b> = <a, window_sum_adjoint(b)>
    assert np.isclose((O.window_sum(a, w) * b).sum(), (a * O.window_sum_adjoint(b, w)).sum(), rtol=1e-13)


def test_ssim_of_an_image_with_itself_is_one_with_zero_gradient():
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(3, 12, 15))
    s, g = O.ssim(x, x)
    assert abs(s - 1.0) < 1e-12
    assert np.abs(g).max() < 1e-12


def test_ssim_is_symmetric():
    rng = np.random.default_rng(3)
    x, y = rng.uniform(size=(3, 10, 11)), rng.uniform(size=(3, 10, 11))
    assert np.isclose(O.ssim(x, y)[0], O.ssim(y, x)[0], rtol=1e-13)


def test_constant_images_have_the_closed_form_in_the_interior():
    """With no variance the contrast/structure factor is C2 / C2 = 1 and the
    map reduces to the luminance term (2ab + C1) / (a^2 + b^2 + C1) wherever
    the window lies inside the image."""
    a, b = 0.3, 0.7
    S_map, *_ = O.ssim_map(np.full((20, 24), a), np.full((20, 24), b))
    ref = (2 * a * b + O.SSIM_C1) / (a * a + b * b + O.SSIM_C1)
    assert np.allclose(S_map[5:-5, 5:-5], ref, rtol=1e-12)
    assert O.SSIM_C1 == 1e-4 and abs(O.SSIM_C2 - 9e-4) < 1e-18
    # near the border the zero padding pulls the means down: not the closed form
    assert not np.isclose(S_map[0, 0], ref)


def test_ssim_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    x, y = rng.uniform(size=(3, 9, 12)), rng.uniform(size=(3, 9, 12))
    _, g = O.ssim(x, y)
    eps = 1e-6
    for _ in range(12):
        c, i, j = rng.integers(3), rng.integers(9), rng.integers(12)
        xp, xm = x.copy(), x.copy()
        xp[c, i, j] += eps
        xm[c, i, j] -= eps
        fd = (O.ssim(xp, y)[0] - O.ssim(xm, y)[0]) / (2 * eps)
        assert np.isclose(g[c, i, j], fd, rtol=1e-6, atol=1e-11), (c, i, j, g[c, i, j], fd)


def test_loss_with_dssim_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    views = S.ring_views([0, 1], 1, 10, 7)
    n = sum(3 * v.width * v.height for v in views)
    img, tgt = rng.uniform(size=n), rng.uniform(size=n)
    A = np.zeros(4, bool)
    params = S.make_gaussians(4, 0, 0)
    L, part, g, _ = O.loss_and_grad(img, tgt, views, params, A, lam_dssim=0.2)
    # image part: 0.8 L1 + 0.2 (1 - SSIM), averaged over the views
    o, ref = 0, 0.0
    for v in views:
        k = 3 * v.width * v.height
        sv, _ = O.ssim(img[o:o + k].reshape(3, v.height, v.width), tgt[o:o + k].reshape(3, v.height, v.width))
        ref += (0.8 * np.abs(img[o:o + k] - tgt[o:o + k]).mean() + 0.2 * (1 - sv)) / len(views)
        o += k
    assert np.isclose(part, ref, rtol=1e-13)
    eps = 1e-7
    for idx in rng.choice(n, size=10, replace=False):
        if abs(img[idx] - tgt[idx]) < 10 * eps:
            continue
        ip, im = img.copy(), img.copy()
        ip[idx] += eps
        im[idx] -= eps
        fd = (O.loss_and_grad(ip, tgt, views, params, A, lam_dssim=0.2)[0] -
              O.loss_and_grad(im, tgt, views, params, A, lam_dssim=0.2)[0]) / (2 * eps)
        assert np.isclose(g[idx], fd, rtol=1e-5, atol=1e-10), (idx, g[idx], fd)


def test_dssim_off_is_the_l1_loss():
    rng = np.random.default_rng(6)
    views = S.ring_views([0], 1, 6, 5)
    n = 3 * 6 * 5
    img, tgt = rng.uniform(size=n), rng.uniform(size=n)
    A = np.zeros(2, bool)
    params = S.make_gaussians(2, 0, 0)
    L0, p0, g0, _ = O.loss_and_grad(img, tgt, views, params, A)
    assert np.isclose(p0, np.abs(img - tgt).mean(), rtol=1e-14)
    assert np.array_equal(g0, np.sign(img - tgt) / n)

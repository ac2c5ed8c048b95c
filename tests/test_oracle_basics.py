"""Pins for the oracle's building blocks: the counter-based generator, the
spherical-harmonic basis and the lifespan gate.  CPU only."""
import math

import numpy as np
import pytest
from scipy import special

import oracle as O


# --- Philox4x32-10: known-answer vectors published with the generator
# (Salmon et al., SC'11, Random123 distribution), stored with their source.
def _kat():
    path = __file__.replace("test_oracle_basics.py", "golden/philox4x32_10_kat.txt")
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_philox_known_answers(ctr, key, expect):
    assert list(O.philox4x32_10(ctr, key)) == expect


def test_box_muller_normals_are_standard():
    eta = O.normals(seed=123, step=7, slots=range(20000))
    # mean 0 and variance 1 within 5 standard errors, and no correlation
    for row in eta:
        assert abs(row.mean()) < 5 / math.sqrt(row.size)
        assert abs(row.var() - 1.0) < 5 * math.sqrt(2.0 / row.size)
    c = np.corrcoef(eta)
    assert np.all(np.abs(c - np.eye(3)) < 5 / math.sqrt(eta.shape[1]))


def test_normals_depend_on_seed_step_and_slot():
    a = O.normals(1, 0, [0, 1])
    assert not np.allclose(a, O.normals(2, 0, [0, 1]))
    assert not np.allclose(a, O.normals(1, 1, [0, 1]))
    assert not np.allclose(a[:, 0], a[:, 1])


# --- spherical harmonics
def _sphere_quadrature(n=48):
    x, w = np.polynomial.legendre.leggauss(n)      # cos(theta)
    phi = (np.arange(2 * n) + 0.5) * (2 * np.pi / (2 * n))
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wt = (w[:, None] * np.full(phi.shape, 2 * np.pi / (2 * n))[None, :]).reshape(-1)
    return dirs, wt


def test_sh_basis_is_orthonormal():
    dirs, wt = _sphere_quadrature()
    Y = np.stack([O.sh_basis(3, d)[0] for d in dirs])
    G = (Y * wt[:, None]).T @ Y
    assert np.allclose(G, np.eye(16), atol=1e-12)


def test_sh_dc_constant():
    # Y_00 = 1/(2 sqrt(pi)) = 0.28209479177387814...
    assert O.sh_basis(0, [0, 0, 1])[0][0] == pytest.approx(0.28209479177387814, rel=1e-15)


def _real_sh(l, m, d):
    """Real SH from scipy's complex ones (theta polar from +z, phi azimuth)."""
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    if hasattr(special, "sph_harm_y"):
        Yc = lambda mm: special.sph_harm_y(l, mm, theta, phi)
    else:
        Yc = lambda mm: special.sph_harm(mm, l, phi, theta)
    if m == 0:
        return Yc(0).real
    if m > 0:
        return math.sqrt(2) * (-1) ** m * Yc(m).real
    return math.sqrt(2) * (-1) ** m * Yc(-m).imag


def test_sh_basis_matches_library_up_to_the_3dgs_signs():
    rng = np.random.default_rng(0)
    dirs = rng.normal(size=(20, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    # index k <-> (l, m) with k = l^2 + l + m; the renderer's basis is the
    # library's real SH (with the Condon-Shortley phase) times (-1)^m
    for k in range(16):
        l = int(math.isqrt(k))
        m = k - l * l - l
        ours = np.array([O.sh_basis(3, d)[0][k] for d in dirs])
        ref = np.array([_real_sh(l, m, d) for d in dirs])
        s = np.sign(np.dot(ours, ref))
        assert np.allclose(ours, s * ref, atol=1e-12), k
        # the fixed sign convention: degree-1 terms are -y, +z, -x etc.
        assert s == (-1) ** (m % 2), k
    d = np.array([0.0, 1.0, 0.0])
    Y = O.sh_basis(1, d)[0]
    assert Y[1] < 0 and Y[2] == 0 and Y[3] == 0      # -C1 y
    d = np.array([1.0, 0.0, 0.0])
    Y = O.sh_basis(1, d)[0]
    assert Y[3] < 0                                  # -C1 x
    d = np.array([0.0, 0.0, 1.0])
    assert O.sh_basis(1, d)[0][2] > 0                # +C1 z


def test_sh_gradient_by_central_differences():
    rng = np.random.default_rng(1)
    for _ in range(10):
        d = rng.normal(size=3)
        Y, dY = O.sh_basis(3, d)
        h = 1e-6
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            fd = (O.sh_basis(3, d + e)[0] - O.sh_basis(3, d - e)[0]) / (2 * h)
            assert np.allclose(dY[:, j], fd, atol=1e-8)


# --- lifespan gate (start <= frame < expire)
def test_active_gate_half_open():
    start = np.array([0, 2, 2, 5])
    expire = np.array([1, 2, 4, 6])
    assert O.active(start, expire, 0).tolist() == [True, False, False, False]
    assert O.active(start, expire, 2).tolist() == [False, False, True, False]
    assert O.active(start, expire, 3).tolist() == [False, False, True, False]
    assert O.active(start, expire, 4).tolist() == [False, False, False, False]
    assert O.active(start, expire, 5).tolist() == [False, False, False, True]


def test_threaded_oracle_loops_agree_with_one_thread():
    """The OpenMP loops used by the CPU-baseline timing change nothing but
    the order of the adjoint's sums over pixels: preprocess and render are
    bit-identical, the record and parameter gradients agree to rounding."""
    import oracle as O
    from paper_2409_07759_amd import synth as S
    params = S.make_gaussians(1500, 1, 4)
    birth, start, expire = S.lifespans_tiny(1500, 4)
    v = S.ring_views([1], 2, 80, 60)[1]
    rng = np.random.default_rng(3)
    out = []
    for nt in (1, 4):
        O.set_threads(nt)
        try:
            vis, rec, rect = O.preprocess(params, 1, start, expire, v)
            rgb = O.render_records(vis, rec, v)[0]
            dl = rng.uniform(-1, 1, size=(3, v.width * v.height)) if nt == 1 else dl
            drec = O.blend_backward(vis, rec, v, dl)
            gp = O.preprocess_backward_visible(params, 1, v, drec, vis, 1500)
        finally:
            O.set_threads(1)
        out.append((vis, rec, rect, rgb, drec, gp))
    a, b = out
    for k in range(4):
        assert np.array_equal(a[k], b[k])
    assert np.allclose(a[4], b[4], rtol=1e-12, atol=1e-18) and np.abs(a[4]).max() > 0
    assert np.allclose(a[5], b[5], rtol=1e-11, atol=1e-16)
    # the C loop over visible slots equals the per-slot Python loop
    ref = O.preprocess_backward(params, 1, v, a[4], np.nonzero(vis)[0])
    assert np.array_equal(a[5], ref)

"""Pins for the oracle renderer (Eqs. 1-3, Sec. 2.1): closed-form single
Gaussians, a hand-computed composite, a finite-difference Jacobian of the
pinhole map, invariants and lifespan gating.  CPU only."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle as O
from paper_2409_07759_amd import synth as S

Y00 = 0.5 / math.sqrt(math.pi)


def one_view(W, H, frame=0):
    # camera at (0, 0, 4) looking at the origin: camera x = world x,
    # camera y = -world y, camera z = 4 - world z
    return S.ring_views([frame], 1, W, H)[0]


def scene(rows):
    """rows: list of dicts with mean, logscale(3), quat, logit, rgb."""
    n = len(rows)
    p = np.zeros((14, n), np.float64)
    for i, r in enumerate(rows):
        p[0:3, i] = r["mean"]
        p[3:6, i] = r["logscale"]
        p[6:10, i] = r.get("quat", (1, 0, 0, 0))
        p[10, i] = r["logit"]
        p[11:14, i] = (np.asarray(r["rgb"]) - 0.5) / Y00
    return p


def always(n):
    return np.zeros(n, np.int32), np.full(n, 10, np.int32)


def logit(o):
    return math.log(o / (1 - o))


def test_isotropic_gaussian_on_axis_closed_form():
    W, H = 64, 48
    v = one_view(W, H)
    s, o, c = 0.03, 0.8, (0.9, 0.4, 0.1)
    p = scene([dict(mean=(0, 0, 0), logscale=[math.log(s)] * 3, logit=logit(o), rgb=c)])
    st, ex = always(1)
    rgb, T, n, dm, _ = O.render_view(p, 0, st, ex, v)
    sig2 = (v.fx * s / 4.0) ** 2 + 0.3
    xs = np.arange(W) + 0.5 - v.cx
    ys = np.arange(H) + 0.5 - v.cy
    r2 = ys[:, None] ** 2 + xs[None, :] ** 2
    a = np.minimum(0.99, o * np.exp(-r2 / (2 * sig2)))
    a[a < 1 / 255] = 0.0
    for ch in range(3):
        assert np.allclose(rgb[ch].reshape(H, W), c[ch] * a, atol=1e-13, rtol=0)
    assert np.allclose(T.reshape(H, W), 1 - a, atol=1e-13)
    assert n.reshape(H, W)[a == 0].max() == 0 and n.reshape(H, W)[a > 0].min() == 1


@pytest.mark.parametrize("phi", [0.0, 0.4, 1.3, -2.0])
def test_anisotropic_gaussian_rotated_about_view_axis(phi):
    W, H = 65, 49
    v = one_view(W, H)
    sx, sy, sz = 0.05, 0.015, 0.02
    o = 0.6
    q = (math.cos(phi / 2), 0.0, 0.0, math.sin(phi / 2))
    p = scene([dict(mean=(0, 0, 0), logscale=[math.log(sx), math.log(sy), math.log(sz)],
                    quat=q, logit=logit(o), rgb=(1.0, 0.5, 0.25))])
    st, ex = always(1)
    rgb, T, n, _, _ = O.render_view(p, 0, st, ex, v)
    # world x-y covariance of the ellipse, flipped to camera y (down)
    Rz = np.array([[math.cos(phi), -math.sin(phi)], [math.sin(phi), math.cos(phi)]])
    Sw = Rz @ np.diag([sx * sx, sy * sy]) @ Rz.T
    F = np.diag([1.0, -1.0])
    cov = (v.fx / 4.0) ** 2 * (F @ Sw @ F) + 0.3 * np.eye(2)
    inv = np.linalg.inv(cov)
    xs = np.arange(W) + 0.5 - v.cx
    ys = np.arange(H) + 0.5 - v.cy
    X, Y = np.meshgrid(xs, ys)
    Q = inv[0, 0] * X * X + 2 * inv[0, 1] * X * Y + inv[1, 1] * Y * Y
    a = np.minimum(0.99, o * np.exp(-0.5 * Q))
    a[a < 1 / 255] = 0.0
    assert np.allclose(rgb[0].reshape(H, W), a, atol=1e-12)
    assert np.allclose(rgb[2].reshape(H, W), 0.25 * a, atol=1e-12)


def test_projected_covariance_matches_numeric_jacobian():
    """Off-axis Gaussians: cov2 = J Sigma_cam J^T + 0.3 I with J the numeric
    Jacobian of the pinhole map (central differences) and the rotation built
    by scipy from the quaternion."""
    rng = np.random.default_rng(3)
    views = S.ring_views([0], 3, 128, 96)
    n = 40
    p = S.make_gaussians(n, 0, 5).astype(np.float64)
    p[0:3] *= 0.6
    st, ex = always(n)
    for v in views:
        vis, rec, _ = O.preprocess(p, 0, st, ex, v)
        for i in np.nonzero(vis)[0]:
            mu = p[0:3, i]
            pc = v.R @ mu + v.t
            lx, ly = 1.3 * 0.5 * v.width / v.fx, 1.3 * 0.5 * v.height / v.fy
            if abs(pc[0] / pc[2]) > lx or abs(pc[1] / pc[2]) > ly:
                continue

            def proj(x):
                return np.array([v.fx * x[0] / x[2] + v.cx, v.fy * x[1] / x[2] + v.cy])

            h = 1e-6
            J = np.stack([(proj(pc + h * e) - proj(pc - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
            w, x, y, z = p[6:10, i]
            Rq = Rotation.from_quat([x, y, z, w]).as_matrix()
            Sig = Rq @ np.diag(np.exp(2 * p[3:6, i])) @ Rq.T
            cov = J @ (v.R @ Sig @ v.R.T) @ J.T + 0.3 * np.eye(2)
            got = rec[i, O.R_COV:O.R_COV + 3]
            assert np.allclose(got, [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-7, atol=1e-9)
            inv = np.linalg.inv(cov)
            assert np.allclose(rec[i, [O.R_A, O.R_B, O.R_C]], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-7)
            assert np.allclose(rec[i, [O.R_U, O.R_V]], proj(pc), rtol=1e-12)
            assert rec[i, O.R_DEPTH] == np.float32(pc[2])


def test_eq3_three_stacked_gaussians_in_depth_order():
    W, H = 65, 49
    v = one_view(W, H)
    v.bg = (0.1, 0.2, 0.3)
    # slots in non-depth order: world z 0.5, 1.5, 1.0 -> depths 3.5, 2.5, 3.0
    cols = [(0.9, 0.1, 0.1), (0.1, 0.9, 0.1), (0.1, 0.1, 0.9)]
    ops = [0.5, 0.3, 0.6]
    p = scene([dict(mean=(0, 0, z), logscale=[math.log(0.02)] * 3, logit=logit(o), rgb=c)
               for z, o, c in zip([0.5, 1.5, 1.0], ops, cols)])
    st, ex = always(3)
    pix = [24 * W + 32]   # centre at (32.5, 24.5) = principal point
    rgb, T, n, _, _ = O.render_view(p, 0, st, ex, v, pixels=pix)
    order = [1, 2, 0]
    Tacc, C = 1.0, np.zeros(3)
    for i in order:
        C += np.asarray(cols[i]) * ops[i] * Tacc
        Tacc *= 1 - ops[i]
    C += Tacc * np.asarray(v.bg)
    assert np.allclose(rgb[:, 0], C, atol=1e-14)
    assert T[0] == pytest.approx(Tacc, abs=1e-15) and n[0] == 3


def test_early_stop_and_clamp():
    W, H = 65, 49
    v = one_view(W, H)
    # alphas 0.98, clamp(0.995) = 0.99, 0.9: T 1 -> 0.02 -> 2e-4 (blended)
    # -> 2e-5 < 1e-4, so the third Gaussian is not blended
    ops = [0.98, 0.995, 0.9]
    cols = [(0.2, 0.2, 0.2), (0.6, 0.6, 0.6), (1.0, 1.0, 1.0)]
    p = scene([dict(mean=(0, 0, z), logscale=[math.log(0.02)] * 3, logit=logit(o), rgb=c)
               for z, o, c in zip([1.5, 1.0, 0.5], ops, cols)])
    st, ex = always(3)
    rgb, T, n, _, _ = O.render_view(p, 0, st, ex, v, pixels=[24 * W + 32])
    exp = 0.2 * 0.98 + 0.6 * 0.99 * 0.02
    assert rgb[0, 0] == pytest.approx(exp, abs=1e-14)
    assert T[0] == pytest.approx(0.02 * 0.01, rel=1e-12) and n[0] == 2


def test_faint_gaussian_is_skipped_entirely():
    W, H = 65, 49
    v = one_view(W, H)
    p = scene([dict(mean=(0, 0, 0.5), logscale=[math.log(0.02)] * 3, logit=logit(0.5), rgb=(1, 1, 1)),
               dict(mean=(0, 0, 0.0), logscale=[math.log(0.02)] * 3, logit=logit(0.5), rgb=(0, 1, 0))])
    st, ex = always(2)
    # pixel where the first Gaussian's alpha is just below 1/255
    sig2 = (v.fx * 0.02 / 3.5) ** 2 + 0.3
    r = math.sqrt(2 * sig2 * math.log(0.5 * 255)) + 0.3
    px = int(v.cx + r)
    rgb, T, n, _, _ = O.render_view(p, 0, st, ex, v, pixels=[24 * W + px])
    d0 = px + 0.5 - v.cx
    a1 = 0.5 * math.exp(-d0 * d0 / (2 * sig2))
    assert a1 < 1 / 255
    sig2b = (v.fx * 0.02 / 4.0) ** 2 + 0.3
    a2 = 0.5 * math.exp(-d0 * d0 / (2 * sig2b))
    expect_g = a2 if a2 >= 1 / 255 else 0.0
    assert rgb[1, 0] == pytest.approx(expect_g, abs=1e-14) and rgb[0, 0] == 0.0


def tiny_scene(seed=0):
    p = S.make_gaussians(2000, 0, seed).astype(np.float64)
    _, st, ex = S.lifespans_tiny(2000, seed)
    views = S.ring_views([0, 1, 2], 3, 128, 96)
    return p, st, ex, views


def test_invariants_on_tiny_window():
    p, st, ex, views = tiny_scene()
    for v in views[::4]:
        v.bg = (0.3, 0.0, 1.0)
        rgb, T, n, dm, _ = O.render_view(p, 0, st, ex, v)
        vis, rec, _ = O.preprocess(p, 0, st, ex, v)
        mx = rec[vis == 1][:, O.R_RGB:O.R_RGB + 3].max()
        assert T.min() >= 1e-4 and T.max() <= 1.0
        assert rgb.min() >= 0.0
        for ch in range(3):
            assert np.all(rgb[ch] <= mx * (1 - T) + T * v.bg[ch] + 1e-12)


def test_inactive_gaussians_contribute_exactly_nothing():
    p, st, ex, views = tiny_scene()
    v = views[4]                  # frame 1
    rgb0, T0, *_ = O.render_view(p, 0, st, ex, v)
    off = ~O.active(st, ex, v.frame)
    p2 = p.copy()
    rng = np.random.default_rng(9)
    p2[:, off] = rng.normal(size=(p.shape[0], off.sum()))
    st2, ex2 = st.copy(), ex.copy()
    # move out-of-frame lifespans elsewhere, still excluding this frame
    st2[off] = np.where(ex[off] <= v.frame, st[off] - 5, st[off] + 7)
    ex2[off] = st2[off] + 1
    rgb1, T1, *_ = O.render_view(p2, 0, st2, ex2, v)
    assert np.array_equal(rgb0, rgb1) and np.array_equal(T0, T1)


@pytest.mark.parametrize("tw,th", [(8, 8), (16, 16), (32, 8)])
def test_tile_lists_cover_every_contributing_pair(tw, th):
    """Every (pixel, Gaussian) with alpha >= 1/255 lies in a tile of the
    Gaussian's tile range, so tiling never drops a contribution."""
    p, st, ex, views = tiny_scene()
    v = views[2]
    vis, rec, rect = O.preprocess(p, 0, st, ex, v, tw, th)
    W, H = v.width, v.height
    X, Y = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    tx, ty = (X // tw).astype(int), (Y // th).astype(int)
    # also the slots that preprocess at another tile size calls visible
    for i in np.nonzero(vis)[0]:
        r = rec[i]
        dx, dy = X - r[O.R_U], Y - r[O.R_V]
        Q = r[O.R_A] * dx * dx + 2 * r[O.R_B] * dx * dy + r[O.R_C] * dy * dy
        a = np.minimum(0.99, r[O.R_OPA] * np.exp(-0.5 * Q))
        hit = a >= 1 / 255
        x0, y0, x1, y1 = rect[i]
        inside = (tx >= x0) & (tx < x1) & (ty >= y0) & (ty < y1)
        assert np.all(inside[hit])
    # invisible slots that pass the gate have no pixel with alpha >= 1/255
    act = O.active(st, ex, v.frame)
    for i in np.nonzero(act & (vis == 0))[0][:200]:
        sub = O.preprocess(p[:, i:i + 1], 0, st[i:i + 1], ex[i:i + 1], v, 1, 1)
        assert sub[0][0] == 0


def test_tile_pairs_are_sorted_by_tile_depth_slot():
    p, st, ex, views = tiny_scene()
    v = views[0]
    vis, rec, rect = O.preprocess(p, 0, st, ex, v, 16, 16)
    tiles, slots, ranges = O.tile_pairs(vis, rec, rect, v, 16, 16)
    keys = [(int(t), float(np.float32(rec[s, O.R_DEPTH])), int(s)) for t, s in zip(tiles, slots)]
    assert keys == sorted(keys)
    counts = ((rect[:, 2] - rect[:, 0]) * (rect[:, 3] - rect[:, 1]))[vis == 1]
    assert len(tiles) == counts.sum()
    assert ranges[-1, 1] == len(tiles) and np.all(ranges[:, 0] <= ranges[:, 1])


@pytest.mark.parametrize("tw,th", [(16, 16), (8, 8), (32, 8)])
def test_tile_rect_of_hand_placed_gaussians_closed_form(tw, th):
    """The support rectangle, pinned from both sides.  An isotropic Gaussian
    of scale s and opacity o at camera-space (x, 0, z) projects to
    u = f x / z + c_x with projected variances a = (f s / z)^2 (1 + (x/z)^2)
    + 0.3 along the image x axis and c = (f s / z)^2 + 0.3 along y.  Its
    support {alpha >= 1/255} has half-extents h_x = sqrt(2 ln(255 o) a),
    h_y = sqrt(2 ln(255 o) c); the rect covers tiles
    floor((u - h_x - 1) / T_w) .. floor((u + h_x + 1) / T_w) (one pixel of
    padding), clipped to the grid.  Two on-axis Gaussians (opacity 0.9 and
    0.01) are scaled to h = 15.5 px, so the padded edge crosses a tile
    boundary that the unpadded edge does not, and a 3-sigma extent (first)
    or an extent without the opacity term (second) lands in another tile;
    the third Gaussian's rect is clipped at the grid's left edge."""
    W, H = 256, 192
    v = one_view(W, H)
    z = 4.0                                   # the camera sits at world z = 4
    f = v.fx
    h = 15.5
    gs = []
    for (o, u_want) in ((0.9, v.cx), (0.01, v.cx), (0.9, 10.0)):
        kappa = 2.0 * math.log(255.0 * o)
        var = h * h / kappa                   # projected variance on the axis
        gs.append(dict(o=o, kappa=kappa, var=var, s=z * math.sqrt(var - 0.3) / f, x=(u_want - v.cx) * z / f))
    p = scene([dict(mean=(g["x"], 0, 0), logscale=[math.log(g["s"])] * 3, logit=logit(g["o"]), rgb=(0.5,) * 3)
               for g in gs])
    st, ex = always(len(gs))
    vis, rec, rect = O.preprocess(p, 0, st, ex, v, tw, th)
    assert (vis == 1).all()
    tx, ty = -(-W // tw), -(-H // th)
    for i, g in enumerate(gs):
        s, x = g["s"], g["x"]
        u = f * x / z + v.cx
        a = (f * s / z) ** 2 * (1.0 + (x / z) ** 2) + 0.3
        c = (f * s / z) ** 2 + 0.3
        hx, hy = math.sqrt(g["kappa"] * a), math.sqrt(g["kappa"] * c)
        want = (max(0, math.floor((u - hx - 1.0) / tw)), max(0, math.floor((v.cy - hy - 1.0) / th)),
                min(tx, math.floor((u + hx + 1.0) / tw) + 1), min(ty, math.floor((v.cy + hy + 1.0) / th) + 1))
        assert tuple(int(k) for k in rect[i]) == want, (i, rect[i], want)
        assert rec[i, O.R_U] == pytest.approx(u, abs=1e-9)
    assert rect[2, 0] == 0                    # clipped at the grid's left edge
    # the rect tells the exact extent from the plausible wrong ones
    if (tw, th) == (16, 16):
        right = lambda e: math.floor((v.cx + e) / tw) + 1
        assert int(rect[0, 2]) == int(rect[1, 2]) == right(h + 1.0) == 10 and int(rect[0, 0]) == 6
        assert right(h) != right(h + 1.0)                                         # no padding
        assert right(3.0 * math.sqrt(gs[0]["var"]) + 1.0) != right(h + 1.0)      # 3 sigma
        assert right(math.sqrt(2.0 * math.log(255.0) * gs[1]["var"]) + 1.0) != right(h + 1.0)  # no opacity term

"""FP64 CPU oracle for the SwinGS hot path (arXiv 2409.07759).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of bench.py, never by the product path.  It shares no code
with the HIP library.  Heavy per-pixel work lives in swgs_oracle.c (plain C,
FP64); the rest is plain numpy in FP64.  Each function names the passage of
the paper it follows; where the paper defers to prior 3DGS / 3DGS-MCMC work,
the reading taken is the one recorded in DESIGN.md ("readings").
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "swgs_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
REC = 16
R_U, R_V, R_A, R_B, R_C, R_OPA, R_RGB, R_DEPTH = 0, 1, 2, 3, 4, 5, 6, 9
R_COV, R_HX, R_HY, R_MARGIN = 10, 13, 14, 15

_lib = None


def build(force: bool = False) -> str:
    """Compile swgs_oracle.c with gcc into oracle/liborc.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"])
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u64 = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_sh_basis.argtypes = [i32, P, P, P]
        L.orc_preprocess.argtypes = [P, i64, i32, P, P, i32, P, i32, i32, i32, i32, P, P, P]
        L.orc_render.argtypes = [i64, P, P, i32, i32, P, i64, P, P, P, P, P, P]
        L.orc_blend_backward.argtypes = [i64, P, P, i32, i32, P, P, P]
        L.orc_blend_backward_pixels.argtypes = [i64, P, P, i32, i32, P, P, i64, P, P]
        L.orc_preprocess_backward_one.argtypes = [P, i64, i64, i32, P, i32, i32, P, P]
        L.orc_view_backward.argtypes = [P, i64, i32, P, P, i32, P, i32, i32, P, i64, P, P, P]
        L.orc_reloc_SN.argtypes = [i32, ctypes.c_double]
        L.orc_reloc_SN.restype = ctypes.c_double
        L.orc_relocate.argtypes = [i64, i64, i32, P, P, P, P, u64, u64, i32, P, P, P]
        L.orc_relocate.restype = i64
        L.orc_set_threads.argtypes = [i32]
        L.orc_get_threads.restype = i32
        L.orc_preprocess_backward_many.argtypes = [P, i64, i32, P, i32, i32, P, i64, P, P]
        L.orc_set_threads(1)
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ------------------------------------------------------------------ basics

def philox4x32_10(ctr, key):
    """Philox4x32-10 block (Salmon et al., SC'11) of a 4-word counter."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def sh_basis(deg: int, d):
    d = _f64(d)
    Y = np.zeros(16)
    dY = np.zeros(48)
    lib().orc_sh_basis(int(deg), _p(d), _p(Y), _p(dY))
    n = (deg + 1) ** 2
    return Y[:n], dY[:3 * n].reshape(n, 3)


def active(start, expire, frame):
    """Lifespan gate: start <= frame < expire (Sec. 4.2, Algorithm 1)."""
    return (np.asarray(start) <= frame) & (frame < np.asarray(expire))


# ------------------------------------------------------------ render path

def preprocess(params, sh_degree, start, expire, view, tw=16, th=16):
    """Per-slot screen-space records of one view (Eqs. 1-3, Sec. 2.1)."""
    P = _f64(params)
    S = P.shape[1]
    vis = np.zeros(S, np.int32)
    rec = np.zeros((S, REC))
    rect = np.zeros((S, 4), np.int32)
    cam = _f64(view.cam16())
    lib().orc_preprocess(_p(P), S, int(sh_degree), _p(_i32(start)), _p(_i32(expire)), int(view.frame),
                         _p(cam), int(view.width), int(view.height), int(tw), int(th),
                         _p(vis), _p(rec), _p(rect))
    return vis, rec, rect


def render_records(vis, rec, view, pixels=None):
    """Eq. 3 per pixel by brute force over all visible Gaussians in depth
    order.  Returns rgb [3, n], T_final [n], contributor count [n], decision
    margin [n] and clamp margin [n]; n = all pixels when pixels is None."""
    S = vis.shape[0]
    W, H = view.width, view.height
    bg = _f64(view.bg)
    if pixels is None:
        n = W * H
        pix_p = None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        n = pix.shape[0]
        pix_p = _p(pix)
    rgb = np.zeros((3, n))
    T = np.zeros(n)
    cnt = np.zeros(n, np.int32)
    dm = np.zeros(n)
    cm = np.zeros(n)
    lib().orc_render(S, _p(_i32(vis)), _p(_f64(rec)), W, H, _p(bg), n, pix_p,
                     _p(rgb), _p(T), _p(cnt), _p(dm), _p(cm))
    return rgb, T, cnt, dm, cm


def render_view(params, sh_degree, start, expire, view, pixels=None, tw=16, th=16):
    vis, rec, _ = preprocess(params, sh_degree, start, expire, view, tw, th)
    return render_records(vis, rec, view, pixels)


def tile_pairs(vis, rec, rect, view, tw, th):
    """Binning definition: every (tile, slot) with the tile inside the slot's
    tile range, ordered by tile, then FP32 depth ("close to far", Sec. 2.1),
    then slot.  Returns (tile_id, slot) int64 arrays and per-tile [first, last)
    ranges over ntiles = ceil(W/tw)*ceil(H/th)."""
    ntx = (view.width + tw - 1) // tw
    nty = (view.height + th - 1) // th
    tiles, slots, depth = [], [], []
    for i in np.nonzero(vis)[0]:
        x0, y0, x1, y1 = rect[i]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                tiles.append(ty * ntx + tx)
                slots.append(i)
                depth.append(np.float32(rec[i, R_DEPTH]))
    tiles = np.asarray(tiles, np.int64)
    slots = np.asarray(slots, np.int64)
    depth = np.asarray(depth, np.float32)
    order = np.lexsort((slots, depth, tiles))
    tiles, slots = tiles[order], slots[order]
    nt = ntx * nty
    first = np.searchsorted(tiles, np.arange(nt), side="left")
    last = np.searchsorted(tiles, np.arange(nt), side="right")
    return tiles, slots, np.stack([first, last], axis=1)


def blend_backward(vis, rec, view, dLdC):
    """Adjoint of Eq. 3 for one view: d/d(u, v, A, B, C, o, r, g, b) per slot."""
    S = vis.shape[0]
    drec = np.zeros((S, 9))
    lib().orc_blend_backward(S, _p(_i32(vis)), _p(_f64(rec)), view.width, view.height,
                             _p(_f64(view.bg)), _p(_f64(dLdC)), _p(drec))
    return drec


def blend_backward_pixels(vis, rec, view, pixels, dLdC):
    """Adjoint of Eq. 3 restricted to a pixel list; dLdC is [3, len(pixels)]."""
    S = vis.shape[0]
    drec = np.zeros((S, 9))
    pix = np.ascontiguousarray(pixels, dtype=np.int64)
    lib().orc_blend_backward_pixels(S, _p(_i32(vis)), _p(_f64(rec)), view.width, view.height,
                                    _p(_f64(view.bg)), _p(_f64(dLdC)), len(pix), _p(pix), _p(drec))
    return drec


def preprocess_backward(params, sh_degree, view, drec, slots):
    """Chain rule from record gradients to parameter gradients (planar rows)."""
    P = _f64(params)
    S = P.shape[1]
    out = np.zeros_like(P)
    cam = _f64(view.cam16())
    dr = _f64(drec)
    for i in slots:
        lib().orc_preprocess_backward_one(_p(P), S, int(i), int(sh_degree), _p(cam),
                                          view.width, view.height, _p(np.ascontiguousarray(dr[i])), _p(out))
    return out


def set_threads(n: int) -> None:
    """Threads of the oracle's per-slot and per-pixel loops (1 by default;
    the CPU-baseline timing uses all host cores)."""
    lib().orc_set_threads(int(n))


def preprocess_backward_visible(params, sh_degree, view, drec, visible, n_opt):
    """preprocess_backward over every visible slot below n_opt, in C."""
    P = _f64(params)
    S = P.shape[1]
    out = np.zeros_like(P)
    lib().orc_preprocess_backward_many(_p(P), S, int(sh_degree), _p(_f64(view.cam16())), view.width, view.height,
                                       _p(_i32(visible)), int(min(n_opt, S)), _p(_f64(drec)), _p(out))
    return out


def view_backward(params, sh_degree, start, expire, view, n_opt, dLdC):
    """d/dparams of sum(dLdC * image) for one view; frozen slots (>= n_opt)
    get none (Sec. 4.2: no gradient for matured Gaussians)."""
    P = _f64(params)
    S = P.shape[1]
    dparams = np.zeros_like(P)
    drec = np.zeros((S, 9))
    lib().orc_view_backward(_p(P), S, int(sh_degree), _p(_i32(start)), _p(_i32(expire)), int(view.frame),
                            _p(_f64(view.cam16())), view.width, view.height, _p(_f64(view.bg)),
                            int(n_opt), _p(_f64(dLdC)), _p(dparams), _p(drec))
    return dparams, drec


def split_images(flat, views):
    """Concatenated planar images -> list of [3, H, W] arrays."""
    out, o = [], 0
    for v in views:
        n = 3 * v.width * v.height
        out.append(np.asarray(flat[o:o + n]).reshape(3, v.height, v.width))
        o += n
    return out


def window_render(params, sh_degree, start, expire, views):
    imgs, Ts = [], []
    for v in views:
        rgb, T, _, _, _ = render_view(params, sh_degree, start, expire, v)
        imgs.append(rgb.reshape(-1))
        Ts.append(T)
    return np.concatenate(imgs), np.concatenate(Ts)


# ------------------------------------------------------------ loss

def window_set(start, expire, num_gs, frames):
    """A = optimisable slots (< num_gs) active in at least one window frame."""
    m = np.zeros(num_gs, bool)
    for f in set(int(x) for x in frames):
        m |= active(start[:num_gs], expire[:num_gs], f)
    return m


def loss_and_grad(images, targets, views, params, in_A, lam_o=2e-2, lam_s=1e-2, lam_dssim=0.0):
    """Window loss (Algorithm 1; image term after 3DGS-MCMC, Sec. 4.4;
    regulariser weights from Sec. 8.1):
    L = (1/V) sum_v [(1 - lam_dssim) mean|C - GT| + lam_dssim (1 - SSIM(C, GT))]
        + lam_o mean_A sigmoid(logit) + lam_s mean_A sum_j exp(s_j).
    Returns (L, image part, dL/dimages, dL/dparams of the regulariser)."""
    V = len(views)
    g = np.zeros(images.shape[0])
    l1, o = 0.0, 0
    for v in views:
        n = 3 * v.width * v.height
        d = images[o:o + n].astype(np.float64) - targets[o:o + n].astype(np.float64)
        l1 += (1.0 - lam_dssim) * np.abs(d).mean() / V
        g[o:o + n] = (1.0 - lam_dssim) * np.sign(d) / (V * n)
        if lam_dssim != 0.0:
            shape = (3, v.height, v.width)
            sv, gs = ssim(images[o:o + n].reshape(shape), targets[o:o + n].reshape(shape))
            l1 += lam_dssim * (1.0 - sv) / V
            g[o:o + n] -= lam_dssim * gs.reshape(-1) / V
        o += n
    P = _f64(params)
    dreg = np.zeros_like(P)
    nA = int(in_A.sum())
    reg = 0.0
    if nA:
        idx = np.nonzero(in_A)[0]
        sig = 1.0 / (1.0 + np.exp(-P[10, idx]))
        es = np.exp(P[3:6][:, idx])
        reg = lam_o * sig.mean() + lam_s * es.sum(axis=0).mean()
        dreg[10, idx] = lam_o * sig * (1.0 - sig) / nA
        dreg[3:6, idx] = lam_s * es / nA
    return l1 + reg, l1, g, dreg


# ------------------------------------------------------------ D-SSIM
# The loss follows 3DGS-MCMC's practice (Sec. 4.4): an image term
# (1 - lam) L1 + lam (1 - SSIM) with lam = 0.2.  SSIM is the structural
# similarity index of Wang, Bovik, Sheikh and Simoncelli (2004) with their
# constants C1 = (0.01 L)^2, C2 = (0.03 L)^2, L = 1, an 11x11 Gaussian window
# of standard deviation 1.5 normalised to sum 1, zero padding outside the
# image, averaged over pixels and colour channels.
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window(size: int = 11, sigma: float = 1.5):
    """w[i, j] = g[i] g[j], g[k] proportional to exp(-(k - size//2)^2 / (2 sigma^2)), sum 1."""
    k = np.arange(size, dtype=np.float64) - size // 2
    g = np.exp(-k * k / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def window_sum(img, w):
    """out(p) = sum_o w(o) img(p + o - r), r = size // 2, zero outside the image."""
    img = _f64(img)
    H, W = img.shape
    r = w.shape[0] // 2
    pad = np.zeros((H + 2 * r, W + 2 * r))
    pad[r:r + H, r:r + W] = img
    out = np.zeros((H, W))
    for dy in range(w.shape[0]):
        for dx in range(w.shape[1]):
            out += w[dy, dx] * pad[dy:dy + H, dx:dx + W]
    return out


def window_sum_adjoint(g, w):
    """Adjoint of window_sum: in(q) = sum_p w(q - p + r) g(p) over pixels p of the image."""
    g = _f64(g)
    H, W = g.shape
    r = w.shape[0] // 2
    pad = np.zeros((H + 2 * r, W + 2 * r))
    pad[r:r + H, r:r + W] = g
    out = np.zeros((H, W))
    for dy in range(w.shape[0]):
        for dx in range(w.shape[1]):
            out += w[dy, dx] * pad[2 * r - dy:2 * r - dy + H, 2 * r - dx:2 * r - dx + W]
    return out


def ssim_map(x, y, w=None):
    """Per-pixel SSIM of two single-channel images [H, W] and the partial
    derivatives of the map with respect to the window mean of x, the window
    mean of x^2 and the window mean of x y."""
    w = ssim_window() if w is None else w
    x, y = _f64(x), _f64(y)
    mx, my = window_sum(x, w), window_sum(y, w)
    exx, eyy, exy = window_sum(x * x, w), window_sum(y * y, w), window_sum(x * y, w)
    A = 2.0 * mx * my + SSIM_C1
    B = 2.0 * (exy - mx * my) + SSIM_C2
    C = mx * mx + my * my + SSIM_C1
    D = (exx - mx * mx) + (eyy - my * my) + SSIM_C2
    S = A * B / (C * D)
    dS_dmx = 2.0 * my * (B - A) / (C * D) - 2.0 * mx * S / C + 2.0 * mx * S / D
    dS_dexx = -S / D
    dS_dexy = 2.0 * A / (C * D)
    return S, dS_dmx, dS_dexx, dS_dexy


def ssim(x, y):
    """Mean SSIM of two planar images [3, H, W] over pixels and channels, and
    its gradient with respect to x (chain rule through the window sums)."""
    w = ssim_window()
    x, y = _f64(x), _f64(y)
    n = x.size
    total, grad = 0.0, np.zeros_like(x)
    for c in range(x.shape[0]):
        S, a, b, e = ssim_map(x[c], y[c], w)
        total += S.sum()
        grad[c] = (window_sum_adjoint(a, w) + 2.0 * x[c] * window_sum_adjoint(b, w)
                   + y[c] * window_sum_adjoint(e, w))
    return total / n, grad / n


def psnr(images, targets):
    mse = np.mean((images.astype(np.float64) - targets.astype(np.float64)) ** 2)
    return 10.0 * math.log10(1.0 / mse) if mse > 0 else float("inf")


# ------------------------------------------------------------ step

DEFAULT_LR = dict(mean=1.6e-4, scale=5e-3, quat=1e-3, logit=5e-2, sh_dc=2.5e-3, sh_rest=1.25e-4)


def lr_rows(sh_degree, lr=DEFAULT_LR):
    F = 11 + 3 * (sh_degree + 1) ** 2
    r = np.zeros(F)
    r[0:3] = lr["mean"]
    r[3:6] = lr["scale"]
    r[6:10] = lr["quat"]
    r[10] = lr["logit"]
    r[11:14] = lr["sh_dc"]
    r[14:] = lr["sh_rest"]
    return r


def normals(seed: int, step: int, slots):
    """Three N(0,1) draws per slot from Philox4x32-10 keyed by the seed with
    counter (slot, step lo, step hi, 'NOIS'), Box-Muller on 24-bit uniforms:
    u1 = (x0>>8 + 1) 2^-24, u2 = (x1>>8) 2^-24, similarly (x2, x3)."""
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    out = np.zeros((3, len(slots)))
    for j, i in enumerate(slots):
        x = philox4x32_10([int(i), step & 0xFFFFFFFF, (step >> 32) & 0xFFFFFFFF, 0x4E4F4953], key)
        u1 = ((int(x[0]) >> 8) + 1) * 2.0 ** -24
        u2 = (int(x[1]) >> 8) * 2.0 ** -24
        u3 = ((int(x[2]) >> 8) + 1) * 2.0 ** -24
        u4 = (int(x[3]) >> 8) * 2.0 ** -24
        r1 = math.sqrt(-2.0 * math.log(u1))
        r2 = math.sqrt(-2.0 * math.log(u3))
        out[0, j] = r1 * math.cos(2 * math.pi * u2)
        out[1, j] = r1 * math.sin(2 * math.pi * u2)
        out[2, j] = r2 * math.cos(2 * math.pi * u4)
    return out


def covariance(params, idx):
    """3D covariance R(q) diag(e^{2s}) R(q)^T of slots idx (Eq. 2)."""
    P = _f64(params)
    out = np.zeros((len(idx), 3, 3))
    for j, i in enumerate(idx):
        q = P[6:10, i] / np.linalg.norm(P[6:10, i])
        w, x, y, z = q
        Rq = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                       [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                       [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        M = Rq * np.exp(P[3:6, i])[None, :]
        out[j] = M @ M.T
    return out


def adam_sgld_step(params, grads, m, v, in_A, t, sh_degree, seed, step,
                   lr=DEFAULT_LR, betas=(0.9, 0.999), eps=1e-15,
                   noise_lr=5e4, k=100.0, t0=0.005, eta=None,
                   grad_scale_base=0.0, window_start=0, swin=1, start=None):
    """One optimiser step over A (Algorithm 1 after the backward; Sec. 4.4 and
    Sec. 4.5.1), in this order:
      1. optional adaptive scaling of the mean gradient by
         base^(w/swin), w = windows already trained = clip(st - start + swin - 1, 0, swin-1);
      2. Adam (Kingma & Ba) with global bias-correction step t, sparse over A;
      3. SGLD noise on means: mu += noise_lr lr_mu sigmoid(-k(o - t0)) Sigma eta,
         Sigma and o taken after the Adam update, eta ~ N(0, I3) (normals()).
    Arrays are planar [F, num_gs] float64 copies; returns (params, m, v)."""
    P = _f64(params).copy()
    G = _f64(grads).copy()
    M = _f64(m).copy()
    Vv = _f64(v).copy()
    idx = np.nonzero(in_A)[0]
    if grad_scale_base > 0.0:
        w = np.clip(window_start - start[idx] + swin - 1, 0, swin - 1)
        G[0:3, idx] *= grad_scale_base ** (w / swin)
    lrr = lr_rows(sh_degree, lr)[:, None]
    b1, b2 = betas
    g = G[:, idx]
    M[:, idx] = b1 * M[:, idx] + (1 - b1) * g
    Vv[:, idx] = b2 * Vv[:, idx] + (1 - b2) * g * g
    mh = M[:, idx] / (1 - b1 ** t)
    vh = Vv[:, idx] / (1 - b2 ** t)
    P[:, idx] = P[:, idx] - lrr * mh / (np.sqrt(vh) + eps)
    if noise_lr != 0.0 and len(idx):
        e = normals(seed, step, idx) if eta is None else _f64(eta)
        Sig = covariance(P, idx)
        o = 1.0 / (1.0 + np.exp(-P[10, idx]))
        gate = 1.0 / (1.0 + np.exp(k * (o - t0)))
        coef = noise_lr * lr["mean"] * gate
        P[0:3, idx] += coef[None, :] * np.einsum("nij,jn->in", Sig, e)
    return P, M, Vv


# ------------------------------------------------------------ relocation

def reloc_SN(N: int, a: float) -> float:
    return lib().orc_reloc_SN(int(N), float(a))


def relocate(params, m, v, in_A, seed, step, n_max=32):
    """Dead-Gaussian relocation (Sec. 3.2, Algorithm 1); see swgs_oracle.c.
    params [F, S] (slots >= len(in_A) untouched), m, v [F, num_gs].
    Returns (params, m, v, dst, src, weight_margin)."""
    P = _f64(params).copy()
    M = _f64(m).copy()
    Vv = _f64(v).copy()
    F, S = P.shape
    n_opt = M.shape[1]
    A = np.ascontiguousarray(in_A, dtype=np.uint8)
    dst = np.zeros(n_opt, np.int32)
    src = np.zeros(n_opt, np.int32)
    wm = np.zeros(1)
    nd = lib().orc_relocate(S, n_opt, F, _p(P), _p(M), _p(Vv), _p(A), int(seed), int(step), int(n_max),
                            _p(dst), _p(src), _p(wm))
    return P, M, Vv, dst[:nd].copy(), src[:nd].copy(), float(wm[0])


# ------------------------------------------------------------ window schedule

def genesis(num_gs: int, swin: int):
    """Algorithm 1 main: every optimisable slot starts with birth 0 and the
    lifespan [0, swin); the frozen store [num_gs, 2 num_gs) is empty."""
    birth = np.zeros(2 * num_gs, np.int32)
    start = np.zeros(2 * num_gs, np.int32)
    expire = np.zeros(2 * num_gs, np.int32)
    expire[:num_gs] = swin
    return birth, start, expire


def schedule_expire(num_gs: int, swin: int, expire):
    """Reading of Algorithm 1's schedule_expire: block k (slots
    [k S, (k+1) S), S = num_gs/swin) expires at frame k for k >= 1 and block
    0 at swin, so exactly one block matures per frame afterwards (Sec. 4.2.1)."""
    S = num_gs // swin
    for k in range(1, swin):
        expire[k * S:(k + 1) * S] = k
    expire[0:S] = swin
    return expire


def mature(st: int, num_gs: int, swin: int, params, birth, start, expire):
    """Algorithm 1 mature(st): optimisable slots whose start < st are
    snapshotted into the frozen store (slot-indexed: slot i -> num_gs + i) and
    emitted in slot order; their lifespan is re-armed to
    [old expire, old expire + swin) with birth = new start.  Arrays are
    modified in place; returns the emitted record as a dict."""
    idx = np.nonzero(start[:num_gs] < st)[0]
    rec = dict(slots=idx.astype(np.int32), birth=birth[idx].copy(), start=start[idx].copy(),
               expire=expire[idx].copy(), params=np.array(params[:, idx], copy=True))
    params[:, num_gs + idx] = params[:, idx]
    birth[num_gs + idx] = birth[idx]
    start[num_gs + idx] = start[idx]
    expire[num_gs + idx] = expire[idx]
    birth[idx] = expire[idx]
    start[idx] = expire[idx]
    expire[idx] = start[idx] + swin
    return rec

"""ctypes binding of libswgs.so (include/swgs.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
the library.  The raw entry points keep the C names (swgs_plan_create,
swgs_window_step, ...); the classes below hold the torch tensors that own the
device memory and call those entry points.  Importing this module raises if
the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswgs.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "swgs.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
_lib = ctypes.CDLL(LIB_PATH)

SWGS_OK, SWGS_ERR_INVALID_ARG, SWGS_ERR_UNSUPPORTED, SWGS_ERR_WORKSPACE_TOO_SMALL, SWGS_ERR_CAPACITY, SWGS_ERR_HIP = range(6)
SWGS_MODE_PLAIN, SWGS_MODE_BATCHED, SWGS_MODE_GRAPH = range(3)
SWGS_TIMING_EVENTS, SWGS_TIMING_COUNT = 1, 2
SWGS_ENC_FP32, SWGS_ENC_Q = 1, 2
(SWGS_BUF_ACTIVE_LIST, SWGS_BUF_ACTIVE_COUNT, SWGS_BUF_RECORD_VIEW_BASE, SWGS_BUF_DEPTH_KEY, SWGS_BUF_TILE_COUNT,
 SWGS_BUF_RECT, SWGS_BUF_SPLAT, SWGS_BUF_PAIR_KEY, SWGS_BUF_PAIR_VAL, SWGS_BUF_PAIR_COUNT, SWGS_BUF_TILE_RANGE,
 SWGS_BUF_T_FINAL, SWGS_BUF_DLDC, SWGS_BUF_RECORD_GRAD, SWGS_BUF_DEPTH_ORDER) = range(15)


class SwgsPool(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("num_gs", ctypes.c_int32), ("n_slots", ctypes.c_int32),
                ("swin", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
                ("params", ctypes.c_void_p), ("grads", ctypes.c_void_p), ("adam_m", ctypes.c_void_p),
                ("adam_v", ctypes.c_void_p), ("birth", ctypes.c_void_p), ("start", ctypes.c_void_p),
                ("expire", ctypes.c_void_p)]


class SwgsView(ctypes.Structure):
    _fields_ = [("frame", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("bg", ctypes.c_float * 3), ("reserved2", ctypes.c_float)]


class SwgsPlanOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("lds_batch", ctypes.c_int32), ("reserved", ctypes.c_int32), ("pair_capacity", ctypes.c_int64)]


class SwgsStepCfg(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t)] + [(n, ctypes.c_float) for n in (
        "lr_mean", "lr_scale", "lr_quat", "lr_logit", "lr_sh_dc", "lr_sh_rest", "beta1", "beta2", "eps",
        "noise_lr", "noise_k", "noise_t0", "lambda_opacity", "lambda_scale", "lambda_dssim", "grad_scale_base")] + [
        (n, ctypes.c_int32) for n in ("window_start", "relocate_period", "reloc_n_max", "mode", "reserved")]


class SwgsServerOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("n_frames", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("lds_batch", ctypes.c_int32), ("max_batch_pixels", ctypes.c_int64), ("pair_ratio", ctypes.c_double)]


class SwgsPlayerOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("queue_depth", ctypes.c_int32), ("max_record_bytes", ctypes.c_int64)]


class SwgsRequest(ctypes.Structure):
    _fields_ = [("view", SwgsView), ("image", ctypes.c_void_p), ("arrival", ctypes.c_double),
                ("ready", ctypes.c_double), ("status", ctypes.c_int32), ("batch", ctypes.c_int32)]


class SwgsServeStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("redone", ctypes.c_int64), ("wall_s", ctypes.c_double),
                ("mean_batch", ctypes.c_double), ("peak_bytes", ctypes.c_size_t), ("budget_bytes", ctypes.c_size_t),
                ("resident_bytes", ctypes.c_size_t)]


P, I32, I64, U64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
_sigs = {
    "swgs_version": ([], ctypes.c_int),
    "swgs_context_create": ([ctypes.c_int, P, P], ctypes.c_int),
    "swgs_context_set_stream": ([P, P], ctypes.c_int),
    "swgs_context_destroy": ([P], ctypes.c_int),
    "swgs_last_error": ([P], ctypes.c_char_p),
    "swgs_plan_create": ([P, P, P, I32, P, P, P], ctypes.c_int),
    "swgs_pool_bind": ([P, P, P], ctypes.c_int),
    "swgs_pool_desc": ([P], P),
    "swgs_pool_release": ([P], ctypes.c_int),
    "swgs_query_workspace_batch": ([P, P, P, I32, P, P], ctypes.c_int),
    "swgs_render_batch": ([P, P, P, I32, P, P, SZ], ctypes.c_int),
    "swgs_plan_destroy": ([P], ctypes.c_int),
    "swgs_plan_measure": ([P, P, P, SZ, P, P], ctypes.c_int),
    "swgs_plan_buffer": ([P, I32, P, P], ctypes.c_int),
    "swgs_plan_info": ([P, P, P, P, P], ctypes.c_int),
    "swgs_render_forward": ([P, P, P, SZ, P, P, P], ctypes.c_int),
    "swgs_render_backward": ([P, P, P, SZ, P, I32, P], ctypes.c_int),
    "swgs_step_cfg_default": ([P], None),
    "swgs_step": ([P, P, P, SZ, P, I64, U64, U64, P], ctypes.c_int),
    "swgs_relocate": ([P, P, P, SZ, P, U64, U64, P, P, P], ctypes.c_int),
    "swgs_window_step": ([P, P, P, SZ, P, P, P, I64, U64, U64, P], ctypes.c_int),
    "swgs_mature": ([P, P, I32, P, SZ, P, P], ctypes.c_int),
    "swgs_mature_noalloc": ([P, P, I32, P, SZ, P, P], ctypes.c_int),
    "swgs_mature_noalloc_max_gs": ([], I64),
    "swgs_record_bytes": ([I64, I32], SZ),
    "swgs_plan_set_timing": ([P, P, P, SZ, I32], ctypes.c_int),
    "swgs_plan_timing": ([P, P, P, SZ, P, P, P], ctypes.c_int),
    "swgs_apply_update": ([P, P, P, SZ, I64, P], ctypes.c_int),
    "swgs_encode_update": ([P, P, SZ, I32, I64, P, SZ, P], ctypes.c_int),
    "swgs_trainer_create": ([P, P, P, I32, P, P], ctypes.c_int),
    "swgs_trainer_run": ([P, P, P, I64, I64, U64, P, P], ctypes.c_int),
    "swgs_trainer_destroy": ([P], None),
    "swgs_trainer_view": ([U64, I64, I32], ctypes.c_int32),
    "swgs_schedule_expire": ([P, P], ctypes.c_int),
    "swgs_player_create": ([P, P, P, P], ctypes.c_int),
    "swgs_player_push": ([P, P, SZ], ctypes.c_int),
    "swgs_player_advance": ([P, I32, P], ctypes.c_int),
    "swgs_player_queued": ([P, P, P], ctypes.c_int),
    "swgs_player_destroy": ([P], None),
    "swgs_server_create": ([P, P, P, P, SZ, P], ctypes.c_int),
    "swgs_server_destroy": ([P], ctypes.c_int),
    "swgs_server_submit": ([P, P, I32], ctypes.c_int),
    "swgs_server_progress": ([P, I32, P], ctypes.c_int),
    "swgs_server_run": ([P, P, I32, I32, P], ctypes.c_int),
    "swgs_server_stats": ([P, P], ctypes.c_int),
}
TIMING_CLASSES = ("gate", "preprocess", "sort", "blend_fwd", "blend_bwd", "preprocess_bwd", "adam_sgld", "relocate",
                  "dssim")
for _n, (_a, _r) in _sigs.items():
    _f = getattr(_lib, _n)
    _f.argtypes = _a
    _f.restype = _r
    globals()[_n] = _f


def header_functions(path: str = HEADER):
    """Names of every function the public header declares."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(swgs_[a-z0-9_]+)\s*\(", txt)))


class SwgsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"swgs status {status}: {msg}")
        self.status = status


def ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """A device binding plus the (non-default, default-priority) stream all
    library work runs on; calls are ordered after torch's current stream and
    torch's current stream waits for them."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        st = swgs_context_create(device, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != SWGS_OK:
            raise SwgsError(st, "context create failed")
        self.h = h

    def check(self, st):
        if st != SWGS_OK:
            raise SwgsError(st, swgs_last_error(self.h).decode())

    def __enter__(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        return self

    def __exit__(self, *exc):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return False

    def close(self):
        if self.h:
            self.stream.synchronize()
            swgs_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """Device tensors of a slot pool (planar rows [F, n_slots])."""

    def __init__(self, params, birth, start, expire, num_gs, swin, sh_degree, device, train=True):
        dev = torch.device(device)
        self.params = torch.as_tensor(np.ascontiguousarray(params, np.float32)).to(dev)
        self.birth = torch.as_tensor(np.ascontiguousarray(birth, np.int32)).to(dev)
        self.start = torch.as_tensor(np.ascontiguousarray(start, np.int32)).to(dev)
        self.expire = torch.as_tensor(np.ascontiguousarray(expire, np.int32)).to(dev)
        self.num_gs, self.swin, self.sh_degree = int(num_gs), int(swin), int(sh_degree)
        F = self.params.shape[0]
        n = max(self.num_gs, 1)
        if train:
            self.grads = torch.zeros((F, n), dtype=torch.float32, device=dev)
            self.adam_m = torch.zeros((F, n), dtype=torch.float32, device=dev)
            self.adam_v = torch.zeros((F, n), dtype=torch.float32, device=dev)
        else:
            self.grads = self.adam_m = self.adam_v = None

    @classmethod
    def from_synth(cls, pool, device="cuda", train=True):
        return cls(pool.params, pool.birth, pool.start, pool.expire, pool.num_gs, pool.swin, pool.sh_degree,
                   device, train)

    def c(self) -> SwgsPool:
        return SwgsPool(ctypes.sizeof(SwgsPool), self.num_gs, self.params.shape[1], self.swin, self.sh_degree,
                        self.params.data_ptr(), self.grads.data_ptr() if self.grads is not None else None,
                        self.adam_m.data_ptr() if self.adam_m is not None else None,
                        self.adam_v.data_ptr() if self.adam_v is not None else None,
                        self.birth.data_ptr(), self.start.data_ptr(), self.expire.data_ptr())


def c_views(views):
    arr = (SwgsView * len(views))()
    for i, v in enumerate(views):
        arr[i].frame = int(v.frame)
        arr[i].width = int(v.width)
        arr[i].height = int(v.height)
        R = np.asarray(v.R, np.float64).reshape(-1)
        t = np.asarray(v.t, np.float64).reshape(-1)
        for k in range(9):
            arr[i].R[k] = float(R[k])
        for k in range(3):
            arr[i].t[k] = float(t[k])
            arr[i].bg[k] = float(v.bg[k])
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = float(v.fx), float(v.fy), float(v.cx), float(v.cy)
    return arr


def step_cfg(**kw) -> SwgsStepCfg:
    c = SwgsStepCfg()
    swgs_step_cfg_default(ctypes.byref(c))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


class Plan:
    """A plan over a pool and a list of views, with its workspace."""

    def __init__(self, ctx: Context, pool: Pool, views, tile=(16, 16), lds_batch=0, pair_capacity=None,
                 headroom=1.3):
        self.ctx, self.pool, self.views = ctx, pool, list(views)
        self.cviews = c_views(self.views)
        self.tile, self.lds_batch = tile, lds_batch
        self.h = None
        self._cpool = pool.c()
        cap = int(pair_capacity) if pair_capacity else 1 << 16
        self._create(cap)
        if pair_capacity is None:
            k = self.measure()
            self._create(int(k * headroom) + 65536)

    def _create(self, cap):
        if self.h:
            swgs_plan_destroy(self.h)
            self.h = None
        opts = SwgsPlanOpts(ctypes.sizeof(SwgsPlanOpts), self.tile[0], self.tile[1], self.lds_batch, 0, cap)
        h = ctypes.c_void_p()
        nb = ctypes.c_size_t()
        with self.ctx:
            self.ctx.check(swgs_plan_create(self.ctx.h, ctypes.byref(self._cpool), self.cviews, len(self.views),
                                            ctypes.byref(opts), ctypes.byref(h), ctypes.byref(nb)))
        self.h = h
        self.cap = cap
        self.ws_bytes = nb.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.ctx.device)
        ng, nr, npx, nt = (ctypes.c_int64() for _ in range(4))
        swgs_plan_info(self.h, ctypes.byref(ng), ctypes.byref(nr), ctypes.byref(npx), ctypes.byref(nt))
        self.n_groups, self.n_records, self.n_pixels, self.n_tiles = ng.value, nr.value, npx.value, nt.value

    def measure(self):
        k, r = ctypes.c_int64(), ctypes.c_int64()
        with self.ctx:
            self.ctx.check(swgs_plan_measure(self.ctx.h, self.h, ptr(self.ws), self.ws_bytes, ctypes.byref(k),
                                             ctypes.byref(r)))
        return k.value

    def buffer(self, which, dtype=torch.uint32):
        off, nb = ctypes.c_size_t(), ctypes.c_size_t()
        self.ctx.check(swgs_plan_buffer(self.h, which, ctypes.byref(off), ctypes.byref(nb)))
        b = self.ws[off.value:off.value + nb.value]
        return b.view(dtype)

    def image_buffer(self):
        return torch.empty(3 * self.n_pixels, dtype=torch.float32, device=self.ctx.device)

    def forward(self, images=None, targets=None, stats=None):
        images = self.image_buffer() if images is None else images
        with self.ctx:
            self.ctx.check(swgs_render_forward(self.ctx.h, self.h, ptr(self.ws), self.ws_bytes, ptr(images),
                                               ptr(targets), ptr(stats)))
        return images

    def backward(self, dL=None, add_reg=0, cfg=None):
        with self.ctx:
            self.ctx.check(swgs_render_backward(self.ctx.h, self.h, ptr(self.ws), self.ws_bytes, ptr(dL),
                                                int(add_reg), ctypes.byref(cfg) if cfg is not None else None))

    def step(self, cfg, adam_t, step, seed, eta=None):
        with self.ctx:
            self.ctx.check(swgs_step(self.ctx.h, self.h, ptr(self.ws), self.ws_bytes, ctypes.byref(cfg),
                                     int(adam_t), int(step), int(seed), ptr(eta)))

    def relocate(self, cfg, step, seed):
        n = max(self.pool.num_gs, 1)
        dst = torch.empty(n, dtype=torch.int32, device=self.ctx.device)
        src = torch.empty(n, dtype=torch.int32, device=self.ctx.device)
        cnt = torch.zeros(1, dtype=torch.int32, device=self.ctx.device)
        with self.ctx:
            self.ctx.check(swgs_relocate(self.ctx.h, self.h, ptr(self.ws), self.ws_bytes, ctypes.byref(cfg),
                                         int(step), int(seed), ptr(dst), ptr(src), ptr(cnt)))
        c = int(cnt.item())
        return dst[:c], src[:c]

    def window_step(self, cfg, targets, adam_t, step, seed, images=None, stats=None):
        with self.ctx:
            self.ctx.check(swgs_window_step(self.ctx.h, self.h, ptr(self.ws), self.ws_bytes, ctypes.byref(cfg),
                                            ptr(targets), ptr(images), int(adam_t), int(step), int(seed),
                                            ptr(stats)))

    def set_timing(self, flags: int):
        """SWGS_TIMING_EVENTS | SWGS_TIMING_COUNT, or 0 (off)."""
        with self.ctx:
            self.ctx.check(swgs_plan_set_timing(self.ctx.h, self.h, ptr(self.ws), self.ws_bytes, int(flags)))

    def timing(self):
        """{class: (total ms, launches)} and (fwd evaluated, bwd evaluated, blended) pairs since the last reset."""
        ms = (ctypes.c_double * len(TIMING_CLASSES))()
        n = (ctypes.c_int64 * len(TIMING_CLASSES))()
        ev = (ctypes.c_uint64 * 3)()
        with self.ctx:
            self.ctx.check(swgs_plan_timing(self.ctx.h, self.h, ptr(self.ws), self.ws_bytes, ms, n, ev))
        return {k: (ms[i], n[i]) for i, k in enumerate(TIMING_CLASSES)}, (ev[0], ev[1], ev[2])

    def close(self):
        if self.h:
            self.ctx.stream.synchronize()
            swgs_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mature(ctx: Context, pool: Pool, st: int):
    """Algorithm 1's mature(st) on the device; returns the packed record
    (uint8 device tensor) and the number of Gaussians it holds."""
    cap = swgs_record_bytes(pool.num_gs, pool.sh_degree)
    rec = torch.empty(cap, dtype=torch.uint8, device=ctx.device)
    cnt, nb = ctypes.c_int64(), ctypes.c_size_t()
    cp = pool.c()
    with ctx:
        ctx.check(swgs_mature(ctx.h, ctypes.byref(cp), int(st), ptr(rec), cap, ctypes.byref(cnt), ctypes.byref(nb)))
    return rec[:nb.value], cnt.value


def mature_noalloc(ctx: Context, pool: Pool, st: int, record):
    """swgs_mature_noalloc into the caller's `record` (uint8 device tensor of
    at least swgs_record_bytes(num_gs, sh_degree) bytes); returns the used
    part of the record and the number of Gaussians it holds."""
    cnt, nb = ctypes.c_int64(), ctypes.c_size_t()
    cp = pool.c()
    with ctx:
        ctx.check(swgs_mature_noalloc(ctx.h, ctypes.byref(cp), int(st), ptr(record), record.numel(),
                                      ctypes.byref(cnt), ctypes.byref(nb)))
    return record[:nb.value], cnt.value


def encode_update(ctx: Context, record, enc: int = SWGS_ENC_Q, keep: int = -1):
    """The compact per-frame update of a mature record (uint8 device tensor):
    mean, log-scale, rotation, opacity and SH DC per Gaussian, in FP32
    (SWGS_ENC_FP32) or at Table 6's precisions (SWGS_ENC_Q); keep >= 0 keeps
    only the `keep` most opaque entries.  Returns a uint8 device tensor."""
    nb = ctypes.c_size_t()
    with ctx:
        ctx.check(swgs_encode_update(ctx.h, ptr(record), int(record.numel()), int(enc), int(keep), None, 0,
                                     ctypes.byref(nb)))
        out = torch.empty(nb.value, dtype=torch.uint8, device=ctx.device)
        ctx.check(swgs_encode_update(ctx.h, ptr(record), int(record.numel()), int(enc), int(keep), ptr(out),
                                     nb.value, ctypes.byref(nb)))
    return out[:nb.value]


class Trainer:
    """The paper's loop over one window (Algorithm 1's train_swin): one
    single-view plan per (frame, camera) in `views`; run() samples a view per
    iteration and steps on it.  The pool's lifespans must stay fixed while
    the trainer lives (close it before mature())."""

    def __init__(self, ctx: Context, pool: Pool, views, tile=(16, 16), lds_batch=0, headroom=1.5):
        self.ctx, self.pool, self.views = ctx, pool, list(views)
        # one pair capacity for all views: the largest measured count, with headroom
        k = 0
        for v in self.views:
            probe = Plan(ctx, pool, [v], tile=tile, lds_batch=lds_batch, pair_capacity=1 << 16)
            k = max(k, probe.measure())
            probe.close()
        self.pair_capacity = int(k * headroom) + 65536
        opts = SwgsPlanOpts(ctypes.sizeof(SwgsPlanOpts), tile[0], tile[1], lds_batch, 0, self.pair_capacity)
        self._cp = pool.c()
        self._cv = c_views(self.views)
        h = ctypes.c_void_p()
        with ctx:
            ctx.check(swgs_trainer_create(ctx.h, ctypes.byref(self._cp), self._cv, len(self.views), ctypes.byref(opts),
                                          ctypes.byref(h)))
        self.h = h

    def run(self, cfg, targets, iterations: int, iter0: int, seed: int, stats=None):
        """targets: one device tensor per view.  Returns the sampled view of
        each iteration (numpy int32)."""
        tp = (ctypes.c_void_p * len(self.views))(*[t.data_ptr() for t in targets])
        vo = np.zeros(max(1, iterations), np.int32)
        with self.ctx:
            self.ctx.check(swgs_trainer_run(self.h, ctypes.byref(cfg), tp, int(iterations), int(iter0), int(seed),
                                            ptr(stats), vo.ctypes.data_as(ctypes.c_void_p)))
        return vo[:iterations]

    def close(self):
        if self.h:
            swgs_trainer_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trainer_view(seed: int, iteration: int, n_views: int) -> int:
    return int(swgs_trainer_view(int(seed), int(iteration), int(n_views)))


def schedule_expire(ctx: Context, pool: Pool):
    cp = pool.c()
    with ctx:
        ctx.check(swgs_schedule_expire(ctx.h, ctypes.byref(cp)))


class Player:
    """Client playback of the update stream (Algorithm 2): push() records
    (host bytes) as they arrive, advance(frame) once per frame; the buffer
    pool then holds the slices live at that frame."""

    def __init__(self, ctx: Context, buffer: Pool, queue_depth: int = 4, max_record_bytes: int = 1 << 20):
        self.ctx, self.buffer = ctx, buffer
        o = SwgsPlayerOpts(ctypes.sizeof(SwgsPlayerOpts), int(queue_depth), int(max_record_bytes))
        self._cp = buffer.c()
        h = ctypes.c_void_p()
        with ctx:
            ctx.check(swgs_player_create(ctx.h, ctypes.byref(self._cp), ctypes.byref(o), ctypes.byref(h)))
        self.h = h

    def push(self, record):
        a = np.ascontiguousarray(np.frombuffer(bytes(record), np.uint8) if isinstance(record, (bytes, bytearray))
                                 else record, dtype=np.uint8)
        with self.ctx:
            self.ctx.check(swgs_player_push(self.h, a.ctypes.data_as(ctypes.c_void_p), a.nbytes))

    def advance(self, frame: int) -> int:
        n = ctypes.c_int32()
        with self.ctx:
            self.ctx.check(swgs_player_advance(self.h, int(frame), ctypes.byref(n)))
        return n.value

    def queued(self):
        q, a = ctypes.c_int32(), ctypes.c_int64()
        self.ctx.check(swgs_player_queued(self.h, ctypes.byref(q), ctypes.byref(a)))
        return q.value, a.value

    def close(self):
        if self.h:
            swgs_player_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def parse_record(rec: np.ndarray):
    """Decode a packed mature record (host bytes) into a dict."""
    h = np.frombuffer(rec[:32].tobytes(), np.int32)
    assert h[0] == 0x53475753 and h[1] == 1
    n, F = int(h[3]), int(h[5])
    o = 32
    slots = np.frombuffer(rec[o:o + 4 * n].tobytes(), np.uint32); o += 4 * n
    lb = np.frombuffer(rec[o:o + 12 * n].tobytes(), np.int32).reshape(3, n); o += 12 * n
    params = np.frombuffer(rec[o:o + 4 * F * n].tobytes(), np.float32).reshape(F, n)
    return dict(st=int(h[2]), count=n, sh_degree=int(h[4]), F=F, swin=int(h[6]), slots=slots,
                birth=lb[0], start=lb[1], expire=lb[2], params=params)


class RenderFunction(torch.autograd.Function):
    """images = render(params) over a plan's views; the backward runs the
    library's adjoint kernels and returns dL/dparams for the optimisable
    slots live in the plan's frames (zero elsewhere, frozen slots included)."""

    @staticmethod
    def forward(fctx, params, plan: Plan):
        assert params.data_ptr() == plan.pool.params.data_ptr(), "params must be the plan's pool tensor"
        images = plan.forward()
        fctx.plan = plan
        return images

    @staticmethod
    def backward(fctx, grad_images):
        plan = fctx.plan
        pool = plan.pool
        pool.grads.zero_()
        plan.backward(grad_images.contiguous())
        g = torch.zeros_like(pool.params)
        g[:, :pool.num_gs] = pool.grads[:, :pool.num_gs]
        return g, None


def render(params, plan: Plan):
    return RenderFunction.apply(params, plan)


def apply_update(ctx: Context, pool: Pool, record, slot_base: int = -1) -> int:
    """Algorithm 2's update: scatter a mature record (uint8 device tensor)
    into the pool, at the slots it was emitted from (slot_base < 0) or at
    slot_base + k.  Returns the number of entries."""
    cnt = ctypes.c_int64()
    cp = pool.c()
    with ctx:
        ctx.check(swgs_apply_update(ctx.h, ctypes.byref(cp), ptr(record), int(record.numel()), int(slot_base),
                                    ctypes.byref(cnt)))
    return cnt.value


def c_requests(views, images=None, arrivals=None):
    arr = (SwgsRequest * len(views))()
    cv = c_views(views)
    for i in range(len(views)):
        arr[i].view = cv[i]
        arr[i].image = images[i].data_ptr() if images is not None and images[i] is not None else None
        arr[i].arrival = float(arrivals[i]) if arrivals is not None else 0.0
        arr[i].status = -1
        arr[i].batch = -1
    return arr


class BoundPool:
    """A pool bound with swgs_pool_bind (descriptor checked once, device
    pointers verified); .desc() is the descriptor every call takes."""

    def __init__(self, ctx: Context, pool: Pool):
        self.ctx, self.pool = ctx, pool
        self._cpool = pool.c()
        h = ctypes.c_void_p()
        with ctx:
            ctx.check(swgs_pool_bind(ctx.h, ctypes.byref(self._cpool), ctypes.byref(h)))
        self.h = h

    def desc(self):
        return swgs_pool_desc(self.h)

    def close(self):
        if self.h:
            swgs_pool_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def render_batch(ctx: Context, pool: Pool, views, images=None, tile=(16, 16), lds_batch=0, pair_capacity=1 << 22):
    """swgs_render_batch of one batch of (frame, camera, resolution)
    requests into `images` (list of device [3, H, W] tensors or None);
    returns the per-request statuses and the workspace bytes used."""
    reqs = c_requests(views, images)
    cp = pool.c()
    opts = SwgsPlanOpts(ctypes.sizeof(SwgsPlanOpts), int(tile[0]), int(tile[1]), int(lds_batch), 0, int(pair_capacity))
    nb = ctypes.c_size_t()
    with ctx:
        ctx.check(swgs_query_workspace_batch(ctx.h, ctypes.byref(cp), reqs, len(views), ctypes.byref(opts),
                                             ctypes.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device=ctx.device)
        st = swgs_render_batch(ctx.h, ctypes.byref(cp), reqs, len(views), ctypes.byref(opts), ptr(ws), nb.value)
    status = np.array([reqs[i].status for i in range(len(views))])
    if st != SWGS_OK:
        raise SwgsError(st, (swgs_last_error(ctx.h) or b"").decode())
    return status, nb.value


class Server:
    """Render server over a resident pool (forward only).  arena_bytes of
    device memory are allocated here and handed to the library: per-frame
    live lists at its head, the rest is the memory budget for batches."""

    def __init__(self, ctx: Context, pool: Pool, n_frames: int, arena_bytes: int, lanes: int = 3,
                 max_batch: int = 16, tile=(16, 16), lds_batch: int = 0, max_batch_pixels: int = 0,
                 pair_ratio: float = 0.0):
        self.ctx, self.pool = ctx, pool
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=ctx.device)
        opts = SwgsServerOpts(ctypes.sizeof(SwgsServerOpts), int(n_frames), int(lanes), int(max_batch),
                              int(tile[0]), int(tile[1]), int(lds_batch), int(max_batch_pixels), float(pair_ratio))
        self._cpool = pool.c()
        h = ctypes.c_void_p()
        with ctx:
            ctx.check(swgs_server_create(ctx.h, ctypes.byref(self._cpool), ctypes.byref(opts), ptr(self.arena),
                                         int(arena_bytes), ctypes.byref(h)))
        self.h = h
        self._live = []          # request arrays the library may still write into

    def run(self, views, arrivals=None, images=None, realtime=False):
        """Replay requests (views with frame/resolution/camera); arrivals in
        seconds (realtime) or all at once.  images: optional list of device
        tensors [3, H, W] to receive each render.  Returns (arrival, ready,
        status, batch) numpy arrays and the stats dict."""
        reqs = c_requests(views, images, arrivals)
        st = SwgsServeStats()
        st.struct_size = ctypes.sizeof(SwgsServeStats)
        torch.cuda.synchronize(self.ctx.device)
        self.ctx.check(swgs_server_run(self.h, reqs, len(views), int(bool(realtime)), ctypes.byref(st)))
        out = (np.array([r.arrival for r in reqs]), np.array([r.ready for r in reqs]),
               np.array([r.status for r in reqs], np.int32), np.array([r.batch for r in reqs], np.int32))
        return out, {k: getattr(st, k) for k, _ in SwgsServeStats._fields_ if k != "struct_size"}

    def submit(self, views, images=None):
        reqs = c_requests(views, images)
        torch.cuda.synchronize(self.ctx.device)
        self.ctx.check(swgs_server_submit(self.h, reqs, len(views)))
        self._live.append(reqs)
        return reqs

    def progress(self, wait=False) -> int:
        n = ctypes.c_int64()
        self.ctx.check(swgs_server_progress(self.h, int(bool(wait)), ctypes.byref(n)))
        if n.value == 0:
            self._live = []
        return n.value

    def stats(self):
        st = SwgsServeStats()
        st.struct_size = ctypes.sizeof(SwgsServeStats)
        self.ctx.check(swgs_server_stats(self.h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in SwgsServeStats._fields_ if k != "struct_size"}

    def close(self):
        if self.h:
            swgs_server_destroy(self.h)
            self.h = None
            self._live = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Python handle of the neural guiding field (wost_guide_*)."""
from __future__ import annotations

import ctypes as C
import dataclasses

import torch

from . import _lib as L
from .api import _ptr, _stream


@dataclasses.dataclass
class GuideConfig:
    dim: int = 2
    levels: int = 8
    feats: int = 2
    log2_table: int = 16
    n_min: int = 16
    n_max: int = 1024
    hidden: int = 64
    n_hidden: int = 2
    K: int = 8
    aabb_lo: tuple = (-1.0, -1.0, 0.0)
    aabb_hi: tuple = (1.0, 1.0, 0.0)

    @property
    def n_out(self):
        return self.K * (self.dim + 2) + 1

    def to_c(self):
        lo = list(self.aabb_lo) + [0.0] * (3 - len(self.aabb_lo))
        hi = list(self.aabb_hi) + [0.0] * (3 - len(self.aabb_hi))
        return L.wost_guide_config(self.dim, self.levels, self.feats, self.log2_table, self.n_min, self.n_max,
                                   self.hidden, self.n_hidden, self.K, (C.c_float * 3)(*lo[:3]),
                                   (C.c_float * 3)(*hi[:3]))

    @classmethod
    def for_scene(cls, scene, pad=0.01, **kw):
        lo = scene.verts.min(axis=0)
        hi = scene.verts.max(axis=0)
        ext = hi - lo
        lo = lo - pad * ext
        hi = hi + pad * ext
        base = dict(dim=scene.dim, aabb_lo=tuple(float(v) for v in lo), aabb_hi=tuple(float(v) for v in hi))
        if scene.dim == 3:
            base.update(levels=16, log2_table=19, n_min=16, n_max=512, n_hidden=3)
        base.update(kw)
        return cls(**base)


class Guide:
    """Parameters (fp32 master, fp16 shadow), Adam state and gradient live in
    torch tensors bound to the library handle."""

    def __init__(self, cfg: GuideConfig, seed=1, device=None, train=True):
        lib = L.load()
        self.cfg = cfg
        h = C.c_void_p()
        c = cfg.to_c()
        L.check(lib.wost_guide_create(C.byref(c), C.byref(h)), "wost_guide_create")
        self.h = h
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.n_params = lib.wost_guide_param_count(h)
        nshadow = lib.wost_guide_shadow_bytes(h)
        self.master = torch.zeros(self.n_params, dtype=torch.float32, device=dev)
        self.shadow = torch.zeros((nshadow + 1) // 2, dtype=torch.float16, device=dev)
        self.adam_m = torch.zeros_like(self.master) if train else None
        self.adam_v = torch.zeros_like(self.master) if train else None
        self.grad = torch.zeros_like(self.master) if train else None
        L.check(lib.wost_guide_bind(h, _ptr(self.master), _ptr(self.shadow), _ptr(self.adam_m), _ptr(self.adam_v),
                                    _ptr(self.grad)), "wost_guide_bind")
        L.check(lib.wost_guide_init(h, int(seed), _stream()), "wost_guide_init")

    def __del__(self):
        # at interpreter shutdown the binding module may already be torn down
        lib = getattr(L, "_lib", None) if L is not None else None
        if getattr(self, "h", None) is not None and lib is not None:
            lib.wost_guide_free(self.h)
            self.h = None

    @property
    def reflect(self) -> bool:
        """Sample reflection at Neumann points (Sec. 4.3); False selects the
        variant without it (guided draws into the wall are wasted)."""
        return bool(L.load().wost_guide_get_reflect(self.h))

    @reflect.setter
    def reflect(self, on):
        L.check(L.load().wost_guide_set_reflect(self.h, 1 if on else 0), "wost_guide_set_reflect")

    def set_params(self, flat):
        """Overwrite the fp32 master parameters and refresh the fp16 shadow."""
        self.master.copy_(torch.as_tensor(flat, dtype=torch.float32))
        L.check(L.load().wost_guide_sync_shadow(self.h, _stream()), "wost_guide_sync_shadow")

    def sync_shadow(self):
        L.check(L.load().wost_guide_sync_shadow(self.h, _stream()), "wost_guide_sync_shadow")

    def infer(self, pts):
        pts = pts.contiguous()
        out = torch.empty(pts.shape[0], self.cfg.n_out, dtype=torch.float32, device=pts.device)
        L.check(L.load().wost_guide_infer(self.h, _ptr(pts), pts.shape[0], _ptr(out), _stream()), "wost_guide_infer")
        return out

    # ------------------------------------------------------------ training
    def _ws(self, count):
        need = int(L.load().wost_guide_train_workspace_bytes(self.h, int(count)))
        ws = getattr(self, "_workspace", None)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.master.device)
            self._workspace = ws
        return ws

    def loss_fwd(self, records, begin=0, count=None, e_mis=0.2):
        count = records.n() - begin if count is None else count
        out = torch.empty(max(count, 1), dtype=torch.float32, device=self.master.device)
        rec = records.to_c()
        L.check(L.load().wost_guide_loss_fwd(self.h, C.byref(rec), int(begin), int(count), float(e_mis), _ptr(out),
                                             _stream()), "wost_guide_loss_fwd")
        return out[:count]

    def loss_bwd(self, records, begin=0, count=None, e_mis=0.2, scale=1.0, dloss=None, grad=None):
        count = records.n() - begin if count is None else count
        rec = records.to_c()
        ws = self._ws(count)
        L.check(L.load().wost_guide_loss_bwd(self.h, C.byref(rec), int(begin), int(count), float(e_mis),
                                             float(scale), _ptr(dloss.contiguous()) if dloss is not None else None,
                                             _ptr(grad), _ptr(ws), ws.numel(), _stream()), "wost_guide_loss_bwd")

    def adam_step(self, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, e_mis=0.2):
        opt = L.wost_adam(lr, beta1, beta2, eps, e_mis)
        L.check(L.load().wost_guide_adam_step(self.h, C.byref(opt), _stream()), "wost_guide_adam_step")

    def train_step(self, records, begin, count, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, e_mis=0.2, loss_out=None):
        opt = L.wost_adam(lr, beta1, beta2, eps, e_mis)
        rec = records.to_c()
        ws = self._ws(count)
        L.check(L.load().wost_guide_train_step(self.h, C.byref(rec), int(begin), int(count), C.byref(opt),
                                               _ptr(loss_out), _ptr(ws), ws.numel(), _stream()),
                "wost_guide_train_step")

    def train_step_noalloc(self, records, begin, count, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, e_mis=0.2,
                           loss_out=None):
        """``train_step`` through the allocation-free entry point (workspace
        in the library's own device array; nothing is allocated)."""
        opt = L.wost_adam(lr, beta1, beta2, eps, e_mis)
        rec = records.to_c()
        L.check(L.load().wost_guide_train_step_noalloc(self.h, C.byref(rec), int(begin), int(count), C.byref(opt),
                                                       _ptr(loss_out), _stream()),
                "wost_guide_train_step_noalloc")

    def sample(self, pts, normals=None, sampling="mis_learned", c_fixed=0.5, seed=18944, walk_index=0):
        pts = pts.contiguous()
        n = pts.shape[0]
        nu = torch.empty(n, self.cfg.dim, dtype=torch.float32, device=pts.device)
        pdf = torch.empty(n, dtype=torch.float32, device=pts.device)
        s = L.SAMPLING[sampling] if isinstance(sampling, str) else int(sampling)
        L.check(L.load().wost_guide_sample(self.h, s, float(c_fixed), _ptr(pts),
                                           _ptr(normals.contiguous()) if normals is not None else None, n,
                                           int(seed), int(walk_index), _ptr(nu), _ptr(pdf), _stream()),
                "wost_guide_sample")
        return nu, pdf


def tail_pass(records, walk_value):
    """Fill the p_t field of the records from the per-walk estimates."""
    rec = records.to_c()
    L.check(L.load().wost_tail_pass(records.dim, C.byref(rec), _ptr(walk_value), walk_value.numel(), _stream()),
            "wost_tail_pass")


class GuideLoss(torch.autograd.Function):
    """Per-record guide loss as a torch op: forward runs wost_guide_loss_fwd,
    backward runs the hand-written wost_guide_loss_bwd.  ``params`` is the
    guide's master parameter tensor (the kernels read its fp16 shadow)."""

    @staticmethod
    def forward(ctx, params, guide, records, begin, count, e_mis):
        ctx.guide, ctx.records, ctx.begin, ctx.count, ctx.e_mis = guide, records, begin, count, e_mis
        return guide.loss_fwd(records, begin, count, e_mis)

    @staticmethod
    def backward(ctx, dloss):
        g = ctx.guide
        grad = torch.zeros_like(g.master)
        g.loss_bwd(ctx.records, ctx.begin, ctx.count, ctx.e_mis, scale=1.0, dloss=dloss.float(), grad=grad)
        return grad, None, None, None, None, None


def sample_records(src, seed, m, dst):
    """dst <- m rows of src drawn uniformly with replacement (wost_records_sample)."""
    a, b = src.to_c(), dst.to_c()
    L.check(L.load().wost_records_sample(src.dim, C.byref(a), int(seed), int(m), C.byref(b), _stream()),
            "wost_records_sample")

"""Python binding of libnst: same entry points, argument marshalling only.

PyTorch supplies device memory (inputs, outputs, the workspace) and the stream;
every step of the loss and gradient runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_double, c_float, c_int, c_size_t, c_void_p

import numpy as np
import torch

from ._lib import (NST_BF16, NST_BOTH, NST_CHECK_FINITE, NST_FP32, NST_RESIDENT, NST_STEP1, NST_STEP2,
                   NST_STRICT_HALO, MeanStd, NetDesc, Tile, check, lib)

PRECISIONS = {"fp32": NST_FP32, "bf16": NST_BF16}


def vgg19_desc(tiny: bool = False, with_content: bool = True, avg_pool: bool = False) -> NetDesc:
    """The VGG-19 prefix; avg_pool replaces every max pool by a 2x2 average pool."""
    d = NetDesc()
    check("nst_net_vgg19", lib().nst_net_vgg19(byref(d), int(tiny), int(with_content)))
    if avg_pool:
        d.pool_avg = d.pool_after
    return d


def desc_info(d: NetDesc):
    convs = [(d.c_in[i], d.c_out[i]) for i in range(d.n_conv)]
    style = [d.style_conv[k] for k in range(d.n_style)]
    return convs, style, d.content_conv


def min_halo(d: NetDesc) -> int:
    r = lib().nst_min_halo(byref(d))
    if r < 0:
        check("nst_min_halo", r)
    return r


def plan(d: NetDesc, H: int, W: int, T: int, m: int):
    """Tiles of the plan as tuples (by0, by1, bx0, bx1, ey0, ey1, ex0, ex1, own[n_conv][4])."""
    n = c_int(0)
    r = lib().nst_plan(byref(d), H, W, T, m, None, 0, byref(n))
    if r not in (0, -6):
        check("nst_plan", r)
    arr = (Tile * max(n.value, 1))()
    check("nst_plan", lib().nst_plan(byref(d), H, W, T, m, arr, n.value, byref(n)))
    out = []
    for t in arr[: n.value]:
        own = tuple(tuple(t.own[i][j] for j in range(4)) for i in range(d.n_conv))
        out.append((t.by0, t.by1, t.bx0, t.bx1, t.ey0, t.ey1, t.ex0, t.ex1, own))
    return out


def workspace_bytes(d: NetDesc, precision: str, H: int, W: int, T: int, m: int, batch: int) -> int:
    b = c_size_t(0)
    check("nst_workspace_bytes",
          lib().nst_workspace_bytes(byref(d), PRECISIONS[precision], H, W, T, m, batch, byref(b)))
    return b.value


def _ptr(t: torch.Tensor):
    return c_void_p(t.data_ptr())


def _stream(dev):
    return c_void_p(torch.cuda.current_stream(dev).cuda_stream)


class MeanStdTerms:
    """Weights and statistics of the mean and std terms of the augmented style loss
    (Eq. 5): w_mean = w'_l and w_std = w''_l per style layer, target_means = the style
    image's channel means (Context.style_stats), means_x = the channel means of x
    (written by Step 1, read by a Step-2-only call; allocated on first use)."""

    def __init__(self, w_mean, w_std, target_means: torch.Tensor, means_x: torch.Tensor | None = None):
        self.w_mean, self.w_std = list(w_mean), list(w_std)
        self.target_means, self.means_x = target_means, means_x

    def _struct(self, n_style):
        if self.means_x is None:
            self.means_x = torch.empty_like(self.target_means)
        self._wm = (c_double * max(n_style, 1))(*[float(v) for v in self.w_mean])
        self._wsd = (c_double * max(n_style, 1))(*[float(v) for v in self.w_std])
        return MeanStd(self._wm, self._wsd, _ptr(self.target_means), _ptr(self.means_x))


class Context:
    """An nst_ctx: packed weights of one network in one precision on one device."""

    def __init__(self, weights, biases=None, precision: str = "fp32", desc: NetDesc | None = None,
                 tiny: bool = False, with_content: bool = True, ws_limit: int = 96 << 30,
                 tile_batch: int = 32, resident: bool = False, avg_pool: bool = False):
        """resident: keep every tile's activations from Step 1 to Step 2 of a loss_grad call
        (NST_RESIDENT, a workspace for every tile) instead of recomputing them per tile
        batch as Algorithm 1 does."""
        self.desc = desc if desc is not None else vgg19_desc(tiny, with_content, avg_pool)
        self.convs, self.style, self.content = desc_info(self.desc)
        self.precision = precision
        self.device = torch.device("cuda", torch.cuda.current_device())
        n = self.desc.n_conv
        self._w = [np.ascontiguousarray(w, np.float32) for w in weights[:n]]
        self._b = [None if b is None else np.ascontiguousarray(b, np.float32)
                   for b in (biases[:n] if biases is not None else [None] * n)]
        wp = (POINTER(c_float) * n)(*[w.ctypes.data_as(POINTER(c_float)) for w in self._w])
        bp = (POINTER(c_float) * n)(*[(b.ctypes.data_as(POINTER(c_float)) if b is not None
                                        else POINTER(c_float)()) for b in self._b])
        h = c_void_p()
        check("nst_create", lib().nst_create(byref(self.desc), wp, bp, PRECISIONS[precision], byref(h)))
        self._h = h
        self.ws_limit = ws_limit
        self.tile_batch = tile_batch
        self.resident = resident
        self._ws = {}
        strides, s = [], 1
        for i in range(n):
            strides.append(s)
            if (self.desc.pool_after >> i) & 1:
                s *= 2
        self.strides = strides

    def close(self):
        if getattr(self, "_h", None):
            lib().nst_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- profiling
    def profile(self, enable: bool):
        check("nst_profile", lib().nst_profile(self._h, int(enable)))

    def profile_read(self):
        """Per-kernel [name, launches, ms, flops, bytes], longest total time first."""
        from ._lib import KStat
        n = c_int(0)
        arr = (KStat * 256)()
        check("nst_profile_read", lib().nst_profile_read(self._h, arr, 256, byref(n)))
        return [dict(name=k.name.decode(), launches=k.launches, ms=k.ms, flops=k.flops, bytes=k.bytes)
                for k in arr[: min(n.value, 256)]]

    # --------------------------------------------------------------- helpers
    def gram_sizes(self):
        return [self.convs[i][1] for i in self.style]

    def split_grams(self, flat: torch.Tensor):
        out, o = [], 0
        for c in self.gram_sizes():
            out.append(flat[o:o + c * c].view(c, c))
            o += c * c
        return out

    def workspace(self, H, W, T, m):
        """Device workspace: the largest tile batch (at most tile_batch) that fits in
        ws_limit, or a slot for every tile when the context is resident."""
        key = (H, W, T, m)
        if key not in self._ws:
            nt = len(plan(self.desc, H, W, T, m))
            b = nt if self.resident else max(1, min(self.tile_batch, nt))
            nbytes = workspace_bytes(self.desc, self.precision, H, W, T, m, b)
            if self.resident and nbytes > self.ws_limit:
                raise MemoryError(f"resident workspace {nbytes} B exceeds ws_limit {self.ws_limit} B")
            while b > 1 and nbytes > self.ws_limit:
                b -= 1
                nbytes = workspace_bytes(self.desc, self.precision, H, W, T, m, b)
            self._ws = {}
            self._ws = {key: torch.empty(nbytes, dtype=torch.uint8, device=self.device)}
        return self._ws[key]

    def _img(self, x: torch.Tensor):
        if x.dim() == 4:
            x = x[0]
        assert x.dim() == 3 and x.shape[0] == 3 and x.dtype == torch.float32 and x.is_cuda
        return x.contiguous()

    # ------------------------------------------------------------ entry points
    def style_grams(self, s: torch.Tensor, T: int, m: int) -> torch.Tensor:
        s = self._img(s)
        H, W = s.shape[1:]
        g = torch.empty(sum(c * c for c in self.gram_sizes()), dtype=torch.float64, device=self.device)
        ws = self.workspace(H, W, T, m)
        check("nst_style_grams", lib().nst_style_grams(self._h, _ptr(s), H, W, T, m, _ptr(g), _ptr(ws),
                                                       ws.numel(), _stream(self.device)))
        return g

    def style_stats(self, s: torch.Tensor, T: int, m: int):
        """(Grams, channel means) of the style layers of image s (nst_style_stats)."""
        s = self._img(s)
        H, W = s.shape[1:]
        g = torch.empty(sum(c * c for c in self.gram_sizes()), dtype=torch.float64, device=self.device)
        mu = torch.empty(sum(self.gram_sizes()), dtype=torch.float64, device=self.device)
        ws = self.workspace(H, W, T, m)
        check("nst_style_stats", lib().nst_style_stats(self._h, _ptr(s), H, W, T, m, _ptr(g), _ptr(mu), _ptr(ws),
                                                       ws.numel(), _stream(self.device)))
        return g, mu

    def split_means(self, flat: torch.Tensor):
        out, o = [], 0
        for c in self.gram_sizes():
            out.append(flat[o:o + c])
            o += c
        return out

    def layer_feats(self, img: torch.Tensor, T: int, m: int, conv: int) -> torch.Tensor:
        img = self._img(img)
        H, W = img.shape[1:]
        s = self.strides[conv]
        f = torch.empty((H // s, W // s, self.convs[conv][1]), dtype=torch.float32, device=self.device)
        ws = self.workspace(H, W, T, m)
        check("nst_layer_feats", lib().nst_layer_feats(self._h, _ptr(img), H, W, T, m, conv, _ptr(f), _ptr(ws),
                                                       ws.numel(), _stream(self.device)))
        return f

    def content_feats(self, c: torch.Tensor, T: int, m: int) -> torch.Tensor:
        c = self._img(c)
        H, W = c.shape[1:]
        s = self.strides[self.content]
        f = torch.empty((H // s, W // s, self.convs[self.content][1]), dtype=torch.float32, device=self.device)
        ws = self.workspace(H, W, T, m)
        check("nst_content_feats", lib().nst_content_feats(self._h, _ptr(c), H, W, T, m, _ptr(f), _ptr(ws),
                                                           ws.numel(), _stream(self.device)))
        return f

    def loss_grad(self, x, target_grams, content_feats, w_style, alpha, T, m, flags=NST_BOTH,
                  grams_x=None, want_energy=True, grad=None, ms: MeanStdTerms | None = None):
        """Returns (energy list [E, E_content, E_style...] or None, grams_x, grad or None).
        With ms (MeanStdTerms) the style terms are the augmented ones of Eq. 5 and ms.means_x
        receives the channel means of x."""
        x = self._img(x)
        H, W = x.shape[1:]
        if grams_x is None:
            grams_x = torch.empty(sum(c * c for c in self.gram_sizes()), dtype=torch.float64, device=self.device)
        if (flags & NST_STEP2) and grad is None:
            grad = torch.empty_like(x)
        ws = self.workspace(H, W, T, m)
        ns = len(self.style)
        wst = (c_double * max(ns, 1))(*[float(v) for v in w_style])
        en = (c_double * (2 + ns))()
        cf = _ptr(content_feats) if content_feats is not None else c_void_p()
        if self.resident:
            flags |= NST_RESIDENT
        if ms is None:
            check("nst_loss_grad", lib().nst_loss_grad(
                self._h, _ptr(x), H, W, _ptr(target_grams), cf, wst, float(alpha), T, m, flags, _ptr(grams_x),
                en if want_energy else None, _ptr(grad) if grad is not None else c_void_p(), _ptr(ws), ws.numel(),
                _stream(self.device)))
        else:
            st = ms._struct(ns)
            check("nst_loss_grad_ms", lib().nst_loss_grad_ms(
                self._h, _ptr(x), H, W, _ptr(target_grams), cf, wst, float(alpha), byref(st), T, m, flags,
                _ptr(grams_x), en if want_energy else None, _ptr(grad) if grad is not None else c_void_p(),
                _ptr(ws), ws.numel(), _stream(self.device)))
        energy = list(en) if want_energy else None
        return energy, grams_x, (grad if flags & NST_STEP2 else None)


class StyleEnergy(torch.autograd.Function):
    """image -> E(image) (Eq. 1-3).  forward runs Step 1 of Algorithm 1; backward runs
    Step 2 from the saved Grams, recomputing each tile's activations."""

    @staticmethod
    def forward(ctx, x, nst: Context, target_grams, content_feats, w_style, alpha, T, m, ms=None):
        if ms is not None:
            ms = MeanStdTerms(ms.w_mean, ms.w_std, ms.target_means)
        energy, grams_x, _ = nst.loss_grad(x, target_grams, content_feats, w_style, alpha, T, m, flags=NST_STEP1,
                                           ms=ms)
        ctx.save_for_backward(x, grams_x)
        ctx.args = (nst, target_grams, content_feats, w_style, alpha, T, m, ms)
        return torch.tensor(energy[0], dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, g_e):
        x, grams_x = ctx.saved_tensors
        nst, target_grams, content_feats, w_style, alpha, T, m, ms = ctx.args
        _, _, grad = nst.loss_grad(x, target_grams, content_feats, w_style, alpha, T, m, flags=NST_STEP2,
                                   grams_x=grams_x, want_energy=False, ms=ms)
        return g_e.to(grad.dtype) * grad, None, None, None, None, None, None, None, None


__all__ = ["Context", "StyleEnergy", "MeanStdTerms", "vgg19_desc", "min_halo", "plan", "workspace_bytes", "NST_STEP1",
           "NST_STEP2", "NST_BOTH", "NST_STRICT_HALO", "NST_CHECK_FINITE", "NST_RESIDENT"]

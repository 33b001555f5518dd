"""Multiscale style transfer (Algorithm 2) driven by L-BFGS over the localized loss and
gradient of Algorithm 1 (``StyleEnergy``).

For scale s = 1 .. n the content and style images are downscaled by 2^(n - s) (2 x 2 box
averages, repeated); the first scale starts from the downscaled content image, each later
one from the previous result upscaled by 2 (bilinear, to the next scale's exact size).
At each scale ``iterations[s]`` L-BFGS iterations run with a history of ``history[s]``
gradients; every iteration evaluates the energy and its gradient once, through
libnst's kernels (the optimiser's own vector updates are PyTorch tensor arithmetic).

Schedules (Sec. 5.2): SPST runs 600 iterations at the first scale and 300 at each later
one; SPST-fast divides the count by 3 from one scale to the next with a floor of 30
(600, 200, 66, 30 for four scales).  The history is 100 at the first scale and 10 after
it.  ``cpu_last`` keeps the image and the optimiser's history in host memory at the last
scale and moves only the evaluation to the GPU, as the paper does for its largest images.
"""
from __future__ import annotations

import time

import torch
import torch.nn.functional as F

from .nst import Context, MeanStdTerms, StyleEnergy


def iteration_schedule(n_scales: int, fast: bool = False, first: int = 600, later: int = 300,
                       floor: int = 30):
    """L-BFGS iterations per scale: SPST (first, later, later, ...) or SPST-fast (first,
    then a third of the previous count, at least ``floor``)."""
    if n_scales < 1:
        raise ValueError("n_scales must be >= 1")
    if not fast:
        return [first] + [later] * (n_scales - 1)
    its = [first]
    for _ in range(n_scales - 1):
        its.append(max(floor, its[-1] // 3))
    return its


def history_schedule(n_scales: int, first: int = 100, later: int = 10):
    return [first] + [later] * (n_scales - 1)


def scale_sizes(H: int, W: int, n_scales: int):
    """(h, w) of each scale, coarsest first: halved (floor) n_scales - s times."""
    out = []
    for s in range(n_scales):
        h, w = H, W
        for _ in range(n_scales - 1 - s):
            h, w = h // 2, w // 2
        out.append((h, w))
    return out


def downscale(img: torch.Tensor, times: int) -> torch.Tensor:
    """2 x 2 box average (floor size) applied ``times`` times to a 3 x H x W image."""
    for _ in range(times):
        img = F.avg_pool2d(img[None], 2, 2)[0]
    return img.contiguous()


def upscale(img: torch.Tensor, size) -> torch.Tensor:
    """Bilinear upscaling of a 3 x h x w image to ``size`` = (H, W)."""
    return F.interpolate(img[None], size=tuple(size), mode="bilinear", align_corners=False)[0].contiguous()


def style_transfer(ctx: Context, content: torch.Tensor, style: torch.Tensor, n_scales: int,
                   iterations=None, history=None, T: int = 1024, m: int | None = None, w_style=None,
                   alpha: float = 1.0, w_mean=None, w_std=None, cpu_last: bool = False, callback=None):
    """Algorithm 2.  content, style: 3 x H x W float32 on the context's GPU.  Returns the
    final image (3 x H x W float32, on the GPU) and per-scale records
    {size, iterations, evaluations, E_first, E_last, seconds}."""
    return _multiscale(ctx, content, style, None, content.shape[1:], n_scales, iterations, history, T, m,
                       w_style, alpha, w_mean, w_std, cpu_last, callback)


def texture_synthesis(ctx: Context, texture: torch.Tensor, H: int, W: int, n_scales: int, iterations=None,
                      history=None, T: int = 1024, m: int | None = None, w_style=None, w_mean=None,
                      w_std=None, seed: int = 0, cpu_last: bool = False, callback=None):
    """UHR texture synthesis (Sec. 6.2): the style term alone (no content image, alpha = 0),
    the same multiscale procedure, starting at the coarsest scale from white noise
    (uniform in [0, 1], drawn from a generator seeded with ``seed``).  The texture
    exemplar is downscaled like a style image; the output is H x W."""
    h0, w0 = scale_sizes(H, W, n_scales)[0]
    gen = torch.Generator(device=texture.device)
    gen.manual_seed(seed)
    x0 = torch.rand((3, h0, w0), generator=gen, device=texture.device, dtype=torch.float32)
    return _multiscale(ctx, None, texture, x0, (H, W), n_scales, iterations, history, T, m, w_style, 0.0,
                       w_mean, w_std, cpu_last, callback)


def _multiscale(ctx, content, style, x0, size, n_scales, iterations, history, T, m, w_style, alpha, w_mean,
                w_std, cpu_last, callback):
    from . import min_halo
    if m is None:
        m = min_halo(ctx.desc)
    ns = len(ctx.style)
    w_style = [1.0 / ns] * ns if w_style is None else list(w_style)
    iterations = iteration_schedule(n_scales) if iterations is None else list(iterations)
    history = history_schedule(n_scales) if history is None else list(history)
    if len(iterations) != n_scales or len(history) != n_scales:
        raise ValueError("one iteration count and one history size per scale")
    use_ms = w_mean is not None or w_std is not None
    sizes = scale_sizes(size[0], size[1], n_scales)
    x = None
    records = []
    for s in range(n_scales):
        k = n_scales - 1 - s
        u = downscale(content, k) if content is not None else None
        v = downscale(style, k)
        if use_ms:
            gt, mu = ctx.style_stats(v, T, m)
            ms = MeanStdTerms(w_mean if w_mean is not None else [0.0] * ns,
                              w_std if w_std is not None else [0.0] * ns, mu)
        else:
            gt, ms = ctx.style_grams(v, T, m), None
        fc = ctx.content_feats(u, T, m) if u is not None and ctx.content >= 0 and alpha != 0.0 else None
        if s == 0:
            x = u.clone() if x0 is None else x0.clone()
        else:
            x = upscale(x.detach(), sizes[s])
        on_cpu = cpu_last and s == n_scales - 1
        xv = (x.cpu() if on_cpu else x).requires_grad_(True)
        opt = torch.optim.LBFGS([xv], lr=1.0, max_iter=iterations[s], history_size=history[s],
                                tolerance_grad=0.0, tolerance_change=0.0)
        energies = []

        def closure():
            opt.zero_grad()
            xg = xv.to(style.device) if on_cpu else xv
            if on_cpu:
                xg = xg.detach().requires_grad_(True)
            e = StyleEnergy.apply(xg, ctx, gt, fc, w_style, alpha, T, m, ms)
            e.backward()
            if on_cpu:
                xv.grad = xg.grad.cpu()
            energies.append(float(e))
            if callback is not None:
                callback(s, len(energies), float(e))
            return e

        t0 = time.perf_counter()
        if iterations[s] > 0:
            opt.step(closure)
        torch.cuda.synchronize()
        x = xv.detach().to(style.device)
        records.append({"size": tuple(x.shape[1:]), "iterations": iterations[s], "evaluations": len(energies),
                        "E_first": energies[0] if energies else None, "E_last": energies[-1] if energies else None,
                        "seconds": time.perf_counter() - t0})
    return x, records

"""Two-pass localized loss and gradient, FP64 (Algorithm 1; TEST INFRASTRUCTURE ONLY).

Step 1: for each block, run the network on its window without keeping anything
for a backward pass; add the owned features' V^T V to the global Gram sums, their
channel sums to the global means, and the owned content residual to the content
energy.  Divide by the whole-image n_p of each layer; std = (diag G - mean^2)^(1/2).

Step 2: for each block, run the network on its window again, seed the style
gradients with the *global* Step 1 statistics (Table 1, Gram row) and the
content gradient (Table 1, MSE row) at every window feature, backpropagate to
the window image and copy the block's own pixels into the whole-image gradient
(no accumulation between blocks).

The content energy is summed in Step 1 over owned features; the paper adds it
in Step 2, which gives the same value because the owned features are the same.
"""
from __future__ import annotations

import numpy as np

from .loss import MeanStd, backward, content_seed, energy_terms, forward, last_needed, ms_seed, style_seed
from .net import NetSpec
from .plan import make_plan


def _plan(net, h, w, t, m):
    return make_plan(h, w, t, m, net.strides(), net.align())


def _local(tile, i, strides):
    s = strides[i]
    r0, r1, c0, c1 = tile.own[i]
    oy, ox = tile.ey0 // s, tile.ex0 // s
    return r0 - oy, r1 - oy, c0 - ox, c1 - ox


def step1(net: NetSpec, img, ws, bs, t, m, f_c=None, alpha=0.0, upto=None, means=None):
    """Global Grams (normalized) of img and the owned-feature content energy.  With a
    list ``means``, the global channel means of the style layers are appended to it."""
    h, w = img.shape[1:]
    strides = net.strides()
    if upto is None:
        upto = max(net.style)
        if f_c is not None and alpha != 0.0:
            upto = max(upto, net.content)
    sums = [np.zeros((net.convs[i][1],) * 2) for i in net.style]
    csum = [np.zeros(net.convs[i][1]) for i in net.style]
    e_c = 0.0
    for tile in _plan(net, h, w, t, m):
        acts = forward(net, img[:, tile.ey0:tile.ey1, tile.ex0:tile.ex1], ws, bs, upto=upto)
        for k, i in enumerate(net.style):
            r0, r1, c0, c1 = _local(tile, i, strides)
            v = acts[i][:, r0:r1, c0:c1].reshape(acts[i].shape[0], -1)
            sums[k] += v @ v.T
            csum[k] += v.sum(axis=1)
        if f_c is not None and alpha != 0.0:
            i = net.content
            r0, r1, c0, c1 = _local(tile, i, strides)
            gr0, gr1, gc0, gc1 = tile.own[i]
            diff = acts[i][:, r0:r1, c0:c1] - f_c[:, gr0:gr1, gc0:gc1]
            e_c += float(alpha * np.sum(diff * diff))
    grams = []
    for k, i in enumerate(net.style):
        s = strides[i]
        grams.append(sums[k] / float((h // s) * (w // s)))
        if means is not None:
            means.append(csum[k] / float((h // s) * (w // s)))
    return grams, e_c


def tiled_style_grams(net: NetSpec, s_img, ws, bs, t, m):
    return step1(net, s_img, ws, bs, t, m)[0]


def tiled_style_stats(net: NetSpec, s_img, ws, bs, t, m):
    """Grams and channel means of the style image, block by block."""
    means = []
    grams = step1(net, s_img, ws, bs, t, m, means=means)[0]
    return grams, means


def tiled_content_features(net: NetSpec, c_img, ws, bs, t, m):
    h, w = c_img.shape[1:]
    strides = net.strides()
    i = net.content
    s = strides[i]
    out = np.zeros((net.convs[i][1], h // s, w // s))
    for tile in _plan(net, h, w, t, m):
        acts = forward(net, c_img[:, tile.ey0:tile.ey1, tile.ex0:tile.ex1], ws, bs, upto=i)
        r0, r1, c0, c1 = _local(tile, i, strides)
        gr0, gr1, gc0, gc1 = tile.own[i]
        out[:, gr0:gr1, gc0:gc1] = acts[i][:, r0:r1, c0:c1]
    return out


def step2(net: NetSpec, x, ws, grams_x, grams_t, f_c, w_style, alpha, t, m, bs, only=None, ms=None):
    """Step 2 of Algorithm 1.  ``only``: indices of the plan's tiles to process (the
    gradient elsewhere is left at zero).  ``ms``: mean/std terms of Eq. 5 with the
    global means of x set."""
    h, w = x.shape[1:]
    strides = net.strides()
    grad = np.zeros((3, h, w))
    n_ps = [(h // strides[i]) * (w // strides[i]) for i in net.style]
    use_c = net.content is not None and alpha != 0.0
    plan = _plan(net, h, w, t, m)
    for ti, tile in enumerate(plan):
        if only is not None and ti not in only:
            continue
        acts = forward(net, x[:, tile.ey0:tile.ey1, tile.ex0:tile.ex1], ws, bs, upto=last_needed(net))
        seeds = {}
        for k, i in enumerate(net.style):
            seeds[i] = style_seed(acts[i], grams_x[k], grams_t[k], w_style[k], n_ps[k])
            if ms is not None:
                seeds[i] = seeds[i] + ms_seed(acts[i], grams_x[k], grams_t[k], ms, k, n_ps[k])
        if use_c:
            i = net.content
            s = strides[i]
            hl, wl = acts[i].shape[1:]
            oy, ox = tile.ey0 // s, tile.ex0 // s
            cs = content_seed(acts[i], f_c[:, oy:oy + hl, ox:ox + wl], alpha)
            seeds[i] = seeds.get(i, 0.0) + cs
        gw = backward(net, acts, seeds, ws)
        grad[:, tile.by0:tile.by1, tile.bx0:tile.bx1] = \
            gw[:, tile.by0 - tile.ey0:tile.by1 - tile.ey0, tile.bx0 - tile.ex0:tile.bx1 - tile.ex0]
    return grad


def tiled_loss_grad(net: NetSpec, x, ws, bs, grams_t, f_c, w_style, alpha, t, m,
                    grams_fixed=None, want_grad=True, ms: MeanStd | None = None):
    """Algorithm 1.  ``grams_fixed`` replaces the Step 1 Grams in Step 2 (for the
    fixed-statistics invariant).  ``ms``: the mean/std terms of Eq. 5 (weights and the
    style image's means; the means of x come from Step 1)."""
    x = np.asarray(x, np.float64)
    means_x = []
    grams_x, e_c = step1(net, x, ws, bs, t, m, f_c=f_c, alpha=alpha, means=means_x)
    msx = None if ms is None else ms.with_x(means_x)
    terms = energy_terms(grams_x, grams_t, w_style, e_c, msx)
    terms["grams"] = grams_x
    terms["means"] = means_x
    if not want_grad:
        return terms, None
    g_use = grams_x if grams_fixed is None else grams_fixed
    return terms, step2(net, x, ws, g_use, grams_t, f_c, w_style, alpha, t, m, bs, ms=msx)

"""Whole-image transfer energy and its hand-derived gradient, FP64 (TEST INFRASTRUCTURE ONLY).

Definitions followed (Sec. 3.1, Sec. 4.2):

* features V^L(x): post-ReLU activation of the named conv, reshaped n_p x n_c
* Gram (Sec. 3.1):            G^L(x) = V^T V / n_p, n_p = h_L * w_L of the whole image
* style energy (Eq. 2-3):     E_style = sum_L w_L || G^L(x) - G^L(v) ||_F^2
* content energy (Sec. 3.1):  E_content = lambda_c || V^{Lc}(x) - V^{Lc}(u) ||^2
* transfer energy (Eq. 1):    E = E_content + E_style
* feature gradients (Table 1): MSE row  dE/dV = 2 (V - V_ref) (times lambda_c);
  Gram row written without assuming symmetry, dE/dV = (2 w / n_p) V (D + D^T)
  with D = G - G_ref, which equals the printed (4 w / n_p) V D when D is symmetric.
* backward: reverse layer loop with ReLU'(0) = 0, max-pool routing to the
  first maximum (average pools: a quarter to each input), conv adjoint.

Augmented style loss (Sec. 3.2, Eq. 5; Table 1 rows 3-4; Algorithm 1 Step 1):

* mean(V) and std(V): spatial mean and (population) standard deviation per channel;
  the statistics of x are formed from the Gram diagonal and the mean,
  std = (diag(G) - mean^2)^(1/2), as Algorithm 1 Step 1 does;
* E_style^L gains w'_L ||mean(V) - mu_ref||^2 + w''_L ||std(V) - sigma_ref||^2, with
  the reference statistics of the style image (sigma_ref from its Gram and mean);
* seeds: (2 w' / n_p)(mean - mu_ref) at every pixel and
  (2 w'' / n_p)(V - mean)(std - sigma_ref) / std, taken as 0 on channels with
  std = 0 (constant channel: std is not differentiable there).

Arrays are C x H x W float64; V in the paper's n_p x n_c orientation is the
transpose of the C x (H W) reshape used here.
"""
from __future__ import annotations

import numpy as np

from .net import NetSpec
from .ops import conv3x3, conv3x3_adjoint, pool2, pool2_backward, relu


def last_needed(net: NetSpec) -> int:
    return max(list(net.style) + ([net.content] if net.content is not None else []))


def forward(net: NetSpec, x: np.ndarray, ws, bs, upto: int | None = None):
    """Post-ReLU activation A_i of every conv i <= upto (pre-pool)."""
    if upto is None:
        upto = last_needed(net)
    a = np.asarray(x, np.float64)
    acts = []
    for i in range(upto + 1):
        z = conv3x3(a, ws[i], bs[i])
        ai = relu(z)
        acts.append(ai)
        a = pool2(ai, net.avg_pool) if i in net.pool_after else ai
    return acts


def gram(v: np.ndarray, n_p: int) -> np.ndarray:
    """G = V^T V / n_p for a C x h x w feature map (V is (h w) x C)."""
    c = v.shape[0]
    m = v.reshape(c, -1)
    return (m @ m.T) / float(n_p)


def channel_mean(v: np.ndarray, n_p: int) -> np.ndarray:
    """mean(V): the spatial mean of each channel of a C x h x w map (Sec. 3.2)."""
    return v.reshape(v.shape[0], -1).sum(axis=1) / float(n_p)


def std_from_stats(g: np.ndarray, mean: np.ndarray) -> np.ndarray:
    """std(V) = (diag(G) - mean(V)^2)^(1/2) (Algorithm 1 Step 1); a negative radicand,
    which only rounding can produce, is taken as 0."""
    return np.sqrt(np.maximum(np.diag(g) - mean * mean, 0.0))


def content_features(net: NetSpec, c_img: np.ndarray, ws, bs) -> np.ndarray:
    assert net.content is not None
    return forward(net, c_img, ws, bs, upto=net.content)[net.content]


def style_grams(net: NetSpec, s_img: np.ndarray, ws, bs):
    acts = forward(net, s_img, ws, bs, upto=max(net.style))
    return [gram(acts[i], acts[i].shape[1] * acts[i].shape[2]) for i in net.style]


def style_stats(net: NetSpec, s_img: np.ndarray, ws, bs):
    """Grams and channel means of the style image's style layers (Algorithm 1 Require)."""
    acts = forward(net, s_img, ws, bs, upto=max(net.style))
    grams, means = [], []
    for i in net.style:
        n_p = acts[i].shape[1] * acts[i].shape[2]
        grams.append(gram(acts[i], n_p))
        means.append(channel_mean(acts[i], n_p))
    return grams, means


def energy_terms(grams_x, grams_t, w_style, e_content, ms=None):
    """Per-layer style terms w_L ||G_x - G_t||_F^2 and the total (Eq. 1-3).  With ``ms``
    (a MeanStd), each layer's term is the augmented one of Eq. 5, whose three parts are
    also returned (E_gram, E_mean, E_std)."""
    e_gram = [float(wl * np.sum((gx - gt) ** 2)) for gx, gt, wl in zip(grams_x, grams_t, w_style)]
    out = {"E_gram": e_gram}
    e_style = list(e_gram)
    if ms is not None:
        out["E_mean"], out["E_std"] = [], []
        for k, (gx, gt) in enumerate(zip(grams_x, grams_t)):
            em = float(ms.w_mean[k] * np.sum((ms.means_x[k] - ms.means_t[k]) ** 2))
            sx, st = std_from_stats(gx, ms.means_x[k]), std_from_stats(gt, ms.means_t[k])
            es = float(ms.w_std[k] * np.sum((sx - st) ** 2))
            out["E_mean"].append(em)
            out["E_std"].append(es)
            e_style[k] += em + es
    out.update({"E": float(e_content + sum(e_style)), "E_content": float(e_content), "E_style": e_style})
    return out


class MeanStd:
    """Weights and statistics of the mean and std terms of Eq. 5 (per style layer)."""

    def __init__(self, w_mean, w_std, means_t, means_x=None):
        self.w_mean, self.w_std, self.means_t, self.means_x = list(w_mean), list(w_std), means_t, means_x

    def with_x(self, means_x):
        return MeanStd(self.w_mean, self.w_std, self.means_t, means_x)


def style_seed(v: np.ndarray, g: np.ndarray, g_t: np.ndarray, w_l: float, n_p: int) -> np.ndarray:
    """Gram row of Table 1 on a C x h x w map: (2 w / n_p) V (D + D^T), D = G - G_t."""
    c = v.shape[0]
    d = g - g_t
    return (((2.0 * w_l / n_p) * (d + d.T)) @ v.reshape(c, -1)).reshape(v.shape)


def mean_seed(shape, mean: np.ndarray, mean_t: np.ndarray, w1: float, n_p: int) -> np.ndarray:
    """Mean row of Table 1 times w': (2 w' / n_p)(mean(V) - mu_ref) at every pixel."""
    return np.broadcast_to(((2.0 * w1 / n_p) * (mean - mean_t))[:, None, None], shape).copy()


def std_seed(v: np.ndarray, mean: np.ndarray, std: np.ndarray, std_t: np.ndarray, w2: float,
             n_p: int) -> np.ndarray:
    """Std row of Table 1 times w'': (2 w'' / n_p)(V - mean)(std - sigma_ref) / std,
    0 on channels whose std is 0."""
    safe = np.where(std > 0.0, std, 1.0)
    ratio = np.where(std > 0.0, (std - std_t) / safe, 0.0)
    return (2.0 * w2 / n_p) * (v - mean[:, None, None]) * ratio[:, None, None]


def ms_seed(v, g, g_t, ms, k, n_p):
    """Mean and std seeds of style layer k (Table 1 rows 3-4)."""
    mean, mean_t = ms.means_x[k], ms.means_t[k]
    out = mean_seed(v.shape, mean, mean_t, ms.w_mean[k], n_p)
    return out + std_seed(v, mean, std_from_stats(g, mean), std_from_stats(g_t, mean_t), ms.w_std[k], n_p)


def content_seed(v: np.ndarray, f_ref: np.ndarray, alpha: float) -> np.ndarray:
    """MSE row of Table 1 times lambda_c: 2 alpha (V - V_ref)."""
    return 2.0 * alpha * (v - f_ref)


def backward(net: NetSpec, acts, seeds: dict, ws, record: dict | None = None) -> np.ndarray:
    """Reverse pass: seeds[i] is dE/dA_i added at conv i's ReLU output; returns dE/dx.
    With ``record``, stores dE/dA_i (seeds included) under ("dA", i) and the gradient
    reaching a pool's output under ("dP", i) for the pool after conv i."""
    top = len(acts) - 1
    g = None
    for i in range(top, -1, -1):
        da = np.zeros_like(acts[i]) if g is None else g
        if i in seeds:
            da = da + seeds[i]
        if record is not None:
            record[("dA", i)] = da
        dz = np.where(acts[i] > 0.0, da, 0.0)          # ReLU'(0) = 0
        dx = conv3x3_adjoint(dz, ws[i])
        if i > 0 and (i - 1) in net.pool_after:
            if record is not None:
                record[("dP", i - 1)] = dx
            g = pool2_backward(dx, acts[i - 1], net.avg_pool)
        else:
            g = dx
    return g


def loss_grad(net: NetSpec, x, ws, bs, grams_t, f_c, w_style, alpha, want_grad=True, record=None,
              ms: MeanStd | None = None):
    """Whole-image E (with terms), Grams of x and dE/dx (Eq. 1-3, Table 1; with ``ms``
    the augmented style loss of Eq. 5, the means of x returned under "means").
    ``record`` (a dict) receives the activations under ("A", i) and the adjoints of
    ``backward``."""
    acts = forward(net, x, ws, bs)
    grams_x, n_ps, means_x = [], [], []
    for i in net.style:
        n_p = acts[i].shape[1] * acts[i].shape[2]
        n_ps.append(n_p)
        grams_x.append(gram(acts[i], n_p))
        means_x.append(channel_mean(acts[i], n_p))
    e_c = 0.0
    if net.content is not None and alpha != 0.0:
        e_c = float(alpha * np.sum((acts[net.content] - f_c) ** 2))
    msx = None if ms is None else ms.with_x(means_x)
    terms = energy_terms(grams_x, grams_t, w_style, e_c, msx)
    terms["grams"] = grams_x
    terms["means"] = means_x
    if not want_grad:
        return terms, None
    seeds = {}
    for k, i in enumerate(net.style):
        seeds[i] = style_seed(acts[i], grams_x[k], grams_t[k], w_style[k], n_ps[k])
        if msx is not None:
            seeds[i] = seeds[i] + ms_seed(acts[i], grams_x[k], grams_t[k], msx, k, n_ps[k])
    if net.content is not None and alpha != 0.0:
        cs = content_seed(acts[net.content], f_c, alpha)
        seeds[net.content] = seeds.get(net.content, 0.0) + cs
    if record is not None:
        for i, a in enumerate(acts):
            record[("A", i)] = a
    return terms, backward(net, acts, seeds, ws, record)

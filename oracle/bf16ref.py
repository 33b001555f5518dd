"""BF16-storage reference of the transfer energy and its gradient (TEST INFRASTRUCTURE ONLY).

This is the FP64 definition of ``loss.py`` (Sec. 3.1, Eq. 1-3, Table 1, whole image)
with one departure: a value is rounded to the nearest BF16 number (ties to even) at
each point where a BF16 evaluation stores it, namely

* the operands of the convolutions: the network weights and the input image;
* every post-ReLU activation A_i.  The Gram matrices, the max pooling and the ReLU masks
  of the backward pass read these stored values; an average pool's output;
* the residual operand (2 w_l / n_p)(D_l + D_l^T) of each style layer (Table 1, Gram row),
  with the augmented loss (Eq. 5) plus diag(r), r = (2 w'' / n_p)(std - std_ref) / std, the
  part of the std row that multiplies V; the per-channel rest of the mean and std rows,
  (2 w' / n_p)(mean - mean_ref) - r mean, is added unrounded;
* every stored adjoint: the masked dE/dZ_i of each conv, and the gradient that reaches
  a max pool's output before it is routed back.

The content difference V - F_c (the content energy and the MSE-row seed) is taken from
the unrounded activation, which a BF16 evaluation keeps in FP32.  Biases stay as given.
All arithmetic is FP64, in the same order as ``loss.py``; nothing emulates blocking or
accumulation order.  With ``q`` the identity every step is the same FP64 operation as
``loss.loss_grad``, so the two agree bit for bit.

It serves as the reference of BF16 runs: their Grams, energies and gradient differ from
it only by FP32-accumulation rounding (and what that rounding moves), whereas they differ
from the FP64 oracle by the BF16 storage rounding itself.
"""
from __future__ import annotations

import numpy as np

from .loss import channel_mean, energy_terms, gram, last_needed, std_from_stats
from .net import NetSpec
from .ops import conv3x3, conv3x3_adjoint, pool2, pool2_backward, relu


def round_bf16(a) -> np.ndarray:
    """Nearest BF16 value (8 significant bits, ties to even) of each FP64 element.

    a = m 2^e with 0.5 <= |m| < 1 (frexp); m 2^8 rounded to an integer (rint rounds
    halves to even) keeps 8 significant bits.  Values below the BF16 normal range
    (2^-126) are not treated specially; this path never produces them."""
    m, e = np.frexp(np.asarray(a, np.float64))
    return np.ldexp(np.rint(m * 256.0), e - 8)


def identity(a):
    return a


def forward(net: NetSpec, x, ws, bs, q=round_bf16, upto: int | None = None):
    """(stored, raw): stored[i] = q(relu(Z_i)), raw[i] = relu(Z_i), per conv i <= upto."""
    if upto is None:
        upto = last_needed(net)
    a = q(np.asarray(x, np.float64))
    stored, raw = [], []
    for i in range(upto + 1):
        z = conv3x3(a, q(np.asarray(ws[i], np.float64)), bs[i])
        r = relu(z)
        ai = q(r)
        stored.append(ai)
        raw.append(r)
        # a max pool picks a stored value; an average pool's mean is stored rounded
        if i in net.pool_after:
            a = q(pool2(ai, True)) if net.avg_pool else pool2(ai, False)
        else:
            a = ai
    return stored, raw


def backward(net: NetSpec, acts, seeds: dict, ws, q=round_bf16) -> np.ndarray:
    """Reverse pass with rounded adjoints; seeds[i] is added at conv i's ReLU output."""
    top = len(acts) - 1
    g = None
    for i in range(top, -1, -1):
        da = np.zeros_like(acts[i]) if g is None else g
        if i in seeds:
            da = da + seeds[i]
        dz = q(np.where(acts[i] > 0.0, da, 0.0))
        dx = conv3x3_adjoint(dz, q(np.asarray(ws[i], np.float64)))
        if i > 0 and (i - 1) in net.pool_after:
            g = pool2_backward(q(dx), acts[i - 1], net.avg_pool)
        else:
            g = dx
    return g


def ms_operands(g, g_t, mean, mean_t, w1, w2, n_p):
    """(r, b) of the mean and std rows of Table 1 written as V diag(r) + b:
    r = (2 w'' / n_p)(std - std_ref) / std (0 where std = 0), b = (2 w' / n_p)(mean - mean_ref) - r mean."""
    std, std_t = std_from_stats(g, mean), std_from_stats(g_t, mean_t)
    r = np.where(std > 0.0, (2.0 * w2 / n_p) * (std - std_t) / np.where(std > 0.0, std, 1.0), 0.0)
    return r, (2.0 * w1 / n_p) * (mean - mean_t) - r * mean


def loss_grad(net: NetSpec, x, ws, bs, grams_t, f_c, w_style, alpha, q=round_bf16, want_grad=True, ms=None):
    """Energy terms (with the Grams of x under "grams", the channel means under "means")
    and dE/dx, BF16 storage.  ``ms``: the mean/std terms of Eq. 5 (oracle.loss.MeanStd)."""
    acts, raw = forward(net, x, ws, bs, q)
    grams_x, n_ps, means_x = [], [], []
    for i in net.style:
        n_p = acts[i].shape[1] * acts[i].shape[2]
        n_ps.append(n_p)
        grams_x.append(gram(acts[i], n_p))
        means_x.append(channel_mean(acts[i], n_p))
    e_c = 0.0
    if net.content is not None and alpha != 0.0:
        e_c = float(alpha * np.sum((raw[net.content] - f_c) ** 2))
    msx = None if ms is None else ms.with_x(means_x)
    terms = energy_terms(grams_x, grams_t, w_style, e_c, msx)
    terms["grams"] = grams_x
    terms["means"] = means_x
    if not want_grad:
        return terms, None
    seeds = {}
    for k, i in enumerate(net.style):
        d = grams_x[k] - grams_t[k]
        dt = (2.0 * w_style[k] / n_ps[k]) * (d + d.T)
        b = None
        if msx is not None:
            r, b = ms_operands(grams_x[k], grams_t[k], means_x[k], msx.means_t[k], msx.w_mean[k], msx.w_std[k],
                               n_ps[k])
            dt = dt + np.diag(r)
        dt = q(dt)
        c = acts[i].shape[0]
        seeds[i] = (dt @ acts[i].reshape(c, -1)).reshape(acts[i].shape)
        if b is not None:
            seeds[i] = seeds[i] + b[:, None, None]
    if net.content is not None and alpha != 0.0:
        cs = 2.0 * alpha * (raw[net.content] - f_c)
        seeds[net.content] = seeds.get(net.content, 0.0) + cs
    return terms, backward(net, acts, seeds, ws, q)


def features(net: NetSpec, x, ws, bs, conv: int, q=round_bf16) -> np.ndarray:
    """Stored (rounded) post-ReLU features of one conv."""
    return forward(net, x, ws, bs, q, upto=conv)[0][conv]


def style_grams(net: NetSpec, s_img, ws, bs, q=round_bf16):
    acts, _ = forward(net, s_img, ws, bs, q, upto=max(net.style))
    return [gram(acts[i], acts[i].shape[1] * acts[i].shape[2]) for i in net.style]


def style_stats(net: NetSpec, s_img, ws, bs, q=round_bf16):
    acts, _ = forward(net, s_img, ws, bs, q, upto=max(net.style))
    n_ps = [acts[i].shape[1] * acts[i].shape[2] for i in net.style]
    return ([gram(acts[i], n) for i, n in zip(net.style, n_ps)],
            [channel_mean(acts[i], n) for i, n in zip(net.style, n_ps)])

"""Decision margins of the FP64 forward (TEST INFRASTRUCTURE ONLY).

The transfer energy is piecewise smooth in x: every ReLU (sign of its input) and
every 2x2 max pool (which input is largest) is a discrete decision.  A reduced-
precision evaluation whose rounding error exceeds a decision's margin may take the
other branch, and then its gradient legitimately differs from the FP64 one on the
receptive field of that unit.  This module lists the decisions whose margin is
below ``delta`` times the layer's RMS and marks, on the image grid, the union of
their dependency cones [s q - a, s q + b] (closed form of ``net.receptive_fields``),
so that a gradient comparison can be restricted to pixels that no fragile decision
can reach.
"""
from __future__ import annotations

import numpy as np

from .loss import last_needed
from .net import NetSpec, receptive_fields
from .ops import conv3x3, maxpool2


def fragile_decisions(net: NetSpec, x, ws, bs, delta: float):
    """List of (kind, conv index, q_y, q_x, margin/rms) with margin/rms < delta."""
    rf = receptive_fields(net)
    strides = net.strides()
    a = np.asarray(x, np.float64)
    out = []
    for i in range(last_needed(net) + 1):
        z = conv3x3(a, ws[i], bs[i])
        rms = float(np.sqrt(np.mean(z * z))) or 1.0
        m = np.abs(z).min(axis=0) / rms
        for qy, qx in np.argwhere(m < delta):
            out.append(("relu", i, int(qy), int(qx), float(m[qy, qx])))
        act = np.maximum(z, 0.0)
        if i in net.pool_after and i < last_needed(net):
            c, h, w = act.shape
            h2, w2 = h // 2, w // 2
            v = act[:, : 2 * h2, : 2 * w2].reshape(c, h2, 2, w2, 2).transpose(0, 1, 3, 2, 4).reshape(c, h2, w2, 4)
            srt = np.sort(v, axis=-1)
            arms = float(np.sqrt(np.mean(act * act))) or 1.0
            gap = (srt[..., 3] - srt[..., 2]) / arms
            gap[srt[..., 3] <= 0.0] = np.inf          # an all-zero window routes nothing
            g = gap.min(axis=0)
            for py, px in np.argwhere(g < delta):
                out.append(("pool", i, int(py), int(px), float(g[py, px])))
            a = maxpool2(act)
        else:
            a = act
    return out


def fragile_cone_mask(net: NetSpec, x, ws, bs, delta: float):
    """Boolean H x W mask of image pixels inside the cone of a fragile decision."""
    h, w = np.asarray(x).shape[1:]
    rf = receptive_fields(net)
    strides = net.strides()
    diff = np.zeros((h + 1, w + 1), np.int64)
    dec = fragile_decisions(net, x, ws, bs, delta)
    for kind, i, qy, qx, _ in dec:
        s, (a, b) = strides[i], rf[i]
        if kind == "relu":
            y0, y1, x0, x1 = s * qy - a, s * qy + b, s * qx - a, s * qx + b
        else:
            y0, y1, x0, x1 = 2 * s * qy - a, s * (2 * qy + 1) + b, 2 * s * qx - a, s * (2 * qx + 1) + b
        y0, x0 = max(y0, 0), max(x0, 0)
        y1, x1 = min(y1, h - 1), min(x1, w - 1)
        diff[y0, x0] += 1
        diff[y0, x1 + 1] -= 1
        diff[y1 + 1, x0] -= 1
        diff[y1 + 1, x1 + 1] += 1
    mask = np.cumsum(np.cumsum(diff, 0), 1)[:h, :w] > 0
    return mask, dec

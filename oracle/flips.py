"""Exact effect of flipping one near-boundary decision (TEST INFRASTRUCTURE ONLY).

The gradient is piecewise smooth in x; at a ReLU whose input is within rounding of 0,
or at a max pool whose two largest inputs are within rounding of each other, a
reduced-precision evaluation may take the other branch.  Given the FP64 forward and
adjoints (``loss.loss_grad(..., record=...)``), the change of dE/dx caused by flipping
one such decision alone is linear and local:

* ReLU at conv i, unit (c, y, x): dZ_i changes by -dA_i (pass -> block) or +dA_i
  (block -> pass) at that unit;
* pool after conv i, window (c, py, px): the pooled gradient dP moves from the first
  maximum to the runner-up;

and the change is carried to the image by the same reverse pass as ``loss.backward``
(conv adjoint, pool routing to the FP64 argmax, ReLU mask), restricted to an aligned
crop that contains the decision's dependency cone [s q - a, s q + b].

``explain`` subtracts, greedily from the most fragile decision on, the flip effects
that reduce a candidate gradient's deviation from the FP64 one where they act, and
returns what remains.  A correct reduced-precision backward leaves only rounding noise.
"""
from __future__ import annotations

import numpy as np

from .loss import last_needed
from .net import NetSpec, receptive_fields
from .ops import conv3x3, conv3x3_adjoint, maxpool2_backward

_ORDER = ((0, 0), (0, 1), (1, 0), (1, 1))


def fragile_units(net: NetSpec, acts, ws, bs, x, delta: float):
    """(margin/rms, kind, conv i, c, q_y, q_x) for every decision with margin/rms < delta."""
    out = []
    a = np.asarray(x, np.float64)
    for i in range(last_needed(net) + 1):
        z = conv3x3(a, ws[i], bs[i])
        rms = float(np.sqrt(np.mean(z * z))) or 1.0
        m = np.abs(z) / rms
        for c, y, xx in np.argwhere(m < delta):
            out.append((float(m[c, y, xx]), "relu", i, int(c), int(y), int(xx)))
        act = acts[i]
        if i in net.pool_after and i < last_needed(net):
            c_, h, w = act.shape
            h2, w2 = h // 2, w // 2
            v = np.stack([act[:, dy:2 * h2:2, dx:2 * w2:2] for dy, dx in _ORDER], -1)
            srt = np.sort(v, axis=-1)
            arms = float(np.sqrt(np.mean(act * act))) or 1.0
            gap = (srt[..., 3] - srt[..., 2]) / arms
            gap[srt[..., 3] <= 0.0] = np.inf
            for c, py, px in np.argwhere(gap < delta):
                out.append((float(gap[c, py, px]), "pool", i, int(c), int(py), int(px)))
            # next layer input
            a = v.max(axis=-1)
        else:
            a = act
    out.sort()
    return out


def _crop(net, i, qy, qx, span, shape):
    """Aligned image crop [Y0, Y1) x [X0, X1) that holds the cone of a decision at conv i
    covering feature rows/cols [qy, qy + span) with a 16 px margin."""
    h, w = shape
    rf = receptive_fields(net)
    s = net.strides()[i]
    a, b = rf[i]
    S = net.align()
    lo_y, hi_y = s * qy - a - 16, s * (qy + span - 1) + b + 17
    lo_x, hi_x = s * qx - a - 16, s * (qx + span - 1) + b + 17
    Y0, X0 = max(0, S * (lo_y // S)), max(0, S * (lo_x // S))
    Y1, X1 = min(h, S * (-(-hi_y // S))), min(w, S * (-(-hi_x // S)))
    return Y0, Y1, X0, X1


def _backward_from(net, acts_c, i, dz, ws):
    for j in range(i, -1, -1):
        dx = conv3x3_adjoint(dz, ws[j])
        if j == 0:
            return dx
        da = maxpool2_backward(dx, acts_c[j - 1]) if (j - 1) in net.pool_after else dx
        dz = np.where(acts_c[j - 1] > 0.0, da, 0.0)


def flip_effect(net: NetSpec, record, ws, unit, shape):
    """(Y0, Y1, X0, X1, delta_grad on that crop) for flipping one decision alone."""
    _, kind, i, c, qy, qx = unit
    strides = net.strides()
    span = 2 if kind == "pool" else 1
    qy0, qx0 = (2 * qy, 2 * qx) if kind == "pool" else (qy, qx)
    Y0, Y1, X0, X1 = _crop(net, i, qy0, qx0, span, shape)
    acts_c = []
    for j in range(i + 1):
        s = strides[j]
        r0, c0 = Y0 // s, X0 // s
        acts_c.append(record[("A", j)][:, r0:r0 + (Y1 - Y0) // s, c0:c0 + (X1 - X0) // s])
    s = strides[i]
    ly, lx = qy0 - Y0 // s, qx0 - X0 // s
    A = acts_c[i]
    dz = np.zeros_like(A)
    if kind == "relu" and i in net.pool_after and ("dP", i) in record and \
            qy // 2 < record[("dP", i)].shape[1] and qx // 2 < record[("dP", i)].shape[2]:
        # the unit feeds a max pool: flipping it can also move that window's maximum
        # (e.g. a unit that turns positive in an all-zero window takes the pooled gradient)
        py, px = qy // 2, qx // 2
        wy, wx = 2 * py - Y0 // s, 2 * px - X0 // s
        vals = [A[c, wy + dy, wx + dx] for dy, dx in _ORDER]
        new = list(vals)
        k_u = _ORDER.index((qy - 2 * py, qx - 2 * px))
        new[k_u] = 0.0 if vals[k_u] > 0.0 else np.finfo(np.float64).tiny
        dp = record[("dP", i)][c, py, px]
        da_unit = record[("dA", i)][c, qy, qx]
        for vv, sgn in ((vals, -1.0), (new, 1.0)):
            k1 = int(np.argmax(vv))
            for k in range(4):
                dy, dx = _ORDER[k]
                g = dp if k == k1 else 0.0
                if k == k_u:
                    g += da_unit - (dp if int(np.argmax(vals)) == k_u else 0.0)   # the unit's seed part
                if vv[k] > 0.0:
                    dz[c, wy + dy, wx + dx] += sgn * g
    elif kind == "relu":
        da = record[("dA", i)][c, qy, qx]
        dz[c, ly, lx] = -da if A[c, ly, lx] > 0.0 else da
    else:
        vals = [A[c, ly + dy, lx + dx] for dy, dx in _ORDER]
        k1 = int(np.argmax(vals))
        rest = [(v if k != k1 else -np.inf) for k, v in enumerate(vals)]
        k2 = int(np.argmax(rest))
        dp = record[("dP", i)][c, qy, qx]
        for k, sgn in ((k1, -1.0), (k2, 1.0)):
            dy, dx = _ORDER[k]
            if A[c, ly + dy, lx + dx] > 0.0:
                dz[c, ly + dy, lx + dx] += sgn * dp
    return Y0, Y1, X0, X1, _backward_from(net, acts_c, i, dz, ws)


def explain(net: NetSpec, x, ws, bs, record, g_ref, g_test, delta=1e-5, floor=1e-6, max_eval=400,
            passes=3):
    """Greedy flip correction of g_test - g_ref.  Returns (residual, accepted units).

    Candidates are the decisions with margin/rms < delta, most fragile first.  A flip is
    accepted when subtracting its effect shrinks the residual on the effect's support by
    30% or more; passes repeat until one accepts nothing (overlapping flips)."""
    r = np.asarray(g_test, np.float64) - g_ref
    shape = g_ref.shape[1:]
    acts = [record[("A", i)] for i in range(last_needed(net) + 1)]
    cands = fragile_units(net, acts, ws, bs, x, delta)
    thresh = floor * float(np.abs(g_ref).max())
    accepted, cache = [], {}
    for _ in range(passes):
        evals, gained = 0, False
        for u in cands:
            if u in accepted or evals >= max_eval:
                continue
            _, kind, i, c, qy, qx = u
            span = 2 if kind == "pool" else 1
            qy0, qx0 = (2 * qy, 2 * qx) if kind == "pool" else (qy, qx)
            Y0, Y1, X0, X1 = _crop(net, i, qy0, qx0, span, shape)
            rc = r[:, Y0:Y1, X0:X1]
            if float(np.abs(rc).max()) < thresh:
                continue
            evals += 1
            if u not in cache:
                cache[u] = flip_effect(net, record, ws, u, shape)[4]
            d = cache[u]
            sup = np.abs(d) > 1e-12 * max(float(np.abs(d).max()), 1e-300)
            before = float(np.linalg.norm(rc[sup]))
            after = float(np.linalg.norm((rc - d)[sup]))
            if before > 0 and after < 0.7 * before:
                r[:, Y0:Y1, X0:X1] = rc - d
                accepted.append(u)
                gained = True
        if not gained:
            break
    return r, accepted

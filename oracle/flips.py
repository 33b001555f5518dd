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

``flip_fit`` removes from a reduced-precision gradient's deviation the 0/1 combination
of these effects that fits it best (least squares, rounded), and returns what remains.
A correct reduced-precision backward leaves only rounding noise.
"""
from __future__ import annotations

import numpy as np

from .loss import last_needed
from .net import NetSpec, receptive_fields
from .ops import avgpool2, conv3x3, conv3x3_adjoint, pool2_backward

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
        if i in net.pool_after and i < last_needed(net) and net.avg_pool:
            a = avgpool2(act)            # an average pool takes no decision
        elif i in net.pool_after and i < last_needed(net):
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
        da = pool2_backward(dx, acts_c[j - 1], net.avg_pool) if (j - 1) in net.pool_after else dx
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
    if kind == "relu" and i in net.pool_after and not net.avg_pool and ("dP", i) in record and \
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


def flip_fit(net: NetSpec, x, ws, bs, record, g_ref, g_test, delta=1e-5, floor=1e-6):
    """Remove from g_test - g_ref the best 0/1 combination of near-tie flip effects.

    Candidates are the decisions whose FP64 margin is below ``delta`` times the RMS of
    their layer (``fragile_units``) and whose dependency crop carries a residual above
    ``floor`` times max|g_ref| (elsewhere a flip cannot be what the residual shows).  The
    coefficients c_u of their exact effects e_u (``flip_effect``) are fitted to the
    residual r by least squares, through the normal equations M c = b with
    M_uv = <e_u, e_v> and b_u = <e_u, r>, and rounded to 0 or 1 one at a time: the
    coefficient nearest to 0 or 1 is fixed there, the others are fitted again with the
    fixed ones subtracted, until every one is fixed (two candidates with the same effect,
    which plain rounding would split into halves, are then resolved one after the other).

    Returns (r - sum_u c_u e_u, the flipped units, the unrounded first fit)."""
    r = np.asarray(g_test, np.float64) - g_ref
    shape = g_ref.shape[1:]
    acts = [record[("A", i)] for i in range(last_needed(net) + 1)]
    thresh = floor * float(np.abs(g_ref).max())
    units, crops, effects = [], [], []
    for u in fragile_units(net, acts, ws, bs, x, delta):
        _, kind, i, c, qy, qx = u
        span = 2 if kind == "pool" else 1
        qy0, qx0 = (2 * qy, 2 * qx) if kind == "pool" else (qy, qx)
        Y0, Y1, X0, X1 = _crop(net, i, qy0, qx0, span, shape)
        if float(np.abs(r[:, Y0:Y1, X0:X1]).max()) < thresh:
            continue
        units.append(u)
        crops.append((Y0, Y1, X0, X1))
        effects.append(flip_effect(net, record, ws, u, shape)[4])
    n = len(units)
    M = np.zeros((n, n))
    b = np.zeros(n)
    for p in range(n):
        Y0, Y1, X0, X1 = crops[p]
        b[p] = float(np.sum(effects[p] * r[:, Y0:Y1, X0:X1]))
        for q in range(p, n):
            y0, y1 = max(Y0, crops[q][0]), min(Y1, crops[q][1])
            x0, x1 = max(X0, crops[q][2]), min(X1, crops[q][3])
            if y0 >= y1 or x0 >= x1:
                continue
            ep = effects[p][:, y0 - Y0:y1 - Y0, x0 - X0:x1 - X0]
            eq = effects[q][:, y0 - crops[q][0]:y1 - crops[q][0], x0 - crops[q][2]:x1 - crops[q][2]]
            M[p, q] = M[q, p] = float(np.sum(ep * eq))
    coef = np.zeros(n)
    free = list(range(n))
    first = None
    while free:
        fixed = [p for p in range(n) if p not in free]
        rhs = b[free] - M[np.ix_(free, fixed)] @ coef[fixed]
        c = np.linalg.lstsq(M[np.ix_(free, free)], rhs, rcond=None)[0]
        if first is None:
            first = c.copy()
        dist = np.minimum(np.abs(c), np.abs(c - 1.0))
        k = int(np.argmin(dist))
        coef[free[k]] = 0.0 if abs(c[k]) <= abs(c[k] - 1.0) else 1.0
        free.pop(k)
    flipped = []
    for p in range(n):
        if coef[p] == 1.0:
            Y0, Y1, X0, X1 = crops[p]
            r[:, Y0:Y1, X0:X1] -= effects[p]
            flipped.append(units[p])
    return r, flipped, (np.zeros(0) if first is None else first)

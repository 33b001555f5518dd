"""Pure-loop conv, pool and Gram for tiny pins of ``oracle.ops`` (TEST INFRASTRUCTURE ONLY).

These follow the textbook definitions element by element and are only used on
inputs of a few pixels and channels.
"""
from __future__ import annotations

import numpy as np


def conv3x3_loops(a, w, b=None):
    cin, h, wd = a.shape
    cout = w.shape[0]
    z = np.zeros((cout, h, wd))
    for o in range(cout):
        for y in range(h):
            for x in range(wd):
                s = 0.0 if b is None else float(b[o])
                for i in range(cin):
                    for ky in range(3):
                        for kx in range(3):
                            yy, xx = y + ky - 1, x + kx - 1
                            if 0 <= yy < h and 0 <= xx < wd:
                                s += float(w[o, i, ky, kx]) * float(a[i, yy, xx])
                z[o, y, x] = s
    return z


def maxpool2_loops(a):
    c, h, w = a.shape
    out = np.zeros((c, h // 2, w // 2))
    arg = np.zeros((c, h // 2, w // 2), np.int64)
    for ch in range(c):
        for y in range(h // 2):
            for x in range(w // 2):
                best, bk = None, -1
                for k, (dy, dx) in enumerate(((0, 0), (0, 1), (1, 0), (1, 1))):
                    v = a[ch, 2 * y + dy, 2 * x + dx]
                    if best is None or v > best:
                        best, bk = v, k
                out[ch, y, x] = best
                arg[ch, y, x] = bk
    return out, arg


def gram_loops(v, n_p):
    c, h, w = v.shape
    g = np.zeros((c, c))
    for i in range(c):
        for j in range(c):
            s = 0.0
            for y in range(h):
                for x in range(w):
                    s += float(v[i, y, x]) * float(v[j, y, x])
            g[i, j] = s / n_p
    return g

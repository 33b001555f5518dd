"""Plain FP64 building blocks of the VGG feature network (TEST INFRASTRUCTURE ONLY).

Arrays are C x H x W float64.  Convolution follows the deep-learning
convention (cross-correlation) with 1 px zero padding and stride 1:

    Z[o, y, x] = b[o] + sum_{i, ky, kx} W[o, i, ky, kx] * A[i, y + ky - 1, x + kx - 1]

It is written as nine shifted channel matmuls, one per filter tap.  The
adjoint scatters each tap's transposed matmul back to the shifted position.
Max pooling is 2x2, stride 2, floor mode; the backward routes the incoming
gradient to the first maximum in the order (0,0), (0,1), (1,0), (1,1) and gives
0 to rows/columns that floor mode drops.  Average pooling (the variant of the
network with every max pool replaced by a 2x2 mean) has the same geometry.
"""
from __future__ import annotations

import numpy as np


def conv3x3(a: np.ndarray, w: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    cin, h, wd = a.shape
    cout = w.shape[0]
    assert w.shape == (cout, cin, 3, 3)
    ap = np.zeros((cin, h + 2, wd + 2), np.float64)
    ap[:, 1:-1, 1:-1] = a
    z = np.zeros((cout, h * wd), np.float64)
    for ky in range(3):
        for kx in range(3):
            patch = ap[:, ky:ky + h, kx:kx + wd].reshape(cin, h * wd)
            z += w[:, :, ky, kx].astype(np.float64) @ patch
    if b is not None:
        z += np.asarray(b, np.float64)[:, None]
    return z.reshape(cout, h, wd)


def conv3x3_adjoint(dz: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of ``conv3x3`` with respect to its input (bias excluded)."""
    cout, h, wd = dz.shape
    cin = w.shape[1]
    dap = np.zeros((cin, h + 2, wd + 2), np.float64)
    d2 = dz.reshape(cout, h * wd)
    for ky in range(3):
        for kx in range(3):
            dap[:, ky:ky + h, kx:kx + wd] += (w[:, :, ky, kx].astype(np.float64).T @ d2).reshape(cin, h, wd)
    return dap[:, 1:-1, 1:-1]


def relu(z: np.ndarray) -> np.ndarray:
    return np.maximum(z, 0.0)


def _pool_views(a: np.ndarray):
    c, h, w = a.shape
    h2, w2 = h // 2, w // 2
    v = a[:, : 2 * h2, : 2 * w2].reshape(c, h2, 2, w2, 2)
    # window order (0,0), (0,1), (1,0), (1,1)
    return np.stack([v[:, :, 0, :, 0], v[:, :, 0, :, 1], v[:, :, 1, :, 0], v[:, :, 1, :, 1]], 0)


def maxpool2(a: np.ndarray) -> np.ndarray:
    return _pool_views(a).max(axis=0)


def avgpool2(a: np.ndarray) -> np.ndarray:
    """2x2 stride-2 average pooling, floor mode."""
    return _pool_views(a).mean(axis=0)


def avgpool2_backward(dy: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Adjoint of ``avgpool2``: each output's gradient / 4 to its four inputs; rows and
    columns that floor mode drops get 0."""
    c, h, w = a.shape
    h2, w2 = h // 2, w // 2
    da = np.zeros((c, h, w), np.float64)
    for dy_, dx_ in ((0, 0), (0, 1), (1, 0), (1, 1)):
        da[:, dy_: 2 * h2: 2, dx_: 2 * w2: 2] = 0.25 * dy
    return da


def pool2(a: np.ndarray, avg: bool) -> np.ndarray:
    return avgpool2(a) if avg else maxpool2(a)


def pool2_backward(dy: np.ndarray, a: np.ndarray, avg: bool) -> np.ndarray:
    return avgpool2_backward(dy, a) if avg else maxpool2_backward(dy, a)


def maxpool2_backward(dy: np.ndarray, a: np.ndarray) -> np.ndarray:
    c, h, w = a.shape
    h2, w2 = h // 2, w // 2
    win = _pool_views(a)
    arg = np.argmax(win, axis=0)            # first maximum in window order
    da = np.zeros((c, h, w), np.float64)
    for k, (dy_, dx_) in enumerate(((0, 0), (0, 1), (1, 0), (1, 1))):
        da[:, dy_: 2 * h2: 2, dx_: 2 * w2: 2] = np.where(arg == k, dy, 0.0)
    return da

"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's callers.

This module holds none of the method's arithmetic: it only draws the images and
the random network weights that both the FP64 oracle and the HIP path consume.
The paper's photographs, paintings and pretrained VGG-19 weights are not
available, so these arrays stand in for them with the sizes the paper uses
(Fig. 1 / Fig. 3 sizes) and a smooth, photo-like value distribution.

Image recipe (per call):
  1. z ~ N(0, 1), shape 3 x H x W, from numpy PCG64(seed), float64
  2. per-channel Gaussian blur, std ``sigma`` px, reflect borders, truncate 4 sigma
  3. min-max rescale of the whole tensor to [0, 1]
  4. add U(-0.05, 0.05) drawn from the same generator after z
  5. clip to [0, 1] and cast to float32

Weights: He-normal N(0, 2 / (9 C_in)) per conv, drawn layer by layer in
[C_out][C_in][3][3] C-order from PCG64(seed), cast to float32; bias zero unless
``bias_std`` is given (then N(0, bias_std^2) drawn after all weights).
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
from scipy.ndimage import gaussian_filter

SEED_WEIGHTS = 0
SEED_CONTENT = 1
SEED_STYLE = 2
SEED_X = 3
SEED_FD = 4

# VGG-19 prefix conv1_1 .. conv5_1 (13 convs) and the tiny prefix conv1_1 .. conv3_1.
VGG19_CONVS = [(3, 64), (64, 64), (64, 128), (128, 128), (128, 256), (256, 256),
               (256, 256), (256, 256), (256, 512), (512, 512), (512, 512),
               (512, 512), (512, 512)]
VGG19_TINY_CONVS = VGG19_CONVS[:5]


def _blur_one(args):
    a, sigma = args
    return gaussian_filter(a, sigma, mode="reflect", truncate=4.0)


def image(h: int, w: int, sigma: float, seed: int, threads: int = 3) -> np.ndarray:
    """One 3 x h x w float32 image in [0, 1] following the recipe above."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((3, h, w))
    if sigma > 0:
        with ThreadPoolExecutor(max(1, threads)) as ex:
            z = np.stack(list(ex.map(_blur_one, [(z[c], sigma) for c in range(3)])))
    lo, hi = float(z.min()), float(z.max())
    z = (z - lo) / (hi - lo if hi > lo else 1.0)
    z += rng.uniform(-0.05, 0.05, size=z.shape)
    np.clip(z, 0.0, 1.0, out=z)
    return z.astype(np.float32)


def box_down2(img: np.ndarray) -> np.ndarray:
    """2x2 box average (floor size) of a C x H x W array, for image pyramids."""
    c, h, w = img.shape
    h2, w2 = h // 2, w // 2
    a = img[:, : 2 * h2, : 2 * w2].astype(np.float64)
    a = a.reshape(c, h2, 2, w2, 2).mean(axis=(2, 4))
    return a.astype(img.dtype)


def vgg_weights(convs, seed: int = SEED_WEIGHTS, bias_std: float = 0.0):
    """He-normal weights [C_out][C_in][3][3] float32 and biases [C_out] float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ws = []
    for cin, cout in convs:
        std = np.sqrt(2.0 / (9.0 * cin))
        ws.append((rng.standard_normal((cout, cin, 3, 3)) * std).astype(np.float32))
    bs = []
    for cin, cout in convs:
        if bias_std > 0:
            bs.append((rng.standard_normal(cout) * bias_std).astype(np.float32))
        else:
            bs.append(np.zeros(cout, np.float32))
    return ws, bs

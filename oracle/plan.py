"""Tile plan: blocks, margins and owned feature ranges (TEST INFRASTRUCTURE ONLY).

Sec. 4.1 partitions the image into blocks and extracts each with a margin
except on sides that are image borders; Algorithm 1 keeps, per block, the
features of the block with the margin removed (Step 1) and the inner part of
the gradient (Step 2).  Readings taken where the paper is silent:

* blocks: row-major grid, block (i, j) covers rows [i T, min((i+1) T, H)) and
  the same for columns (the last row/column of blocks may be ragged);
* window: the block widened by the margin m, start rounded down and end rounded
  up to a multiple of S (the product of all pooling factors, so the pooling grid
  of every layer inside the window coincides with the whole image's), then
  clipped to the image;
* owned features of a layer of cumulative stride s: feature row q belongs to the
  block whose rows contain s q, i.e. q in [ceil(b0 / s), min(ceil(b1 / s), n)),
  with n = floor(H / s) the whole-image (floor-pooled) size.
All coordinates are whole-image ones (image px for blocks/windows, feature
rows/cols of each conv's output for owned ranges).
"""
from __future__ import annotations

from dataclasses import dataclass


def _ceil_div(a: int, b: int) -> int:
    return -((-a) // b)


@dataclass(frozen=True)
class Tile:
    by0: int
    by1: int
    bx0: int
    bx1: int
    ey0: int
    ey1: int
    ex0: int
    ex1: int
    own: tuple   # per conv: (r0, r1, c0, c1) in whole-image feature coordinates


def _axis(n: int, t: int, m: int, S: int):
    out = []
    for i in range(_ceil_div(n, t)):
        b0, b1 = i * t, min((i + 1) * t, n)
        e0 = max(0, S * ((b0 - m) // S))
        e1 = min(n, S * _ceil_div(b1 + m, S))
        out.append((b0, b1, e0, e1))
    return out


def _own(b0: int, b1: int, s: int, n_img: int):
    n = n_img // s
    return min(_ceil_div(b0, s), n), min(_ceil_div(b1, s), n)


def make_plan(h: int, w: int, t: int, m: int, strides, align: int):
    """List of Tile, row-major over the block grid."""
    assert h >= 1 and w >= 1 and t >= 1 and m >= 0
    rows, cols = _axis(h, t, m, align), _axis(w, t, m, align)
    tiles = []
    for (by0, by1, ey0, ey1) in rows:
        for (bx0, bx1, ex0, ex1) in cols:
            own = []
            for s in strides:
                r0, r1 = _own(by0, by1, s, h)
                c0, c1 = _own(bx0, bx1, s, w)
                own.append((r0, r1, c0, c1))
            tiles.append(Tile(by0, by1, bx0, bx1, ey0, ey1, ex0, ex1, tuple(own)))
    return tiles

"""Plain definitions used to pin the oracle's tile logic.

TEST INFRASTRUCTURE ONLY (see the package docstring).

TILE* is the exact tile predicate behind AccuTile (Sec. 4.1.2): a record
ellipse E = {p : q(p) <= t}, q(p) = a dx^2 + 2 b dx dy + c dy^2 with
(dx, dy) = p - (u, v), touches tile (tx, ty) iff the minimum of q over the
closed square [16 tx, 16 tx + 16] x [16 ty, 16 ty + 16] is <= t.  For a
positive-definite q that minimum is 0 when the centre lies in the square and
otherwise the smallest of the four per-edge minima of a 1-D quadratic,
each clamped to its edge.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

TILE = 16


def _edge_min(a, b, c, u, v, fixed, lo, hi, horizontal):
    """Minimum of q along one edge: y = fixed (horizontal) or x = fixed."""
    if horizontal:
        dy = fixed - v
        x = np.clip(u - b * dy / a, lo, hi)
        dx = x - u
    else:
        dx = fixed - u
        y = np.clip(v - b * dx / c, lo, hi)
        dy = y - v
    return a * dx * dx + 2.0 * b * dx * dy + c * dy * dy


def tile_min_q(geom, conic, tiles_x, tiles_y):
    """FP64 minimum of q over every closed tile square, shape [tiles_y, tiles_x]."""
    u, v, t = (float(geom[0]), float(geom[1]), float(geom[3]))
    a, b, c = (float(conic[0]), float(conic[1]), float(conic[2]))
    ty, tx = np.mgrid[0:tiles_y, 0:tiles_x].astype(np.float64)
    x0, x1, y0, y1 = TILE * tx, TILE * tx + TILE, TILE * ty, TILE * ty + TILE
    m = np.minimum.reduce([
        _edge_min(a, b, c, u, v, y0, x0, x1, True),
        _edge_min(a, b, c, u, v, y1, x0, x1, True),
        _edge_min(a, b, c, u, v, x0, y0, y1, False),
        _edge_min(a, b, c, u, v, x1, y0, y1, False),
    ])
    inside = (x0 <= u) & (u <= x1) & (y0 <= v) & (v <= y1)
    return np.where(inside, 0.0, m), t


def tile_star(geom, conic, tiles_x, tiles_y, band=1e-9):
    """Exact tile set in FP64.  Returns (sure, maybe): ``sure`` are tile ids with
    min q <= t - band*scale, ``maybe`` those within the rounding band
    |min q - t| <= band*scale, where either answer is acceptable."""
    a, b, c = (float(conic[0]), float(conic[1]), float(conic[2]))
    if not (a * c - b * b > 0.0):
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    mq, t = tile_min_q(geom, conic, tiles_x, tiles_y)
    scale = band * max(abs(t), 1.0)
    ids = np.arange(tiles_x * tiles_y).reshape(tiles_y, tiles_x)
    sure = ids[mq <= t - scale]
    maybe = ids[np.abs(mq - t) <= scale]
    return sure, maybe


def tile_star_exact(geom, conic, tiles_x, tiles_y):
    """Exact rational tile set (Fractions of the FP32 record values)."""
    u, v, _, t = (Fraction(float(x)) for x in geom)
    a, b, c = (Fraction(float(x)) for x in conic[:3])
    if not (a * c - b * b > 0):
        return set()

    def q(dx, dy):
        return a * dx * dx + 2 * b * dx * dy + c * dy * dy

    def clamp(x, lo, hi):
        return lo if x < lo else hi if x > hi else x

    out = set()
    for ty in range(tiles_y):
        for tx in range(tiles_x):
            x0, x1, y0, y1 = TILE * tx, TILE * tx + TILE, TILE * ty, TILE * ty + TILE
            if x0 <= u <= x1 and y0 <= v <= y1:
                out.add(ty * tiles_x + tx)
                continue
            best = None
            for Y in (y0, y1):
                dy = Y - v
                dx = clamp(u - b * dy / a, x0, x1) - u
                val = q(dx, dy)
                best = val if best is None or val < best else best
            for X in (x0, x1):
                dx = X - u
                dy = clamp(v - b * dx / c, y0, y1) - v
                val = q(dx, dy)
                best = val if val < best else best
            if best <= t:
                out.add(ty * tiles_x + tx)
    return out


def ellipse_boundary(geom, conic, n=20000):
    """Dense sampling of the record ellipse boundary p = mu + sqrt(t) L (cos, sin),
    L L^T = conic^{-1} (Cholesky), in FP64."""
    u, v, t = float(geom[0]), float(geom[1]), float(geom[3])
    a, b, c = (float(conic[0]), float(conic[1]), float(conic[2]))
    S = np.linalg.inv(np.array([[a, b], [b, c]], dtype=np.float64))
    L = np.linalg.cholesky(S)
    th = np.linspace(0.0, 2.0 * np.pi, n, endpoint=False)
    pts = np.sqrt(t) * (L @ np.stack([np.cos(th), np.sin(th)]))
    return u + pts[0], v + pts[1]


def disk_tiles(cx, cy, radius, tiles_x, tiles_y):
    """Textbook circle-rectangle test: clamp the centre into each tile square and
    compare the distance with the radius."""
    out = set()
    for ty in range(tiles_y):
        for tx in range(tiles_x):
            x = min(max(cx, TILE * tx), TILE * tx + TILE)
            y = min(max(cy, TILE * ty), TILE * ty + TILE)
            if (x - cx) ** 2 + (y - cy) ** 2 <= radius * radius:
                out.add(ty * tiles_x + tx)
    return out

"""Worked examples from the paper, stored under tests/golden with their
citations, against the oracle (CPU)."""
import math
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F32 = np.float32


def _numbers(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


def test_accutile_walkthrough():
    """Speedy-Splat Sec. 4.1.2, the AccuTile walkthrough of the tile figure:
    row extents x_min .. B, A .. x_max and C .. D, from closed-form points of
    the stored conic, equal the oracle's AccuTile tiles row by row."""
    rows = _numbers("accutile_walkthrough.txt")
    u, v, t, a, b, c = (float(x) for x in rows[0])
    roles = {r[1]: int(r[0]) for r in rows[1:]}
    det = a * c - b * b
    hx, hy = math.sqrt(t * c / det), math.sqrt(t * a / det)
    # the box's left and right edges touch the ellipse at dy = -(b / c) dx
    x_min = (u - hx, v + (b / c) * hx)
    x_max = (u + hx, v - (b / c) * hx)

    def cut(y):  # the ellipse's x at height y, smaller root first
        dy = y - v
        qa, qb, qc = a, 2.0 * b * dy, c * dy * dy - t
        r = math.sqrt(qb * qb - 4.0 * qa * qc)
        return u + (-qb - r) / (2.0 * qa), u + (-qb + r) / (2.0 * qa)

    bottom, middle, top = roles["bottom"], roles["middle"], roles["top"]
    assert (bottom, middle, top) == (middle + 1, top + 1, top)
    A, B = cut(16.0 * bottom)          # the bottom row's upper boundary
    C, D = cut(16.0 * middle)          # the middle row's upper boundary
    # the structure the walkthrough describes holds for this record
    assert 16 * top <= v - hy < 16 * middle and 16 * bottom <= v + hy < 16 * (bottom + 1)
    assert 16 * bottom <= x_min[1] < 16 * (bottom + 1)
    assert 16 * middle <= x_max[1] < 16 * bottom
    extent = {bottom: (x_min[0], B), middle: (A, x_max[0]), top: (C, D)}
    for lo, hi in extent.values():
        for x in (lo, hi):
            assert abs(x / 16.0 - round(x / 16.0)) * 16.0 > 0.25   # clear of tile edges
    want = {(tx, ty) for ty, (lo, hi) in extent.items()
            for tx in range(math.floor(lo / 16.0), math.floor(hi / 16.0) + 1)}
    tx_n, ty_n = 10, 6
    geom = np.array([u, v, 1.0, t], F32)
    conic = np.array([a, b, c, 0.5], F32)
    got = {(int(i) % tx_n, int(i) // tx_n)
           for i in oracle.tile_list(geom, conic, "accutile", tx_n, ty_n)}
    assert got == want
    # SnugBox keeps the whole box: every row spans the box's tile columns
    snug = {(int(i) % tx_n, int(i) // tx_n)
            for i in oracle.tile_list(geom, conic, "snugbox", tx_n, ty_n)}
    box_cols = range(math.floor((u - hx) / 16.0), math.floor((u + hx) / 16.0) + 1)
    assert snug == {(tx, ty) for ty in (top, middle, bottom) for tx in box_cols}
    assert got < snug

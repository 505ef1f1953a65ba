"""Structured right-triangle mesh of the unit square.

Oracle module (test infrastructure only).

The paper's tests use uniform triangulations of the unit square (Section 4.1).
Here every one of the ncell x ncell cells is split by its "/" diagonal:
  lower triangle: (i, j), (i+1, j), (i+1, j+1)
  upper triangle: (i, j), (i+1, j+1), (i, j+1)
both counter-clockwise.  Scalar (P1) nodes live on the (ncell+1)^2 lattice,
id = j*(ncell+1) + i; P2 displacement nodes on the (2 ncell+1)^2 lattice of
spacing h/2, id = J*(2 ncell+1) + I.
"""
from __future__ import annotations

import numpy as np

from workloads import XSPLIT, YSPLIT, CORE


class Mesh:
    def __init__(self, ncell: int, order_u: int, layout: str):
        self.n = n = ncell
        self.h = 1.0 / n
        self.order_u = order_u
        self.layout = layout
        ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing='xy')
        ci = ci.ravel()
        cj = cj.ravel()
        # two triangles per cell, stored cell-major: tri 2c (lower), 2c+1 (upper)
        vi = np.empty((2 * n * n, 3), dtype=np.int64)
        vj = np.empty((2 * n * n, 3), dtype=np.int64)
        vi[0::2] = np.stack([ci, ci + 1, ci + 1], 1)
        vj[0::2] = np.stack([cj, cj, cj + 1], 1)
        vi[1::2] = np.stack([ci, ci + 1, ci], 1)
        vj[1::2] = np.stack([cj, cj + 1, cj + 1], 1)
        self.tri_cell_i = np.repeat(ci, 2)
        self.tri_cell_j = np.repeat(cj, 2)
        self.tri_vi = vi
        self.tri_vj = vj
        self.X = np.stack([vi * self.h, vj * self.h], axis=2)   # (E, 3, 2)
        self.p1 = vj * (n + 1) + vi                            # P1 ids (E, 3)
        self.n1 = (n + 1) ** 2
        if order_u == 1:
            self.pu = self.p1.copy()
            self.nu_lat = self.n1
            self.mu = n + 1
        else:
            m = 2 * n + 1
            VI, VJ = 2 * vi, 2 * vj
            mids = []
            for a, b in ((0, 1), (1, 2), (2, 0)):
                mids.append(((VJ[:, a] + VJ[:, b]) // 2) * m + (VI[:, a] + VI[:, b]) // 2)
            self.pu = np.concatenate([VJ * m + VI, np.stack(mids, 1)], axis=1)
            self.nu_lat = m * m
            self.mu = m
        # cell centre decides the region
        xc = (self.tri_cell_i + 0.5) * self.h
        yc = (self.tri_cell_j + 0.5) * self.h
        if layout == XSPLIT:
            poro = xc < 0.5
        elif layout == YSPLIT:
            poro = yc < 0.5
        elif layout == CORE:
            poro = (xc > 0.25) & (xc < 0.75) & (yc > 0.25) & (yc < 0.75)
        else:
            raise ValueError(layout)
        self.tri_poro = poro

    # lattice coordinates ---------------------------------------------------
    def p1_xy(self, ids):
        ids = np.asarray(ids)
        return np.stack([(ids % (self.n + 1)) * self.h, (ids // (self.n + 1)) * self.h], -1)

    def pu_xy(self, ids):
        ids = np.asarray(ids)
        s = self.h if self.order_u == 1 else 0.5 * self.h
        return np.stack([(ids % self.mu) * s, (ids // self.mu) * s], -1)

    def on_side_p1(self, ids, mask):
        return _on_sides(self.p1_xy(ids), mask)

    def on_side_pu(self, ids, mask):
        return _on_sides(self.pu_xy(ids), mask)


def _on_sides(xy, mask):
    x, y = xy[..., 0], xy[..., 1]
    tol = 1e-12
    out = np.zeros(x.shape, dtype=bool)
    if mask & 1:
        out |= np.abs(x) < tol
    if mask & 2:
        out |= np.abs(x - 1) < tol
    if mask & 4:
        out |= np.abs(y) < tol
    if mask & 8:
        out |= np.abs(y - 1) < tol
    return out

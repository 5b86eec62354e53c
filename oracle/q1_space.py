"""Oracle construction of the three-dimensional trilinear spaces (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library or its
binding.  For the trilinear (Q1) discretisation of the cube (0,pi)^3 with N^3
cells (Section 6, Example 6.3), this module builds on its own what the
two-level method needs besides K and M (Section 2.3):

* ``coarse_space`` -- V^H in V^h: every trilinear hat function of the coarse
  grid (Nc^3 cubes) at the fine nodes, from the nodes' coordinates: inside a
  coarse cube the hat of a corner is the product of the three 1-D linear
  weights of that corner;
* ``local_spaces`` -- V^(l): the interior nodes of the coarse cube enlarged
  by delta = L h, i.e. the fine nodes whose coordinates lie within
  (L - 1) h of the closed cube in every direction.

Fine dofs are the interior nodes (i, j, k), numbered with i fastest; coarse dofs
the interior coarse nodes, numbered the same way.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["coarse_space", "local_spaces"]


def coarse_space(N: int, Nc: int) -> sp.csr_matrix:
    h, H = np.pi / N, np.pi / Nc
    rows, cols, vals = [], [], []
    d = 0
    for k in range(1, N):
        for j in range(1, N):
            for i in range(1, N):
                x = np.array([i * h, j * h, k * h])
                cell = np.minimum((x / H + 1e-12).astype(int), Nc - 1)    # coarse cube holding the node
                t = x / H - cell                                           # local coordinates in [0, 1]
                for corner in range(8):
                    off = np.array([(corner >> 0) & 1, (corner >> 1) & 1, (corner >> 2) & 1])
                    v = cell + off                                         # coarse node (a, b, c)
                    if np.any(v < 1) or np.any(v > Nc - 1):
                        continue                                           # Dirichlet coarse node
                    wgt = float(np.prod(np.where(off == 1, t, 1.0 - t)))
                    if wgt != 0.0:
                        rows.append(d)
                        cols.append((v[2] - 1) * (Nc - 1) ** 2 + (v[1] - 1) * (Nc - 1) + (v[0] - 1))
                        vals.append(wgt)
                d += 1
    P = sp.csr_matrix((vals, (rows, cols)), shape=((N - 1) ** 3, (Nc - 1) ** 3))
    P.sum_duplicates()
    return P


def local_spaces(N: int, Nc: int, L: int) -> list:
    h, H = np.pi / N, np.pi / Nc
    g = np.arange(1, N) * h
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    X = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)
    tol = 1e-9 * h
    subs = []
    for c3 in range(Nc):
        for c2 in range(Nc):
            for c1 in range(Nc):
                lo = np.array([c1, c2, c3]) * H - (L - 1) * h - tol
                hi = (np.array([c1, c2, c3]) + 1) * H + (L - 1) * h + tol
                subs.append(np.flatnonzero(np.all((X >= lo) & (X <= hi), axis=1)))
    return subs

"""Oracle construction of the fourth-order (m = 2) spaces (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library or its
binding.  For the Bogner-Fox-Schmit (bicubic Hermite) discretisation of the
clamped unit square (Section 2.2, biharmonic problem, V^h in H^2_0), this
module builds on its own what the two-level method needs besides K and M
(Section 2.3):

* ``coarse_space`` -- V^H in V^h: every coarse BFS basis function written in
  the fine dofs (value, x- and y-derivative and mixed derivative at every fine
  vertex).  Each 1-D coarse basis function is recovered piece by piece as the
  cubic that meets its four Hermite conditions at the ends of a coarse cell
  (a 4 x 4 linear solve), then evaluated at the fine nodes; the 2-D functions
  are products of two such factors.
* ``local_spaces`` -- V^(l) = V^h intersected with H^2_0 of the enlarged cell:
  every dof of the fine vertices that lie strictly inside the coarse cell grown
  by delta = L h, found from the vertex coordinates.

Fine dofs are identified by the (vertex, kind) arrays that come with the
matrices (kind 0 u, 1 u_x, 2 u_y, 3 u_xy).  Coarse dofs are numbered vertex by
vertex, row by row, with the same kind order.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["coarse_space", "local_spaces", "coarse_cubic_pieces"]


def coarse_cubic_pieces(Nc: int):
    """Polynomial coefficients (highest power first, in x) of the 1-D coarse Hermite
    basis functions: pieces[(node, kind)] = {cell: coeffs}, kind 0 value, 1 slope."""
    H = 1.0 / Nc

    def cond(x):
        return np.array([[x**3, x**2, x, 1.0], [3 * x**2, 2 * x, 1.0, 0.0]])
    pieces = {}
    for c in range(Nc + 1):
        for kind in (0, 1):
            cells = {}
            for e in (c - 1, c):
                if e < 0 or e >= Nc:
                    continue
                xa, xb = e * H, (e + 1) * H
                A = np.vstack([cond(xa), cond(xb)])
                rhs = np.zeros(4)
                # the function's value/slope is 1 at its own node and 0 elsewhere
                row = (0 if c == e else 2) + kind
                rhs[row] = 1.0
                cells[e] = np.linalg.solve(A, rhs)
            pieces[(c, kind)] = cells
    return pieces


def _eval_1d(pieces, Nc: int, c: int, kind: int, x: float, deriv: int) -> float:
    """Value (deriv 0) or slope (deriv 1) of coarse function (c, kind) at x."""
    H = 1.0 / Nc
    e = min(int(np.floor(x / H + 1e-12)), Nc - 1)
    coeffs = pieces[(c, kind)].get(e)
    if coeffs is None:
        return 0.0
    p = np.poly1d(coeffs)
    return float((p.deriv() if deriv else p)(x))


def coarse_space(N: int, Nc: int, vert: np.ndarray, kind: np.ndarray) -> sp.csr_matrix:
    """n x n_H matrix whose column j holds the fine dofs of coarse BFS function j
    (clamped: coarse vertices 1..Nc-1 in both directions, four kinds each)."""
    h = 1.0 / N
    pieces = coarse_cubic_pieces(Nc)
    cverts = [(cx, cy) for cy in range(1, Nc) for cx in range(1, Nc)]
    col_of = {}
    for v, (cx, cy) in enumerate(cverts):
        for kk in range(4):
            col_of[(cx, cy, kk)] = 4 * v + kk
    rows, cols, vals = [], [], []
    for d in range(len(kind)):
        x, y = vert[d, 0] * h, vert[d, 1] * h
        dx, dy = kind[d] & 1, kind[d] >> 1          # derivative orders of this fine dof
        ex = min(int(np.floor(x * Nc + 1e-12)), Nc - 1)
        ey = min(int(np.floor(y * Nc + 1e-12)), Nc - 1)
        for cx in (ex, ex + 1):
            for cy in (ey, ey + 1):
                if not (1 <= cx <= Nc - 1 and 1 <= cy <= Nc - 1):
                    continue
                for kk in range(4):
                    kx, ky = kk & 1, kk >> 1
                    v = (_eval_1d(pieces, Nc, cx, kx, x, dx) * _eval_1d(pieces, Nc, cy, ky, y, dy))
                    if abs(v) > 1e-14:
                        rows.append(d)
                        cols.append(col_of[(cx, cy, kk)])
                        vals.append(v)
    P = sp.coo_matrix((vals, (rows, cols)), shape=(len(kind), 4 * len(cverts))).tocsr()
    P.sort_indices()
    return P


def local_spaces(N: int, Nc: int, L: int, vert: np.ndarray) -> list:
    """Dof sets of V^(l): coarse cell (a, b), row by row, grown by delta = L h; a dof
    belongs when its vertex lies strictly inside the grown cell."""
    h, H = 1.0 / N, 1.0 / Nc
    delta = L * h
    x, y = vert[:, 0] * h, vert[:, 1] * h
    eps = 1e-9 * h
    subs = []
    for b in range(Nc):
        for a in range(Nc):
            x0, x1 = a * H - delta, (a + 1) * H + delta
            y0, y1 = b * H - delta, (b + 1) * H + delta
            inside = (x > x0 + eps) & (x < x1 - eps) & (y > y0 + eps) & (y < y1 - eps)
            subs.append(np.flatnonzero(inside))
    return subs

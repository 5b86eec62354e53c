"""Seeded synthetic problem data for the two-level BPJD eigensolver.

This module only *generates inputs*: uniform right-triangle meshes with every
cell cut by its "/" diagonal, the nested coarse mesh (its grid lines), the P1
stiffness and consistent mass matrices of the fine mesh (Section 2.2 of the
paper: a(u,v) = int a grad u . grad v, b(u,v) = int u v, homogeneous Dirichlet
data), optional piecewise-constant coefficients, and seeded random blocks.
It holds no step of the eigensolver itself (no restriction, coarse space,
preconditioner, orthogonalisation or Rayleigh-Ritz): the library and the test
oracle each implement those on their own and both read what is made here.

Matrices are returned as scipy CSR on the *union* pattern of K and M: the
hypotenuse couplings of the right triangles are exact zeros in K but not in M,
so K stores them as explicit zeros.

For the fourth-order case (Section 2.2, the biharmonic problem with clamped
edges, a(u,v) = int Lap u Lap v) the module also makes the Bogner-Fox-Schmit
(bicubic Hermite) discretisation of the unit square, which the paper names for
m = 2.  Its element is not tied to a triangle mesh, so the generic interface
of the library takes it: the caller hands over the coarse space as a
prolongation matrix P (the nested coarse BFS space written in fine dofs) and
the local spaces as dof sets (all dofs of the fine vertices strictly inside
each enlarged coarse cell, i.e. V^h intersected with H^2_0 of that cell).
These are the caller's description of V^H and V^(l); the eigensolver's own
steps (Galerkin products, coarse eigenbasis, local factorisations) are not
here.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Mesh", "p1_mesh", "p1_lshape", "coarse_lines", "config_mesh", "CONFIGS",
    "block_coefficient", "seeded_block", "serving_requests",
    "Plate", "hermite_1d", "bfs_plate", "PLATE_CONFIGS", "config_plate",
]


@dataclass
class Mesh:
    """A uniform fine mesh of [0,Lx]x[0,Ly] with its nested coarse grid lines."""
    Lx: float
    Ly: float
    Nx: int
    Ny: int
    K: sp.csr_matrix            # stiffness, union pattern, float64
    M: sp.csr_matrix            # consistent mass, union pattern, float64
    coords: np.ndarray          # (n, 2) coordinates of the interior (free) nodes
    cx: np.ndarray              # coarse grid lines in x (ascending, incl. 0 and Lx)
    cy: np.ndarray              # coarse grid lines in y
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.K.shape[0]

    @property
    def hx(self) -> float:
        return self.Lx / self.Nx

    @property
    def hy(self) -> float:
        return self.Ly / self.Ny


def coarse_lines(L: float, N: int, cells_per_coarse: int) -> np.ndarray:
    """Coarse grid lines of a fine grid of N cells on [0, L].

    A coarse cell spans ``cells_per_coarse`` fine cells; a remainder of less
    than half a coarse cell is merged into the last coarse cell, a larger one
    forms its own (smaller) cell.  Lines lie exactly on fine grid lines.
    """
    if cells_per_coarse <= 0 or N <= 0:
        raise ValueError("cells_per_coarse and N must be positive")
    nfull, rem = divmod(N, cells_per_coarse)
    idx = [i * cells_per_coarse for i in range(nfull + 1)]
    if rem:
        if rem * 2 < cells_per_coarse and nfull >= 1:
            idx[-1] = N
        else:
            idx.append(N)
    idx = np.asarray(idx, dtype=np.int64)
    return idx * (L / N)


def _p1_assemble(x0: float, y0: float, hx: float, hy: float, Nx: int, Ny: int,
                 node_is_dof: np.ndarray, cell_kept: np.ndarray,
                 coef: Optional[Callable[[np.ndarray, np.ndarray], np.ndarray]] = None):
    """P1 stiffness/mass of the kept cells of a uniform "/" grid.

    Grid node (i, j), 0 <= i <= Nx, 0 <= j <= Ny, sits at (x0 + i hx, y0 + j hy);
    ``node_is_dof[j, i]`` marks the free nodes (dofs numbered row by row, x
    fastest), ``cell_kept[j, i]`` the cells of the domain.  Cell (i, j) is split
    into T1 = {(i,j),(i+1,j),(i+1,j+1)} and T2 = {(i,j),(i+1,j+1),(i,j+1)}.
    Returns (K, M, coords) with K, M on one (union) pattern.
    """
    dofnum = -np.ones((Ny + 1, Nx + 1), dtype=np.int64)
    jj, ii = np.nonzero(node_is_dof)
    dofnum[jj, ii] = np.arange(jj.size)
    n = int(jj.size)
    cj, ci = np.nonzero(cell_kept)
    tri_i = np.concatenate([np.stack([ci, ci + 1, ci + 1], 1), np.stack([ci, ci + 1, ci], 1)])
    tri_j = np.concatenate([np.stack([cj, cj, cj + 1], 1), np.stack([cj, cj + 1, cj + 1], 1)])
    x = x0 + tri_i * hx
    y = y0 + tri_j * hy
    # gradients of the barycentric functions: grad phi_a = (y_b - y_c, x_c - x_b) / (2 area)
    xa, xb, xc = x[:, 0], x[:, 1], x[:, 2]
    ya, yb, yc = y[:, 0], y[:, 1], y[:, 2]
    area2 = (xb - xa) * (yc - ya) - (xc - xa) * (yb - ya)
    gx = np.stack([yb - yc, yc - ya, ya - yb], 1) / area2[:, None]
    gy = np.stack([xc - xb, xa - xc, xb - xa], 1) / area2[:, None]
    area = 0.5 * area2
    if coef is None:
        a = np.ones_like(area)
    else:
        a = np.asarray(coef(x.mean(1), y.mean(1)), dtype=np.float64)
    Ke = a[:, None, None] * area[:, None, None] * (gx[:, :, None] * gx[:, None, :] + gy[:, :, None] * gy[:, None, :])
    Me = (area / 12.0)[:, None, None] * (np.ones((3, 3)) + np.eye(3))[None]
    d = dofnum[tri_j, tri_i]
    rows = np.repeat(d, 3, axis=1).ravel()
    cols = np.tile(d, (1, 3)).ravel()
    keep = (rows >= 0) & (cols >= 0)
    r, c = rows[keep], cols[keep]
    # K and M come from the same (row, col) list, so coo->csr gives both the
    # same (union) pattern; K's hypotenuse couplings stay as explicit zeros.
    K = sp.coo_matrix((Ke.reshape(-1)[keep], (r, c)), shape=(n, n)).tocsr()
    M = sp.coo_matrix((Me.reshape(-1)[keep], (r, c)), shape=(n, n)).tocsr()
    K.sort_indices()
    M.sort_indices()
    assert np.array_equal(K.indptr, M.indptr) and np.array_equal(K.indices, M.indices)
    coords = np.stack([x0 + ii * hx, y0 + jj * hy], 1).astype(np.float64)
    return K, M, coords


def p1_mesh(Lx: float, Ly: float, Nx: int, Ny: int, cells_per_coarse_x: int,
            cells_per_coarse_y: Optional[int] = None,
            coef: Optional[Callable[[np.ndarray, np.ndarray], np.ndarray]] = None) -> Mesh:
    """P1 stiffness/mass on the uniform "/" mesh of [0,Lx]x[0,Ly].

    Cell (i,j) = [i hx,(i+1)hx] x [j hy,(j+1)hy] is split into
    T1 = {(i,j),(i+1,j),(i+1,j+1)} and T2 = {(i,j),(i+1,j+1),(i,j+1)}.
    Interior node (i,j), 1<=i<Nx, 1<=j<Ny, has dof number (j-1)(Nx-1)+(i-1).
    ``coef(xc, yc)`` gives the element coefficient at element centroids
    (default 1).
    """
    if cells_per_coarse_y is None:
        cells_per_coarse_y = cells_per_coarse_x
    hx, hy = Lx / Nx, Ly / Ny
    node = np.zeros((Ny + 1, Nx + 1), dtype=bool)
    node[1:Ny, 1:Nx] = True
    cells = np.ones((Ny, Nx), dtype=bool)
    K, M, coords = _p1_assemble(0.0, 0.0, hx, hy, Nx, Ny, node, cells, coef)
    return Mesh(Lx, Ly, Nx, Ny, K, M, coords,
                coarse_lines(Lx, Nx, cells_per_coarse_x),
                coarse_lines(Ly, Ny, cells_per_coarse_y))


def p1_lshape(N: int, cells_per_coarse: int) -> Mesh:
    """P1 on the L-shaped domain (-pi,pi)^2 minus [0,pi) x (-pi,0] (Section 6,
    Example 6.2), from the uniform "/" mesh of the square with N x N cells (N
    even): the cells of the removed quadrant are dropped and every node on the
    boundary of the L (outer edges and the two re-entrant edges) is fixed.  The
    coarse grid lines split the square into coarse cells of ``cells_per_coarse``
    fine cells; coarse cells of the removed quadrant hold no dof."""
    if N % 2:
        raise ValueError("N must be even")
    h = 2.0 * np.pi / N
    half = N // 2
    node = np.zeros((N + 1, N + 1), dtype=bool)
    node[1:N, 1:N] = True
    node[0:half + 1, half:] = False          # x >= 0 and y <= 0: the removed quadrant, closed
    cells = np.ones((N, N), dtype=bool)
    cells[:half, half:] = False              # cells with x > 0, y < 0
    K, M, coords = _p1_assemble(-np.pi, -np.pi, h, h, N, N, node, cells)
    lines = coarse_lines(2.0 * np.pi, N, cells_per_coarse) - np.pi
    return Mesh(2.0 * np.pi, 2.0 * np.pi, N, N, K, M, coords, lines, lines.copy(),
                meta={"domain": "lshape"})


def block_coefficient(Lx: float, Ly: float, values: np.ndarray):
    """Piecewise-constant coefficient on a (by x bx) block grid over [0,Lx]x[0,Ly]."""
    values = np.asarray(values, dtype=np.float64)
    by, bx = values.shape

    def coef(xc, yc):
        ix = np.minimum((xc / Lx * bx).astype(np.int64), bx - 1)
        iy = np.minimum((yc / Ly * by).astype(np.int64), by - 1)
        return values[iy, ix]
    return coef


def seeded_block(n: int, s: int, seed) -> np.ndarray:
    """(n, s) standard-normal block from numpy's default generator."""
    return np.random.default_rng(seed).standard_normal((n, s))


# ----------------------------------------------------------------------------
# Named workloads.  H is the coarse cell side, L the overlap in element layers
# (delta = L h), k the wanted eigenpairs, guard the extra block columns.
CONFIGS = {
    "c1": dict(Lx=1.0, Ly=1.0, Nx=32, Ny=32, coarse=8, L=2, k=4, guard=0, seed_block=0,
               desc="Laplacian P1 unit square h=1/32, 4x4 subdomains, delta=2h, k=4, seeded initial block"),
    "c2": dict(Lx=1.0, Ly=1.0, Nx=512, Ny=512, coarse=32, L=4, k=8, guard=0, seed_block=None,
               desc="Laplacian P1 unit square h=1/512, 16x16 subdomains, delta=4h, k=8"),
    "c3": dict(Lx=1.0, Ly=1.01, Nx=1024, Ny=1034, coarse=32, L=4, k=12, guard=1, seed_block=None,
               desc="Laplacian P1 [0,1]x[0,1.01] h=1/1024, 32x32 subdomains, delta=4h, k=12"),
    # small cases of the same families (test sizes)
    "t8": dict(Lx=1.0, Ly=1.0, Nx=8, Ny=8, coarse=2, L=1, k=2, guard=0, seed_block=None,
               desc="tiny 8x8 mesh, 4x4 subdomains"),
    "t16": dict(Lx=1.0, Ly=1.0, Nx=16, Ny=16, coarse=4, L=1, k=3, guard=0, seed_block=None,
                desc="16x16 mesh, 4x4 subdomains"),
    "t64": dict(Lx=1.0, Ly=1.0, Nx=64, Ny=64, coarse=16, L=2, k=6, guard=0, seed_block=None,
                desc="64x64 mesh, 4x4 subdomains"),
    "t128": dict(Lx=1.0, Ly=1.0, Nx=128, Ny=128, coarse=16, L=2, k=8, guard=0, seed_block=None,
                 desc="h=1/128 (the 16129-dof mesh of the first Table 1 column), 8x8 subdomains"),
    "w56": dict(Lx=1.0, Ly=1.0, Nx=144, Ny=144, coarse=48, L=4, k=2, guard=0, seed_block=None,
                desc="3x3 wide subdomains: local half-bandwidths 52-56"),
    "w78": dict(Lx=1.0, Ly=1.0, Nx=216, Ny=216, coarse=72, L=3, k=2, guard=0, seed_block=None,
                desc="3x3 wide subdomains: local half-bandwidths 75-78"),
    "w84": dict(Lx=1.0, Ly=1.0, Nx=240, Ny=240, coarse=80, L=2, k=2, guard=0, seed_block=None,
                desc="3x3 wide subdomains: local half-bandwidths 82-84"),
    "h64": dict(Lx=1.0, Ly=1.0, Nx=192, Ny=192, coarse=64, L=1, k=3, guard=0, seed_block=None,
                desc="3x3 coarse cells of 64x64 fine cells: coarse supports above 4096 dofs"),
    "r96": dict(Lx=1.0, Ly=1.01, Nx=96, Ny=97, coarse=12, L=2, k=6, guard=1, seed_block=None,
                desc="rectangle [0,1]x[0,1.01], uneven last coarse row"),
}

# The experiments of Section 6 in 2-D (Examples 6.1 and 6.2): coarse triangles as
# subdomains (shape "triangle"), delta/H = 1/4 in element layers, the paper's stop rule
# sum_i |lambda_i^{k+1} - lambda_i^k| < 1e-10 on the eigenvalues of the stated domain.
#   e1_*: (0,pi)^2, 16 x 16 coarse cells = 512 coarse triangles, s = 19 (Table 1)
#   e2_*: L-shape (-pi,pi)^2 minus [0,pi) x (-pi,0], 384 coarse triangles, s = 20 (Table 3)
for _N, _dofs in ((128, "16129"), (256, "65025"), (512, "261121"), (1024, "1046529")):
    CONFIGS[f"e1_{_N}"] = dict(Lx=np.pi, Ly=np.pi, Nx=_N, Ny=_N, coarse=_N // 16, L=_N // 64, k=19, guard=0,
                               seed_block=None, shape="triangle", stop="paper", tol=1e-10,
                               table1_col=(128, 256, 512, 1024).index(_N),
                               desc=(f"Example 6.1: Laplacian P1 (0,pi)^2, {_dofs} dofs, 512 coarse triangles, "
                                     f"delta/H=1/4, s=19, stop sum|dlambda|<1e-10"))
for _N, _dofs in ((128, "12033"), (256, "48641"), (512, "195585"), (1024, "784385")):
    CONFIGS[f"e2_{_N}"] = dict(domain="lshape", Lx=2 * np.pi, Ly=2 * np.pi, Nx=_N, Ny=_N, coarse=_N // 16,
                               L=_N // 64, k=20, guard=0, seed_block=None, shape="triangle", stop="paper",
                               tol=1e-10, table3_col=(128, 256, 512, 1024).index(_N),
                               desc=(f"Example 6.2: Laplacian P1 on the L-shape, {_dofs} dofs, 384 coarse "
                                     f"triangles, delta/H=1/4, s=20, stop sum|dlambda|<1e-10"))


def config_mesh(name: str) -> tuple[Mesh, dict]:
    """Build the mesh of a named workload; returns (mesh, config dict)."""
    cfg = dict(CONFIGS[name])
    if cfg.get("domain") == "lshape":
        mesh = p1_lshape(cfg["Nx"], cfg["coarse"])
    else:
        mesh = p1_mesh(cfg["Lx"], cfg["Ly"], cfg["Nx"], cfg["Ny"], cfg["coarse"])
    return mesh, cfg


def serving_requests(count: int = 256, base_seed: int = 2203, h_choices=(64, 128, 256, 512),
                     k_range=(4, 16), coarse_H: float = 1.0 / 8.0, L: int = 2, guard: int = 2):
    """Parameters of the served workload: one dict per request (meshes are built lazily).

    Request j draws from numpy.random.default_rng([base_seed, j]): the rectangle
    height r ~ U[1,2], a 4x4 block coefficient with values log-uniform in
    [0.1, 10], the mesh level 1/h from ``h_choices`` and k uniform in k_range.
    """
    reqs = []
    for j in range(count):
        rng = np.random.default_rng([base_seed, j])
        r = float(rng.uniform(1.0, 2.0))
        vals = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=(4, 4)))
        inv_h = int(rng.choice(np.asarray(h_choices)))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        Nx = inv_h
        Ny = int(round(r * inv_h))
        cpc = int(round(coarse_H * inv_h))
        reqs.append(dict(j=j, Lx=1.0, Ly=r, Nx=Nx, Ny=Ny, coarse=cpc, L=L, k=k, guard=guard,
                         coef_values=vals))
    return reqs


def request_mesh(req: dict) -> Mesh:
    coef = block_coefficient(req["Lx"], req["Ly"], req["coef_values"])
    return p1_mesh(req["Lx"], req["Ly"], req["Nx"], req["Ny"], req["coarse"], coef=coef)


# ----------------------------------------------------------------------------
# Fourth order: Bogner-Fox-Schmit elements on the unit square (m = 2)
@dataclass
class Plate:
    """BFS discretisation of Lap^2 u = lambda u on the unit square (N x N cells).

    Dofs sit on the fine vertices, four per vertex in the order u, u_x, u_y,
    u_xy; vertices are numbered row by row (x fastest), so a vertex's dofs are
    consecutive and the dofs of a subdomain keep the row-by-row order.
    """
    N: int
    bc: str                     # "clamped" (u = du/dn = 0) or "simply" (u = 0)
    K: sp.csr_matrix            # int Lap u Lap v, union pattern with M
    M: sp.csr_matrix            # int u v
    vert: np.ndarray            # (n, 2) int: fine vertex (ix, iy) of each dof
    kind: np.ndarray            # (n,) int: 0 u, 1 u_x, 2 u_y, 3 u_xy
    P: Optional[sp.csr_matrix] = None       # n x n_H nested coarse space
    subs: Optional[list] = None             # local dof sets (sorted int32 arrays)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.K.shape[0]


def _hermite_shapes(t: np.ndarray, h: float):
    """Cubic Hermite shape functions on [0, h] at t in [0, 1] (dof order: f(0),
    f'(0), f(h), f'(h)) with their first and second x-derivatives."""
    f = np.stack([1 - 3 * t**2 + 2 * t**3, h * (t - 2 * t**2 + t**3), 3 * t**2 - 2 * t**3, h * (t**3 - t**2)])
    d1 = np.stack([(-6 * t + 6 * t**2) / h, 1 - 4 * t + 3 * t**2, (6 * t - 6 * t**2) / h, 3 * t**2 - 2 * t])
    d2 = np.stack([(-6 + 12 * t) / h**2, (-4 + 6 * t) / h, (6 - 12 * t) / h**2, (6 * t - 2) / h])
    return f, d1, d2


def _free_1d(N: int, bc: str) -> np.ndarray:
    """Kept 1-D dofs (2 i: value at node i, 2 i + 1: slope) under the boundary condition."""
    drop = {0, 2 * N} if bc == "simply" else {0, 1, 2 * N, 2 * N + 1}
    if bc not in ("simply", "clamped"):
        raise ValueError("bc must be 'clamped' or 'simply'")
    return np.array([d for d in range(2 * N + 2) if d not in drop], dtype=np.int64)


def hermite_1d(N: int, bc: str = "clamped"):
    """1-D cubic Hermite matrices on [0, 1] with N cells: (mass, int f'g', int f''g'')
    restricted to the dofs kept by ``bc``, in node order (value, slope).  Element
    integrals by 5-point Gauss-Legendre quadrature (exact for these degree-6 products)."""
    h = 1.0 / N
    xg, wg = np.polynomial.legendre.leggauss(5)
    t = 0.5 * (xg + 1.0)
    w = 0.5 * wg * h
    f, d1, d2 = _hermite_shapes(t, h)
    Me = (f * w) @ f.T
    Ke = (d1 * w) @ d1.T
    Be = (d2 * w) @ d2.T
    nd = 2 * N + 2
    rows, cols, vm, vk, vb = [], [], [], [], []
    for e in range(N):
        dofs = np.arange(2 * e, 2 * e + 4)
        rows.append(np.repeat(dofs, 4))
        cols.append(np.tile(dofs, 4))
        vm.append(Me.ravel())
        vk.append(Ke.ravel())
        vb.append(Be.ravel())
    r, c = np.concatenate(rows), np.concatenate(cols)
    free = _free_1d(N, bc)
    out = []
    for v in (vm, vk, vb):
        A = sp.coo_matrix((np.concatenate(v), (r, c)), shape=(nd, nd)).tocsr()
        out.append(A[free][:, free].tocsr())
    return tuple(out)


def _vertex_major(N: int, bc: str):
    """Permutation from the Kronecker order (y dof major, x dof minor) of the kept
    1-D dofs to vertex-major order; returns (perm, vert, kind)."""
    free = _free_1d(N, bc)
    node, slope = free // 2, free % 2
    ny, nx = np.meshgrid(np.arange(len(free)), np.arange(len(free)), indexing="ij")
    ny, nx = ny.ravel(), nx.ravel()
    iy, ix = node[ny], node[nx]
    kind = slope[nx] + 2 * slope[ny]
    perm = np.lexsort((kind, ix, iy))
    return perm, np.stack([ix[perm], iy[perm]], 1), kind[perm]


def _hermite_prolongation_1d(N: int, Nc: int, bc: str) -> sp.csr_matrix:
    """Fine 1-D dofs of the coarse Hermite basis functions (values and slopes of the
    coarse cubic pieces at the fine nodes): the inclusion of the coarse space."""
    r = N // Nc
    Hc = 1.0 / Nc
    rows, cols, vals = [], [], []
    for i in range(N + 1):
        e = min(i // r, Nc - 1)
        t = np.array([(i - e * r) / r])
        f, d1, _ = _hermite_shapes(t, Hc)
        for a in range(4):
            cdof = 2 * e + a
            for fd, v in ((2 * i, f[a, 0]), (2 * i + 1, d1[a, 0])):
                if v != 0.0:
                    rows.append(fd)
                    cols.append(cdof)
                    vals.append(v)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(2 * N + 2, 2 * Nc + 2)).tocsr()
    A.sum_duplicates()
    return A[_free_1d(N, bc)][:, _free_1d(Nc, bc)].tocsr()


def bfs_plate(N: int, bc: str = "clamped", coarse: Optional[int] = None, L: int = 0) -> Plate:
    """BFS stiffness and mass of the unit square with N x N cells.

    Tensor-product Hermite functions f(x) g(y) give int Lap u Lap v =
    B (x) M + M (x) B + 2 K (x) K with the 1-D mass M, int f'g' = K and
    int f''g'' = B (int f''g = -int f'g' because g vanishes at both ends).
    With ``coarse`` (fine cells per coarse cell) the nested coarse space P and
    the local dof sets with ``L`` element layers of overlap are added.
    """
    M1, K1, B1 = hermite_1d(N, bc)
    K = (sp.kron(M1, B1) + sp.kron(B1, M1) + 2.0 * sp.kron(K1, K1)).tocsr()
    M = sp.kron(M1, M1).tocsr()
    perm, vert, kind = _vertex_major(N, bc)
    K = K[perm][:, perm]
    M = M[perm][:, perm]
    # one (union) pattern for both matrices, explicit zeros kept: both come from the same
    # (row, col) list (a sum that cancels to an exact zero keeps its entry)
    Kc, Mc = K.tocoo(), M.tocoo()
    r = np.concatenate([Kc.row, Mc.row])
    c = np.concatenate([Kc.col, Mc.col])
    zk, zm = np.zeros(Kc.nnz), np.zeros(Mc.nnz)
    Kp = sp.coo_matrix((np.concatenate([Kc.data, zm]), (r, c)), shape=K.shape).tocsr()
    Mp = sp.coo_matrix((np.concatenate([zk, Mc.data]), (r, c)), shape=M.shape).tocsr()
    for A in (Kp, Mp):
        A.sort_indices()
    assert np.array_equal(Kp.indptr, Mp.indptr) and np.array_equal(Kp.indices, Mp.indices)
    plate = Plate(N, bc, Kp, Mp, vert, kind, meta={"h": 1.0 / N})
    if coarse is not None:
        if N % coarse or bc != "clamped":
            raise ValueError("coarse cells must tile the mesh; local spaces need clamped edges")
        Nc = N // coarse
        P1 = _hermite_prolongation_1d(N, Nc, bc)
        pc, _, _ = _vertex_major(Nc, bc)
        P = sp.kron(P1, P1).tocsr()[perm][:, pc].tocsr()
        P.eliminate_zeros()
        P.sort_indices()
        plate.P = P
        subs = []
        ix, iy = vert[:, 0], vert[:, 1]
        for b in range(Nc):
            for a in range(Nc):
                inside = ((ix > a * coarse - L) & (ix < (a + 1) * coarse + L)
                          & (iy > b * coarse - L) & (iy < (b + 1) * coarse + L))
                subs.append(np.flatnonzero(inside).astype(np.int32))
        plate.subs = subs
        plate.meta.update(coarse=coarse, L=L, H=1.0 / Nc)
    return plate


# Named fourth-order workloads (clamped unit square, BFS): N fine cells per side,
# `coarse` fine cells per coarse cell, L overlap layers (delta = L h).
PLATE_CONFIGS = {
    "b16": dict(N=16, coarse=4, L=1, k=4, guard=1,
                desc="BFS plate h=1/16, 4x4 subdomains, delta=h, k=4"),
    "b32": dict(N=32, coarse=8, L=2, k=6, guard=2,
                desc="BFS plate h=1/32, 4x4 subdomains, delta=2h, k=6"),
    "b64": dict(N=64, coarse=8, L=2, k=6, guard=2,
                desc="BFS plate h=1/64, 8x8 subdomains, delta=2h, k=6"),
    "p128": dict(N=128, coarse=16, L=4, k=6, guard=2,
                 desc="clamped plate (biharmonic, BFS) h=1/128, 8x8 subdomains, delta=4h, k=6"),
    # at h = 1/256 FP64 vectors hold the relative residual of this fourth-order pencil
    # only to about u lambda_max / lambda_1 = 3e-6 (lambda_max = 3.7e13), so the stop
    # tolerance is that floor instead of 1e-8
    "c4": dict(N=256, coarse=32, L=4, k=6, guard=2, tol=3.2e-6,
               desc="clamped plate (biharmonic, BFS) h=1/256, 8x8 subdomains, delta=4h, k=6, residual 3.2e-6"),
}


def config_plate(name: str) -> tuple[Plate, dict]:
    """Build a named fourth-order workload; returns (plate, config dict)."""
    cfg = dict(PLATE_CONFIGS[name])
    return bfs_plate(cfg["N"], "clamped", cfg["coarse"], cfg["L"]), cfg


# ----------------------------------------------------------------------------
# Three dimensions: trilinear (Q1) elements on the cube (0,pi)^3 (Section 6, Example 6.3)
@dataclass
class Cube:
    """Q1 discretisation of -Lap u = lambda u on (0,pi)^3 with N^3 cells (Dirichlet).

    Dofs are the interior nodes (i, j, k), 1 <= i, j, k <= N - 1, numbered with i
    fastest.  K and M are tensor sums of the 1-D P1 stiffness K1 and mass M1 (the Q1
    basis functions are products of 1-D hats):  K = K1 (x) M1 (x) M1 + M1 (x) K1 (x) M1
    + M1 (x) M1 (x) K1, M = M1 (x) M1 (x) M1.  With ``coarse`` (fine cells per coarse
    cell) the caller's description of the two-level spaces is added: P, the coarse Q1
    hats written in fine dofs, and the local dof sets (the nodes of each closed coarse
    cube grown by L - 1 node layers: delta = L h).
    """
    N: int
    K: sp.csr_matrix
    M: sp.csr_matrix
    node: np.ndarray            # (n, 3) int: fine node (i, j, k) of each dof
    P: Optional[sp.csr_matrix] = None
    subs: Optional[list] = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.K.shape[0]


def _p1_1d(N: int, h: float):
    """1-D P1 stiffness and consistent mass on N cells of size h, interior nodes only."""
    m = N - 1
    K1 = sp.diags([-np.ones(m - 1), 2.0 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]) / h
    M1 = sp.diags([np.ones(m - 1), 4.0 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]) * (h / 6.0)
    return K1.tocsr(), M1.tocsr()


def _hat_prolongation_1d(N: int, Nc: int) -> sp.csr_matrix:
    """Coarse interior hats evaluated at the fine interior nodes ((N-1) x (Nc-1))."""
    r = N // Nc
    rows, cols, vals = [], [], []
    for c in range(1, Nc):
        for i in range(max(1, (c - 1) * r + 1), min(N, (c + 1) * r)):
            rows.append(i - 1)
            cols.append(c - 1)
            vals.append(1.0 - abs(i - c * r) / r)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N - 1, Nc - 1))


def q1_cube(N: int, coarse: Optional[int] = None, L: int = 1) -> Cube:
    h = np.pi / N
    K1, M1 = _p1_1d(N, h)
    K = (sp.kron(sp.kron(M1, M1), K1) + sp.kron(sp.kron(M1, K1), M1) + sp.kron(sp.kron(K1, M1), M1)).tocoo()
    M = sp.kron(sp.kron(M1, M1), M1).tocoo()
    # one (union) pattern for both matrices, explicit zeros kept
    r = np.concatenate([K.row, M.row])
    c = np.concatenate([K.col, M.col])
    Kp = sp.coo_matrix((np.concatenate([K.data, np.zeros(M.nnz)]), (r, c)), shape=K.shape).tocsr()
    Mp = sp.coo_matrix((np.concatenate([np.zeros(K.nnz), M.data]), (r, c)), shape=M.shape).tocsr()
    Kp.sort_indices()
    Mp.sort_indices()
    m = N - 1
    kk, jj, ii = np.meshgrid(np.arange(1, N), np.arange(1, N), np.arange(1, N), indexing="ij")
    node = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1)
    cube = Cube(N, Kp, Mp, node, meta={"h": h})
    if coarse is not None:
        if N % coarse:
            raise ValueError("coarse cells must tile the mesh")
        Nc = N // coarse
        P1 = _hat_prolongation_1d(N, Nc)
        cube.P = sp.kron(sp.kron(P1, P1), P1).tocsr()
        cube.P.sort_indices()
        subs = []
        for c3 in range(Nc):
            for c2 in range(Nc):
                for c1 in range(Nc):
                    lo = np.array([c1, c2, c3]) * coarse - (L - 1)
                    hi = (np.array([c1, c2, c3]) + 1) * coarse + (L - 1)
                    inside = np.all((node >= lo[None, :]) & (node <= hi[None, :]), axis=1)
                    subs.append(np.flatnonzero(inside).astype(np.int32))
        cube.subs = subs
        cube.meta.update(coarse=coarse, L=L, H=np.pi / Nc)
    assert m ** 3 == Kp.shape[0]
    return cube


# Example 6.3: (0,pi)^3, 8 x 8 x 8 coarse cubes (N = 512, H = pi/8), delta/H = 1/2 in
# node layers, s = 20, the paper's stop rule (Table 5).
CUBE_CONFIGS = {
    "e3_16": dict(N=16, coarse=2, L=1, k=20, guard=0, stop="paper", tol=1e-10, table5_col=0,
                  desc="Example 6.3: Laplacian Q1 (0,pi)^3, 3375 dofs, 512 coarse cubes, delta/H=1/2, s=20"),
    "e3_32": dict(N=32, coarse=4, L=2, k=20, guard=0, stop="paper", tol=1e-10, table5_col=1,
                  desc="Example 6.3: Laplacian Q1 (0,pi)^3, 29791 dofs, 512 coarse cubes, delta/H=1/2, s=20"),
}


def config_cube(name: str) -> tuple[Cube, dict]:
    cfg = dict(CUBE_CONFIGS[name])
    return q1_cube(cfg["N"], cfg["coarse"], cfg["L"]), cfg

"""Pins of the oracle's pieces for the experiments of Section 6 (Examples 6.1
and 6.2), and of its two measuring functions, against facts fixed outside the
oracle:

* the subdomains made of coarse triangles, against a closed-form graph metric
  of the "/" mesh (no breadth-first search);
* the L-shaped domain's discretisation, against the eigenvalues printed in
  Table 3 (Example 6.2);
* the coarse space of the L-shape: P^T K P equals the coarse stiffness matrix
  assembled on the coarse L-shaped mesh;
* Algorithm 3.1 on Example 6.1 at 16,129 dofs: eigenvalues of Table 1 and the
  iteration count the paper prints;
* the gap of Definition 2.1 on subspaces with known principal angles;
* the largest eigenvalue of the pencil against a dense eigensolve.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import bpjd_oracle as o
from paper_2203_06327_amd import workloads as w


# ---------------------------------------------------------------- coarse triangles
def _slash_distance(di, dj):
    """Graph distance on the "/" triangulation: steps (+-1, 0), (0, +-1), +-(1, 1)."""
    same = di * dj >= 0
    return np.where(same, np.maximum(np.abs(di), np.abs(dj)), np.abs(di) + np.abs(dj))


@pytest.mark.parametrize("layers", [1, 2, 3])
def test_triangle_subdomains_match_graph_metric(layers):
    """Omega_l = closed coarse triangle grown by (layers - 1) graph layers: every set
    equals the dofs within that distance of the triangle's dofs (Section 2.3,
    Section 6: the coarse elements are the subdomains)."""
    N, c = 32, 8
    mesh = w.p1_mesh(1.0, 1.0, N, N, c)
    subs = o.subdomain_sets(mesh.coords, mesh.cx, mesh.cy, mesh.K, mesh.M, layers, "triangle")
    assert len(subs) == 2 * (N // c) ** 2
    ij = np.rint(mesh.coords * N).astype(int)
    q = 0
    for B in range(N // c):
        for A in range(N // c):
            li, lj = ij[:, 0] - A * c, ij[:, 1] - B * c
            box = (li >= 0) & (li <= c) & (lj >= 0) & (lj <= c)
            for tri in (box & (li >= lj), box & (li <= lj)):   # below the diagonal, then above
                src = ij[tri]
                dist = _slash_distance(ij[:, None, 0] - src[None, :, 0], ij[:, None, 1] - src[None, :, 1]).min(1)
                expect = np.flatnonzero(dist <= layers - 1)
                np.testing.assert_array_equal(np.sort(subs[q]), expect)
                q += 1
    cover = np.zeros(mesh.n, dtype=int)
    for S in subs:
        cover[S] += 1
    assert cover.min() >= 1


def test_example_61_counts():
    """N = 512 coarse triangles on (0,pi)^2 with H = sqrt(2) pi / 16; the coarse
    space has the 15 x 15 interior coarse vertices."""
    mesh, cfg = w.config_mesh("e1_128")
    dd = o.build_dd(mesh, cfg["L"], "triangle")
    assert len(dd.subs) == 512 and dd.P.shape == (mesh.n, 225) and mesh.n == 16129
    H = np.hypot(mesh.cx[1] - mesh.cx[0], mesh.cy[1] - mesh.cy[0])
    assert abs(H - np.sqrt(2) * np.pi / 16) < 1e-14
    # delta / H = 1/4: 2 layers of fine triangles, each of diameter sqrt(2) pi / 128
    assert cfg["L"] * np.sqrt(2) * np.pi / 128 == pytest.approx(H / 4, rel=1e-14)


# ---------------------------------------------------------------- the L-shaped domain
def test_table3_reproduced(table3):
    """Table 3, column 1 (12033 dofs): all 20 printed eigenvalues to 8 decimals."""
    mesh = w.p1_lshape(128, 8)
    assert mesh.n == 12033
    lam, X = o.reference_eigs(mesh.K, mesh.M, 20)
    np.testing.assert_allclose(lam, table3[:, 0], rtol=0, atol=5.1e-9)
    np.testing.assert_allclose(X.T @ (mesh.M @ X), np.eye(20), atol=1e-10)


def test_lshape_coarse_space_is_galerkin():
    """The coarse vertices that carry a basis function are the free ones (161 of the
    225 interior vertices of the 16 x 16 coarse grid); P^T K_h P and P^T M_h P equal
    the matrices assembled on the coarse L-shaped mesh itself; 384 triangles."""
    fine = w.p1_lshape(64, 4)
    coarse = w.p1_lshape(16, 1)
    P = o.coarse_prolongation(fine.coords, fine.cx, fine.cy)
    assert P.shape == (fine.n, coarse.n) and coarse.n == 161
    np.testing.assert_allclose((P.T @ fine.K @ P).toarray(), coarse.K.toarray(), atol=1e-12)
    np.testing.assert_allclose((P.T @ fine.M @ P).toarray(), coarse.M.toarray(), atol=1e-14)
    subs = o.subdomain_sets(fine.coords, fine.cx, fine.cy, fine.K, fine.M, 1, "triangle")
    assert len(subs) == 384


# ---------------------------------------------------------------- Algorithm 3.1 on Example 6.1
def test_example_61_iteration_count(table1):
    """Example 6.1 at 16,129 dofs (N = 512, delta/H = 1/4, s = 19, stop at
    sum |dlambda| < 1e-10): the 19 eigenvalues of Table 1 column 1, and the
    count of Table 1 (21) within one -- the count after which the stop quantity
    falls below the tolerance; the paper does not say whether it counts that
    last Rayleigh-Ritz step."""
    mesh, cfg = w.config_mesh("e1_128")
    dd = o.build_dd(mesh, cfg["L"], "triangle")
    res = o.bpjd(mesh.K, mesh.M, dd, 19, 0, tol=1e-10, stop_rule="paper", subspace="UU", max_iter=60)
    assert res.converged and res.stop_value < 1e-10
    np.testing.assert_allclose(res.lam, table1[:, 0], rtol=0, atol=5.1e-9)
    assert abs(res.iterations - 21) <= 1, res.iterations


# ---------------------------------------------------------------- gap and lambda_max
def _eigvecs(name, count):
    mesh, _ = w.config_mesh(name)
    _, X = sla.eigh(mesh.K.toarray(), mesh.M.toarray())
    return mesh, X[:, :count]


@pytest.mark.parametrize("theta", [0.0, 1e-6, 0.3, np.pi / 2])
def test_subspace_gap_known_angle(theta):
    """Definition 2.1: span{u1, u2} against span{u1, cos t u2 + sin t u3} (u_i
    M-orthonormal) has gap sin t, whatever basis spans the second space."""
    mesh, U = _eigvecs("t8", 4)
    W1 = U[:, :2]
    v = np.cos(theta) * U[:, 1] + np.sin(theta) * U[:, 2]
    W2 = np.stack([2.0 * U[:, 0] + v, 3.0 * v], 1)           # a non-orthonormal basis
    g = o.subspace_gap_b(W1, W2, mesh.M)
    assert abs(g - np.sin(theta)) <= 1e-12 + 1e-8 * np.sin(theta), (g, np.sin(theta))
    assert abs(o.subspace_gap_b(W2, W1, mesh.M) - g) <= 1e-12 + 1e-8 * g   # equal dimensions: symmetric


def test_subspace_gap_is_the_largest_angle():
    """Two principal angles 0.1 and 0.4: the gap is sin 0.4 (not the smallest one,
    not a cosine)."""
    mesh, U = _eigvecs("t8", 4)
    a, b = 0.1, 0.4
    W1 = U[:, :2]
    W2 = np.stack([np.cos(a) * U[:, 0] + np.sin(a) * U[:, 3], np.cos(b) * U[:, 1] + np.sin(b) * U[:, 2]], 1)
    assert abs(o.subspace_gap_b(W1, W2, mesh.M) - np.sin(b)) < 1e-12


@pytest.mark.parametrize("name", ["t16", "b16", "b32"])
def test_largest_eigenvalue_against_dense(name):
    if name.startswith("b"):
        mesh, _ = w.config_plate(name)
    else:
        mesh, _ = w.config_mesh(name)
    top = sla.eigh(mesh.K.toarray(), mesh.M.toarray(), eigvals_only=True)[-1]
    assert o.largest_eigenvalue(mesh.K, mesh.M) == pytest.approx(top, rel=1e-6)

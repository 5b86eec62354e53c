"""Pins of the three-dimensional trilinear case (Section 6, Example 6.3) and of the
oracle's own 3-D spaces, against facts fixed outside the oracle:

* the closed form of tensor-product Q1 eigenvalues: lambda = mu_a + mu_b + mu_c
  with mu_j = (6/h^2)(1 - cos jh)/(2 + cos jh), the 1-D P1 eigenvalues with a
  consistent mass on (0,pi);
* the eigenvalues Table 5 prints for 3375 and 29,791 dofs;
* the Galerkin identity P^T K_h P = K_H on nested trilinear spaces;
* the oracle's coarse space and local sets equal the caller's description
  that the library receives (the two are built by different routes);
* Algorithm 3.1 as written (W grows) on 3375 dofs: the 20 eigenvalues of
  Table 5 and the iteration count the paper prints for that column.
"""
import numpy as np
import pytest

from oracle import bpjd_oracle as o
from oracle import q1_space as q
from paper_2203_06327_amd import workloads as w


def _closed_form(N, count):
    h = np.pi / N
    j = np.arange(1, N)
    mu = 6.0 / h ** 2 * (1.0 - np.cos(j * h)) / (2.0 + np.cos(j * h))
    return np.sort((mu[:, None, None] + mu[None, :, None] + mu[None, None, :]).ravel())[:count]


@pytest.mark.parametrize("name,col", [("e3_16", 0), ("e3_32", 1)])
def test_table5_and_closed_form(table5, name, col):
    cube, cfg = w.config_cube(name)
    lam, X = o.reference_eigs(cube.K, cube.M, 20)
    np.testing.assert_allclose(lam, _closed_form(cfg["N"], 20), rtol=1e-12)
    np.testing.assert_allclose(lam, table5[:, col], rtol=0, atol=5.1e-9)
    np.testing.assert_allclose(X.T @ (cube.M @ X), np.eye(20), atol=1e-10)


def test_cube_spaces_and_galerkin_identity():
    N, Nc, L = 16, 4, 2
    cube = w.q1_cube(N, N // Nc, L)
    P = q.coarse_space(N, Nc)
    assert abs(P - cube.P).max() < 1e-15
    subs = q.local_spaces(N, Nc, L)
    assert len(subs) == Nc ** 3 and all(np.array_equal(a, b) for a, b in zip(subs, cube.subs))
    coarse = w.q1_cube(Nc)
    np.testing.assert_allclose((P.T @ cube.K @ P).toarray(), coarse.K.toarray(), atol=1e-12)
    np.testing.assert_allclose((P.T @ cube.M @ P).toarray(), coarse.M.toarray(), atol=1e-14)
    # an interior local space: the closed coarse cube (5 nodes a side) grown by one layer
    assert max(len(S) for S in subs) == 7 ** 3
    cover = np.zeros(cube.n, dtype=int)
    for S in subs:
        cover[S] += 1
    assert cover.min() >= 1


def test_example_63_iteration_count(table5):
    """3375 dofs (N = 512 coarse cubes, delta/H = 1/2, s = 20, stop at sum |dlambda| <
    1e-10) with W growing by span{t_i} each step, as Algorithm 3.1 states: the
    eigenvalues of Table 5, column 1, and its count (14)."""
    cube, cfg = w.config_cube("e3_16")
    Nc = cfg["N"] // cfg["coarse"]
    dd = o.DD(q.coarse_space(cfg["N"], Nc), q.local_spaces(cfg["N"], Nc, cfg["L"]))
    res = o.bpjd(cube.K, cube.M, dd, 20, 0, tol=1e-10, stop_rule="paper", subspace="GROW", max_iter=60)
    assert res.converged
    np.testing.assert_allclose(res.lam, table5[:, 0], rtol=0, atol=5.1e-9)
    assert res.iterations == 14

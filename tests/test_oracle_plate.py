"""Pins of the fourth-order (m = 2) case: the Bogner-Fox-Schmit inputs and the
oracle's coarse and local spaces, checked against closed forms and exact
identities, and the oracle's Algorithm 3.1 on a clamped plate against a dense
solve.  CPU only.

* 1-D cubic Hermite matrices: the clamped-clamped beam f'''' = mu f has
  mu_i = beta_i^4 with cos(beta) cosh(beta) = 1 (beta_1 = 4.730040744862704);
  the simply supported beam has (i pi)^4, the string -f'' = mu f has (i pi)^2.
* Simply supported plate (u = Lap u = 0): Lap^2 u = lambda u has the separable
  eigenfunctions sin(i pi x) sin(j pi y), lambda = pi^4 (i^2 + j^2)^2, with their
  multiplicities; BFS eigenvalues converge to them as h^4.
* Clamped plate: no closed form; the first eigenvalue is known to high accuracy,
  1294.9339795917 (Bjorstad and Tjostheim, high-precision solutions of fourth
  order eigenvalue problems, 1999); the second is double by the x <-> y symmetry.
* Nestedness (Section 2.3 requires V^H in V^h): P^T K P and P^T M P equal the
  coarse BFS matrices assembled directly, and the oracle's coarse space (built from
  4 x 4 Hermite solves) equals the generator's.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import bfs_space as bs
from oracle import bpjd_oracle as o
from paper_2203_06327_amd import workloads as w

BETA = [4.730040744862704, 7.853204624095838]          # roots of cos(b) cosh(b) = 1
CLAMPED_PLATE_1 = 1294.9339795917


def _eig(K, M, k):
    return sla.eigh(K.toarray(), M.toarray(), eigvals_only=True, subset_by_index=[0, k - 1])


def test_hermite_1d_beam_and_string():
    err = []
    for N in (8, 16):
        M1, K1, B1 = w.hermite_1d(N, "clamped")
        mu = _eig(B1, M1, 2)
        err.append(np.abs(mu / np.array(BETA) ** 4 - 1.0))
        M1, K1, B1 = w.hermite_1d(N, "simply")
        np.testing.assert_allclose(_eig(B1, M1, 3), (np.pi * np.arange(1, 4)) ** 4, rtol=5e-3 if N == 8 else 3e-4)
        np.testing.assert_allclose(_eig(K1, M1, 3), (np.pi * np.arange(1, 4)) ** 2, rtol=1e-4)
    assert err[1][0] < 2e-5 and err[1][1] < 1.5e-4
    ratio = err[0] / err[1]
    assert np.all(ratio > 12) and np.all(ratio < 20)          # h^4


def _ss_limits(k):
    vals = sorted(np.pi ** 4 * (i * i + j * j) ** 2 for i in range(1, 8) for j in range(1, 8))
    return np.array(vals[:k])


def test_simply_supported_plate_closed_form():
    k = 6
    exact = _ss_limits(k)                        # 4, 25, 25, 64, 100, 100 (times pi^4)
    np.testing.assert_allclose(exact / np.pi ** 4, [4, 25, 25, 64, 100, 100])
    errs = []
    for N in (8, 16):
        pl = w.bfs_plate(N, "simply")
        lam = _eig(pl.K, pl.M, k)
        errs.append(lam / exact - 1.0)
        # multiplicities: the pairs (1,2)/(2,1) and (1,3)/(3,1) stay exactly double
        assert abs(lam[1] - lam[2]) <= 1e-9 * lam[2] and abs(lam[4] - lam[5]) <= 1e-9 * lam[5]
    assert np.all(errs[0] > 0) and np.all(errs[1] > 0)           # conforming: from above
    assert np.abs(errs[1]).max() < 2e-4
    assert np.all(errs[0] / errs[1] > 12)


def test_clamped_plate_first_eigenvalue():
    errs = []
    for N in (8, 16, 32):
        pl = w.bfs_plate(N, "clamped")
        lam = _eig(pl.K, pl.M, 3)
        errs.append(lam[0] / CLAMPED_PLATE_1 - 1.0)
        assert abs(lam[1] - lam[2]) <= 1e-9 * lam[2]
    assert errs[2] > 0 and errs[2] < 2e-6
    assert errs[0] / errs[1] > 10 and errs[1] / errs[2] > 12


@pytest.mark.parametrize("name", ["b16", "b32"])
def test_coarse_space_nested(name):
    pl, cfg = w.config_plate(name)
    Nc = cfg["N"] // cfg["coarse"]
    P = bs.coarse_space(cfg["N"], Nc, pl.vert, pl.kind)
    assert abs(P - pl.P).max() <= 1e-12 * abs(P).max()
    coarse = w.bfs_plate(Nc, "clamped")
    for A, AH in ((pl.K, coarse.K), (pl.M, coarse.M)):
        G = (P.T @ A @ P).toarray()
        assert np.abs(G - AH.toarray()).max() <= 1e-12 * np.abs(AH).max()


def test_coarse_space_catches_a_wrong_slope():
    """A coarse function with one wrong derivative value is not in the fine space's
    Galerkin identity: the check above would catch such a slip."""
    pl, cfg = w.config_plate("b16")
    Nc = cfg["N"] // cfg["coarse"]
    P = bs.coarse_space(cfg["N"], Nc, pl.vert, pl.kind).tolil()
    r = int(np.flatnonzero(pl.kind == 1)[7])
    c = int(P.rows[r][0])
    P[r, c] = P[r, c] * 1.01
    P = P.tocsr()
    coarse = w.bfs_plate(Nc, "clamped")
    G = (P.T @ pl.K @ P).toarray()
    assert np.abs(G - coarse.K.toarray()).max() > 1e-6 * np.abs(coarse.K).max()


@pytest.mark.parametrize("name", ["b16", "b32", "c4"])
def test_local_spaces(name):
    pl, cfg = w.config_plate(name)
    Nc = cfg["N"] // cfg["coarse"]
    subs = bs.local_spaces(cfg["N"], Nc, cfg["L"], pl.vert)
    assert len(subs) == Nc * Nc
    assert all(np.array_equal(a, b) for a, b in zip(subs, pl.subs))
    assert np.array_equal(np.unique(np.concatenate(subs)), np.arange(pl.n))
    # an interior cell grown by L layers holds (coarse + 2L - 1)^2 vertices, 4 dofs each
    assert max(len(S) for S in subs) == 4 * (cfg["coarse"] + 2 * cfg["L"] - 1) ** 2


def test_oracle_bpjd_clamped_plate():
    """Algorithm 3.1 on the clamped plate (b16) reaches the dense solve's eigenpairs."""
    pl, cfg = w.config_plate("b16")
    Nc = cfg["N"] // cfg["coarse"]
    dd = o.DD(bs.coarse_space(cfg["N"], Nc, pl.vert, pl.kind), bs.local_spaces(cfg["N"], Nc, cfg["L"], pl.vert))
    k = cfg["k"]
    r = o.bpjd(pl.K, pl.M, dd, k, cfg["guard"], tol=1e-8, max_iter=200)
    lam_ref, X_ref = o.reference_eigs(pl.K, pl.M, k)
    assert r.converged and r.iterations <= 40
    np.testing.assert_allclose(r.lam[:k], lam_ref, rtol=1e-10)
    assert o.residual_norms(pl.K, pl.M, r.X[:, :k], r.lam[:k]).max() <= 1e-8
    np.testing.assert_allclose(r.X[:, :k].T @ (pl.M @ r.X[:, :k]), np.eye(k), atol=1e-10)
    # Ritz values decrease monotonically towards the eigenvalues
    H = np.array(r.history)[:, :k]
    assert np.all(np.diff(H, axis=0) <= 1e-9 * H[:-1])


def test_local_solve_keeps_scaled_dofs_accurate():
    """The oracle's local solves on the b32 plate (raw condition about 5e8, most of it
    from derivative dofs carrying powers of h) against the same solves refined in
    extended precision (residuals in long double): every dof kind to 1e-13 of its
    largest value."""
    pl, cfg = w.config_plate("b32")
    Nc = cfg["N"] // cfg["coarse"]
    subs = bs.local_spaces(cfg["N"], Nc, cfg["L"], pl.vert)
    S = max(subs, key=len)
    Kl, Ml = pl.K[S][:, S], pl.M[S][:, S]
    kind = pl.kind[S]
    rng = np.random.default_rng(3)
    X = rng.standard_normal((pl.n, 2))
    F = (pl.M @ X) * 25000.0 - pl.K @ X                 # residual-like right-hand sides
    A = (Kl - 25000.0 * Ml).tocsc()
    Ad = A.toarray()
    Al = Ad.astype(np.longdouble)
    for i in range(2):
        f = F[S, i]
        z = o.spd_solve(A, f)
        x = np.linalg.solve(Ad, f)
        for _ in range(4):
            r = (f.astype(np.longdouble) - Al @ x.astype(np.longdouble)).astype(np.float64)
            x = x + np.linalg.solve(Ad, r)
        for q in range(4):
            m = kind == q
            assert np.abs(z[m] - x[m]).max() <= 1e-13 * np.abs(x[m]).max()

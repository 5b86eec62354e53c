"""Plain FP64 CPU oracle of the two-level BPJD method (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module; the product path (the
HIP library and its Python binding) never does.  It shares no code with the
library: it reads the same seeded inputs (meshes, matrices, random blocks) and
implements every step of the method itself, slowly and literally, in float64
with numpy/scipy.

What it computes (reference: Liang, Wang, Xu, "A Two-Level Block
Preconditioned Jacobi-Davidson Method for Multiple and Clustered Eigenvalues
of Elliptic Operators"):

* ``reference_eigs`` -- the plain definition of the result: the k smallest
  eigenpairs of the symmetric-definite pencil (K, M) of the discrete problem
  (Section 2.2, eq. DiscreteVariational), with X^T M X = I.
* ``build_dd`` / ``coarse_prolongation`` -- the domain decomposition of
  Section 2.3: coarse cells enlarged by fine element layers (overlap delta),
  local spaces V^(l) = interior dofs of the enlarged cells, coarse space V^H.
* ``precondition`` -- the two-level preconditioner (eq. Preconditioner),
  one shift lambda_i per column, in matrix form.
* ``bpjd`` -- Algorithm 3.1 (Steps 1-4) with the subspace choices of the
  remark that follows it (grow W, W = U^k + span{t}, W = U^{k-1}+U^k+span{t}).

Readings of points the paper leaves open (each documented in the design
notes of the repository): Step 1 uses H~ = H (the remark after Alg. 3.1);
the projection of Step 2 is I - X X^T M (its matrix-form remark, resolving the
reused summation index); residual r_i is represented by F_i = lambda_i M x_i
- K x_i; rank-deficient directions of W are dropped.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "DD", "build_dd", "coarse_prolongation", "subdomain_sets", "CoarseSetup", "coarse_setup",
    "LocalSetup", "local_setup", "precondition", "coarse_term", "coarse_term_direct",
    "local_term", "spd_solve", "m_orthonormalize", "rayleigh_ritz", "bpjd", "BPJDResult",
    "reference_eigs", "residual_norms", "subspace_gap_b", "largest_eigenvalue",
]


# --------------------------------------------------------------------------
# Domain decomposition (Section 2.3)
# --------------------------------------------------------------------------
@dataclass
class DD:
    P: sp.csr_matrix            # n x n_H coarse prolongation, range(P) = V^H inside V^h
    subs: list                  # list of sorted int arrays: dofs of V^(l)


def coarse_prolongation(coords: np.ndarray, cx: np.ndarray, cy: np.ndarray) -> sp.csr_matrix:
    """Nodal interpolation of the coarse P1 space into the fine dofs.

    The coarse mesh is the grid of lines cx x cy with every coarse cell cut
    by its "/" diagonal (the same triangulation rule as the fine mesh, so
    V^H is a subspace of V^h when coarse cells are unions of fine cells
    along the diagonal).  A coarse vertex carries a basis function of V^H when
    a fine dof sits on it (the free vertices of the coarse mesh: on a
    rectangle every interior one, on the L-shaped domain those off the
    re-entrant edges and the removed quadrant).  Columns follow the coarse
    vertices row by row (x fastest).
    """
    n = coords.shape[0]
    ncx, ncy = len(cx) - 1, len(cy) - 1
    x, y = coords[:, 0], coords[:, 1]
    tol = 1e-9 * min(np.min(np.diff(cx)), np.min(np.diff(cy)))
    # free coarse vertices: coincide with a fine dof
    col_of = {}
    for B in range(1, ncy):
        for A in range(1, ncx):
            if np.any((np.abs(x - cx[A]) <= tol) & (np.abs(y - cy[B]) <= tol)):
                col_of[(A, B)] = len(col_of)
    a = np.clip(np.searchsorted(cx, x, side="right") - 1, 0, ncx - 1)
    b = np.clip(np.searchsorted(cy, y, side="right") - 1, 0, ncy - 1)
    xi = (x - cx[a]) / (cx[a + 1] - cx[a])
    eta = (y - cy[b]) / (cy[b + 1] - cy[b])
    rows, cols, vals = [], [], []
    for d in range(n):
        A, B = a[d], b[d]
        if xi[d] >= eta[d]:      # lower-right triangle (A,B),(A+1,B),(A+1,B+1)
            verts = [(A, B, 1.0 - xi[d]), (A + 1, B, xi[d] - eta[d]), (A + 1, B + 1, eta[d])]
        else:                    # upper-left triangle (A,B),(A+1,B+1),(A,B+1)
            verts = [(A, B, 1.0 - eta[d]), (A + 1, B + 1, xi[d]), (A, B + 1, eta[d] - xi[d])]
        for (VA, VB, wv) in verts:
            c = col_of.get((VA, VB))
            if c is not None and wv != 0.0:
                rows.append(d)
                cols.append(c)
                vals.append(wv)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, len(col_of)))


def subdomain_sets(coords, cx, cy, K, M, layers: int, shape: str = "square") -> list:
    """Local dof sets of the overlapping subdomains Omega'_l.

    Omega_l is a closed coarse cell (shape "square"), or one of the two closed
    coarse triangles a coarse cell is cut into by its "/" diagonal (shape
    "triangle": the coarse elements themselves, as in the experiments of
    Section 6); it is enlarged by ``layers`` layers of fine elements (every
    element touching the current region is added).  The dofs of V^(l) are those
    interior to the enlarged region: the dofs of the closed cell plus those
    within graph distance layers-1 of them in the element adjacency graph (the
    union pattern of K and M).  Triangles are listed cell by cell, the lower-right
    one (below the diagonal) first.
    """
    if layers < 1:
        raise ValueError("overlap must be at least one element layer")
    if shape not in ("square", "triangle"):
        raise ValueError(shape)
    adj = (abs(K) + abs(M)).tocsr()
    adj = (adj != 0).astype(np.int8)
    x, y = coords[:, 0], coords[:, 1]
    tol = 1e-9 * min(np.min(np.diff(cx)), np.min(np.diff(cy)))
    subs = []
    for B in range(len(cy) - 1):
        for A in range(len(cx) - 1):
            inside = (x >= cx[A] - tol) & (x <= cx[A + 1] + tol) & (y >= cy[B] - tol) & (y <= cy[B + 1] + tol)
            if shape == "square":
                parts = [inside]
            else:
                # position along the cell's diagonal: xi - eta >= 0 below it, <= 0 above
                d = (x - cx[A]) / (cx[A + 1] - cx[A]) - (y - cy[B]) / (cy[B + 1] - cy[B])
                parts = [inside & (d >= -1e-9), inside & (d <= 1e-9)]
            for part in parts:
                mask = part.astype(np.int8)
                for _ in range(layers - 1):
                    mask = ((adj @ mask) > 0).astype(np.int8) | mask
                idx = np.flatnonzero(mask)
                if idx.size:
                    subs.append(idx.astype(np.int64))
    return subs


def build_dd(mesh, layers: int, shape: str = "square") -> DD:
    P = coarse_prolongation(mesh.coords, mesh.cx, mesh.cy)
    subs = subdomain_sets(mesh.coords, mesh.cx, mesh.cy, mesh.K, mesh.M, layers, shape)
    return DD(P=P, subs=subs)


# --------------------------------------------------------------------------
# Coarse space and local spaces (Section 3: Q^H, Q^(l), A^H, A^(l))
# --------------------------------------------------------------------------
@dataclass
class CoarseSetup:
    P: sp.csr_matrix
    KH: np.ndarray
    MH: np.ndarray
    lamH: np.ndarray            # all coarse eigenvalues, ascending
    Y: np.ndarray               # coarse eigenvectors, Y^T M_H Y = I


def coarse_setup(K, M, P) -> CoarseSetup:
    """Galerkin coarse operators and the full coarse spectral decomposition
    V^H = U_s^H (+) U_{s+1}^H (Section 3, eq. EigenvalueCoarse)."""
    KH = (P.T @ (K @ P)).toarray()
    MH = (P.T @ (M @ P)).toarray()
    KH = 0.5 * (KH + KH.T)
    MH = 0.5 * (MH + MH.T)
    lamH, Y = sla.eigh(KH, MH)
    return CoarseSetup(P=P, KH=KH, MH=MH, lamH=lamH, Y=Y)


@dataclass
class LocalSetup:
    subs: list
    K_loc: list                 # K_l = R_l K R_l^T
    M_loc: list                 # M_l = R_l M R_l^T


def local_setup(K, M, subs) -> LocalSetup:
    Kc, Mc = K.tocsr(), M.tocsr()
    K_loc = [Kc[S][:, S].tocsc() for S in subs]
    M_loc = [Mc[S][:, S].tocsc() for S in subs]
    return LocalSetup(subs=subs, K_loc=K_loc, M_loc=M_loc)


def coarse_term(F: np.ndarray, lam: np.ndarray, cs: CoarseSetup, s: int) -> np.ndarray:
    """P (B_0,i)^{-1} Q^H_{s+1} Q^H r_i for every column i.

    Q^H r_i has coarse coefficients M_H^{-1} P^T F_i; Q^H_{s+1} removes the
    components along the first s coarse eigenvectors; on U_{s+1}^H the operator
    A^H - lambda_i acts on y_j as (lambda^H_j - lambda_i).
    """
    G = cs.P.T @ F                                   # n_H x s
    Ys = cs.Y[:, s:]                                 # eigenvectors j > s
    C = Ys.T @ G                                     # (n_H - s) x s
    denom = cs.lamH[s:, None] - lam[None, :]
    zH = Ys @ (C / denom)
    return cs.P @ zH


def coarse_term_direct(F: np.ndarray, lam: np.ndarray, cs: CoarseSetup, s: int) -> np.ndarray:
    """The same coarse term by a dense solve instead of the eigenbasis.

    Solves (K_H - lambda_i M_H + M_H Y_s c Y_s^T M_H) z = (I - M_H Y_s Y_s^T) G_i
    with the shift c = lambda^H_{s+1} on U_s^H, which leaves the action on
    U_{s+1}^H unchanged and makes the matrix nonsingular.
    """
    G = cs.P.T @ F
    Ys = cs.Y[:, :s]
    MY = cs.MH @ Ys
    c = cs.lamH[s]
    out = np.empty_like(G)
    for i in range(G.shape[1]):
        A = cs.KH - lam[i] * cs.MH + c * (MY @ MY.T)
        rhs = G[:, i] - MY @ (Ys.T @ G[:, i])
        out[:, i] = np.linalg.solve(A, rhs)
    return cs.P @ out


def _cholesky(A):
    """Cholesky factor of the symmetric sparse matrix A (dense up to 400 rows,
    banded above), or None when A is not positive definite."""
    n = A.shape[0]
    try:
        if n <= 400:
            return ("dense", sla.cho_factor(A.toarray(), lower=True))
        C = A.tocoo()
        low = C.row >= C.col
        d = C.row[low] - C.col[low]
        ab = np.zeros((int(d.max()) + 1, n))
        ab[d, C.col[low]] = C.data[low]
        return ("band", sla.cholesky_banded(ab, lower=True))
    except np.linalg.LinAlgError:
        return None


def _cholesky_solve(fac, b: np.ndarray) -> np.ndarray:
    kind, f = fac
    return sla.cho_solve(f, b) if kind == "dense" else sla.cho_solve_banded((f, True), b)


def positive_definite(A) -> bool:
    """Whether the symmetric sparse matrix A is positive definite: its Cholesky
    factorisation (dense up to 400 rows, banded above) runs to the end."""
    return _cholesky(A) is not None


def local_shift(Kl, Ml, lam_i: float) -> float:
    """Shift of one local solve: lambda_i where K_l - lambda_i M_l is positive
    definite, as the paper's analysis has it (lambda_min(B_l,i) of order H^{-2m},
    far above lambda_i); 0 where a subdomain breaks that premise (a strong
    coefficient contrast puts a local Dirichlet eigenvalue below lambda_i), so that
    the local problem stays a positive definite Schwarz solve."""
    return lam_i if positive_definite((Kl - lam_i * Ml).tocsc()) else 0.0


def spd_solve(A, b: np.ndarray) -> np.ndarray:
    """Solve A z = b for a symmetric positive definite sparse A by Cholesky.  Its
    rounding error depends only on the diagonally scaled matrix, so dofs of very
    different sizes (the derivative dofs of the fourth-order elements carry powers
    of h) keep full accuracy."""
    fac = _cholesky(A)
    if fac is None:
        raise np.linalg.LinAlgError("matrix is not positive definite")
    return _cholesky_solve(fac, b)


def local_term(F: np.ndarray, lam: np.ndarray, ls: LocalSetup) -> np.ndarray:
    """sum_l R_l^T (K_l - sigma_{l,i} M_l)^{-1} R_l F_i (unweighted sum), with
    sigma_{l,i} = local_shift(K_l, M_l, lambda_i): lambda_i on every subdomain
    where the paper's premise holds.  The Cholesky factorisation that decides the
    shift is the one that solves (K_l alone is positive definite)."""
    Z = np.zeros_like(F)
    for S, Kl, Ml in zip(ls.subs, ls.K_loc, ls.M_loc):
        for i in range(F.shape[1]):
            fac = _cholesky((Kl - lam[i] * Ml).tocsc())
            if fac is None:                       # local_shift gives 0 here
                fac = _cholesky(Kl.tocsc())
            Z[S, i] += _cholesky_solve(fac, F[S, i])
    return Z


def precondition(F: np.ndarray, lam: np.ndarray, cs: CoarseSetup, ls: LocalSetup, s: int,
                 use_coarse: bool = True, use_local: bool = True) -> np.ndarray:
    """Z_i = (B_i^k)^{-1} r_i, eq. (Preconditioner), in matrix form."""
    Z = np.zeros_like(F)
    if use_coarse:
        Z += coarse_term(F, lam, cs, s)
    if use_local:
        Z += local_term(F, lam, ls)
    return Z


# --------------------------------------------------------------------------
# Subspace pieces (Step 3)
# --------------------------------------------------------------------------
def m_orthonormalize(cols: np.ndarray, M, basis: np.ndarray | None = None, drop: float = 1e-12):
    """Gram-Schmidt in the M inner product, one column at a time, with
    repeated projection ("twice is enough"); a column whose remaining norm is
    below ``drop`` times its norm before projection is dropped (linearly
    dependent on what is already in the basis).  ``basis`` (M-orthonormal) is
    kept and extended.  Returns the extended basis."""
    Q = [] if basis is None else [basis[:, j] for j in range(basis.shape[1])]
    for j in range(cols.shape[1]):
        w = cols[:, j].copy()
        nrm0 = np.sqrt(max(w @ (M @ w), 0.0))
        if nrm0 == 0.0:
            continue
        nrm = nrm0
        for _ in range(4):
            if Q:
                Qm = np.stack(Q, 1)
                w -= Qm @ (Qm.T @ (M @ w))
            new = np.sqrt(max(w @ (M @ w), 0.0))
            ratio = new / nrm
            nrm = new
            if ratio > 0.5:
                break
        if nrm <= drop * nrm0:
            continue
        Q.append(w / nrm)
    return np.stack(Q, 1)


def rayleigh_ritz(W: np.ndarray, K, s: int):
    """First s Ritz pairs of the pencil on span(W), W M-orthonormal (eq. UpdateRayleighRitz)."""
    H = W.T @ (K @ W)
    H = 0.5 * (H + H.T)
    theta, V = np.linalg.eigh(H)
    return theta[:s], W @ V[:, :s]


def residual_norms(K, M, X, lam):
    """rho_i = ||K x_i - lambda_i M x_i||_2 / (lambda_i ||M x_i||_2)."""
    MX = M @ X
    R = K @ X - MX * lam[None, :]
    return np.linalg.norm(R, axis=0) / (np.abs(lam) * np.linalg.norm(MX, axis=0))


@dataclass
class BPJDResult:
    lam: np.ndarray
    X: np.ndarray
    iterations: int
    converged: bool
    history: list = field(default_factory=list)     # Lambda^k for k = 0, 1, ...
    rho_history: list = field(default_factory=list)
    stop_value: float = float("nan")                # sum_i |lambda_i^{k+1} - lambda_i^k| at exit
    dimW: list = field(default_factory=list)


def bpjd(K, M, dd: DD, k: int, guard: int = 0, tol: float = 1e-8, stop_rule: str = "residual",
         subspace: str = "UU", max_iter: int = 200, X_init: np.ndarray | None = None,
         setups=None) -> BPJDResult:
    """Algorithm 3.1 (two-level BPJD) for the first k eigenpairs of (K, M).

    s = k + guard block columns (Assumption 1 and its remark).  Subspace
    choice (remark after Alg. 3.1): "GROW" W^{k+1} = W^k + span{t}, "U"
    W^{k+1} = U^k + span{t}, "UU" W^{k+1} = U^{k-1} + U^k + span{t}.
    Stop rule: "paper" stops when sum_i |lambda_i^{k+1}-lambda_i^k| < tol (Step 4);
    "residual" stops when max_{i<=k} rho_i <= tol.
    """
    s = k + guard
    K = K.tocsr()
    M = M.tocsr()
    if setups is None:
        cs = coarse_setup(K, M, dd.P)
        ls = local_setup(K, M, dd.subs)
    else:
        cs, ls = setups
    if s >= cs.lamH.size:
        raise ValueError("need s < dim V^H")
    # Step 1 (with H~ = H): Galerkin coarse eigenvectors as the initial block
    X = dd.P @ cs.Y[:, :s]
    lam = cs.lamH[:s].copy()
    if X_init is not None:
        W = m_orthonormalize(np.hstack([X, X_init]), M)
        lam, X = rayleigh_ritz(W, K, s)
    res = BPJDResult(lam=lam, X=X, iterations=0, converged=False)
    res.history.append(lam.copy())
    W = X.copy()
    X_prev = None
    for it in range(max_iter + 1):
        MX = M @ X
        F = MX * lam[None, :] - K @ X
        rho = np.linalg.norm(F, axis=0) / (np.abs(lam) * np.linalg.norm(MX, axis=0))
        res.rho_history.append(rho.copy())
        if stop_rule == "residual" and np.max(rho[:k]) <= tol:
            res.converged = True
            break
        if it == max_iter:
            break
        # Step 2: t_i = (I - Q_{U^k}) (B_i^k)^{-1} r_i
        Z = precondition(F, lam, cs, ls, s)
        T = Z - X @ (MX.T @ Z)
        # Step 3: Rayleigh-Ritz on W^{k+1}
        if subspace == "GROW":
            W = m_orthonormalize(T, M, basis=W)
        elif subspace == "U":
            W = m_orthonormalize(T, M, basis=X)
        elif subspace == "UU":
            base = X if X_prev is None else m_orthonormalize(X_prev, M, basis=X)
            W = m_orthonormalize(T, M, basis=base)
        else:
            raise ValueError(subspace)
        lam_new, X_new = rayleigh_ritz(W, K, s)
        res.dimW.append(W.shape[1])
        stop_val = float(np.sum(np.abs(lam_new - lam)))
        X_prev, X, lam = X, X_new, lam_new
        res.iterations = it + 1
        res.history.append(lam.copy())
        res.stop_value = stop_val
        if stop_rule == "paper" and stop_val < tol:
            res.converged = True
            MX = M @ X
            F = MX * lam[None, :] - K @ X
            res.rho_history.append(np.linalg.norm(F, axis=0) / (np.abs(lam) * np.linalg.norm(MX, axis=0)))
            break
    res.lam, res.X = lam[:k].copy(), X[:, :k].copy()
    return res


# --------------------------------------------------------------------------
# The plain definition of the result
# --------------------------------------------------------------------------
def reference_eigs(K, M, k: int):
    """k smallest eigenpairs of K x = lambda M x with X^T M X = I (ascending).

    Dense symmetric-definite solve for n <= 3000, otherwise shift-invert
    Lanczos about 0 (the pencil is positive definite, so the eigenvalues
    nearest 0 are the smallest) followed by a Rayleigh-Ritz step on the
    Lanczos vectors: a Rayleigh quotient's error is the square of its vector's,
    while the Lanczos values carry the rounding of the factorised K, whose
    condition grows as h^-2m.
    """
    n = K.shape[0]
    if n <= 3000:
        lam, X = sla.eigh(K.toarray(), M.toarray(), subset_by_index=[0, k - 1])
    else:
        lam, X = spla.eigsh(K.tocsc(), k=k, M=M.tocsc(), sigma=0.0, which="LM", tol=1e-14)
        order = np.argsort(lam)
        lam, X = lam[order], X[:, order]
        # Rayleigh-Ritz on span X: values in ascending order, X^T M X = I
        KX, MX = K @ X, M @ X
        A = X.T @ KX
        G = X.T @ MX
        lam, Q = sla.eigh(0.5 * (A + A.T), 0.5 * (G + G.T))
        X = X @ Q
    return lam, X


def largest_eigenvalue(K, M, tol: float = 1e-6) -> float:
    """Largest eigenvalue of the pencil (K, M) (Lanczos on M^-1 K).  With the unit
    roundoff u it bounds what FP64 vectors can attain: a vector whose entries carry
    relative errors of order u has a relative residual of up to u lambda_max / lambda_i."""
    return float(spla.eigsh(K.tocsc(), k=1, M=M.tocsc(), which="LA", return_eigenvectors=False, tol=tol)[0])


def subspace_gap_b(X1: np.ndarray, X2: np.ndarray, M) -> float:
    """theta_b(span X1, span X2) of Definition 2.1 for equal dimensions.

    With both blocks M-orthonormalised, sin{W1;W2} is the largest M-norm of
    the component of a unit vector of W1 that is M-orthogonal to W2.
    """
    def orth(X):
        G = X.T @ (M @ X)
        Lc = np.linalg.cholesky(0.5 * (G + G.T))
        return np.linalg.solve(Lc, X.T).T
    A, B = orth(X1), orth(X2)
    E = A - B @ (B.T @ (M @ A))          # components of W1's basis orthogonal to W2
    G = E.T @ (M @ E)
    return float(np.sqrt(max(0.0, np.linalg.eigvalsh(0.5 * (G + G.T))[-1])))

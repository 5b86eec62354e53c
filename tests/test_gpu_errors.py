"""Failure handling through the C ABI: malformed inputs are rejected with the documented
error code before any kernel runs, a failed coarse factorisation is reported as
BPJD_ERR_NOT_SPD, the iteration cap returns BPJD_ERR_NOCONV with the last iterate, and
calls out of order return BPJD_ERR_STATE.  Every case either stops on the host or runs
kernels whose loops are bounded whatever the values."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import bpjd_oracle as o
from paper_2203_06327_amd import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_06327_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def t16():
    return w.config_mesh("t16")


def _case(msg):
    print(f"\n[gpu case] {msg}", flush=True)


def _geom(mesh, cfg):
    return (mesh.coords, mesh.cx, mesh.cy, cfg["L"])


def _expect(B, code, fn):
    with pytest.raises(B.BPJDError) as e:
        fn()
    assert e.value.code == code, str(e.value)
    return str(e.value)


def test_malformed_csr(B, ctx, t16):
    mesh, cfg = t16
    K = sp.csr_matrix(mesh.K)
    _case("CSR: column index out of range")
    bad = K.copy()
    bad.indices = bad.indices.copy()
    bad.indices[5] = K.shape[0] + 3
    _expect(B, B.ERR_CSR, lambda: B.Problem(ctx, bad, mesh.M, geom=_geom(mesh, cfg), k=cfg["k"]))
    _case("CSR: row pointers not monotone")
    bad = K.copy()
    bad.indptr = bad.indptr.copy()
    bad.indptr[4], bad.indptr[5] = bad.indptr[5], bad.indptr[4]
    _expect(B, B.ERR_CSR, lambda: B.Problem(ctx, bad, mesh.M, geom=_geom(mesh, cfg), k=cfg["k"]))
    _case("CSR: non-finite value")
    bad = K.copy()
    bad.data = bad.data.copy()
    bad.data[7] = np.nan
    _expect(B, B.ERR_CSR, lambda: B.Problem(ctx, bad, mesh.M, geom=_geom(mesh, cfg), k=cfg["k"]))
    _case("CSR: K and M of different sizes")
    small = sp.identity(K.shape[0] - 1, format="csr")
    _expect(B, B.ERR_CSR, lambda: B.Problem(ctx, K, small, geom=_geom(mesh, cfg), k=cfg["k"]))


def test_invalid_decomposition_and_options(B, ctx, t16):
    mesh, cfg = t16
    dd = o.build_dd(mesh, cfg["L"])
    _case("DD: a dof in no subdomain")
    dropped = mesh.K.shape[0] // 2
    subs = [np.asarray([d for d in S if d != dropped]) for S in dd.subs]
    msg = _expect(B, B.ERR_DD, lambda: B.Problem(ctx, mesh.K, mesh.M, dd=(dd.P, subs), k=cfg["k"]))
    assert str(dropped) in msg
    _case("DD: subdomain index out of range")
    subs = [np.asarray(S) for S in dd.subs]
    subs[0] = np.append(subs[0], mesh.K.shape[0] + 1)
    _expect(B, B.ERR_DD, lambda: B.Problem(ctx, mesh.K, mesh.M, dd=(dd.P, subs), k=cfg["k"]))
    _case("DD: block size not below dim V^H")
    _expect(B, B.ERR_DD, lambda: B.Problem(ctx, mesh.K, mesh.M, dd=(dd.P, dd.subs), k=dd.P.shape[1]))
    _case("options: k + guard above the largest block, bad tolerance, unknown precision")
    _expect(B, B.ERR_ARG, lambda: B.Problem(ctx, mesh.K, mesh.M, dd=(dd.P, dd.subs), k=4, guard=17))
    _expect(B, B.ERR_ARG, lambda: B.Problem(ctx, mesh.K, mesh.M, dd=(dd.P, dd.subs), k=2, tol=0.0))
    _expect(B, B.ERR_ARG, lambda: B.Problem(ctx, mesh.K, mesh.M, dd=(dd.P, dd.subs), k=2, precision=7))
    _expect(B, B.ERR_ARG, lambda: B.Problem(ctx, mesh.K, mesh.M, dd=(dd.P, dd.subs), k=2, spmm_form=4))


def test_state_and_breakdown(B, ctx, t16):
    mesh, cfg = t16
    _case("state: preconditioner and coarse eigenvalues before setup")
    prob = B.problem_from_mesh(ctx, mesh, cfg["L"], k=cfg["k"], precision=B.PREC_FP64)
    X = np.ones((mesh.K.shape[0], prob.s))
    _expect(B, B.ERR_STATE, lambda: prob.apply_preconditioner(X, np.zeros(prob.s)))
    _expect(B, B.ERR_STATE, lambda: prob.coarse_eigenvalues())
    prob.close()
    _case("breakdown: M negative definite, the coarse Cholesky fails")
    Mneg = -sp.csr_matrix(mesh.M)
    bad = B.Problem(ctx, mesh.K, Mneg, geom=_geom(mesh, cfg), k=cfg["k"], precision=B.PREC_FP64)
    _expect(B, B.ERR_NOT_SPD, bad.setup)
    bad.close()


def test_iteration_cap(B, ctx):
    mesh, cfg = w.config_mesh("t64")
    _case("iteration cap: max_iter = 2 on t64")
    prob = B.problem_from_mesh(ctx, mesh, cfg["L"], k=cfg["k"], max_iter=2, precision=B.PREC_FP64)
    _expect(B, B.ERR_NOCONV, prob.solve)
    lam, X, st = prob.solve(raise_noconv=False)
    assert st["iterations"] == 2
    assert np.all(np.isfinite(lam)) and np.all(np.isfinite(X))
    ref = o.reference_eigs(mesh.K, mesh.M, cfg["k"])[0]
    # the last iterate is an upper bound of each eigenvalue (Rayleigh-Ritz, conforming space)
    assert np.all(lam >= ref * (1 - 1e-12))
    prob.close()

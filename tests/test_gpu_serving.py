"""The eigensolver server (continuous batching) through the C ABI.

A mix of served requests (rectangles [0,1] x [0,r], piecewise-constant
coefficients on a 4 x 4 block grid, different mesh sizes and k) is solved once
request by request with bpjd_solve and once through a server whose HBM budget
and slot count make requests wait for admission while others run.  Each served
result must equal the result of the same request alone, and both must match
the FP64 oracle's reference eigenpairs.
"""
import time

import numpy as np
import pytest

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


def _case(msg):
    print(f"\n[gpu case] {msg}", flush=True)


def _wait_all(srv, ids, timeout_s=120.0):
    out = {}
    t0 = time.perf_counter()
    while len(out) < len(ids):
        for i in ids:
            if i in out:
                continue
            r = srv.poll(i)
            if r is not None:
                out[i] = r
        if time.perf_counter() - t0 > timeout_s:
            raise TimeoutError(f"{len(ids) - len(out)} requests still pending")
        time.sleep(0.001)
    return out


def _host_residuals(mesh, lam, X):
    KX = mesh.K @ X
    MX = mesh.M @ X
    return np.linalg.norm(KX - MX * lam, axis=0) / (np.abs(lam) * np.linalg.norm(MX, axis=0))


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_served_equals_alone(B, ctx, prec):
    precision = B.PREC_MIXED if prec == "mixed" else B.PREC_FP64
    reqs = w.serving_requests(count=8, h_choices=(64, 128))
    meshes = [w.request_mesh(r) for r in reqs]
    alone, fp = [], []
    for r, mesh in zip(reqs, meshes):
        _case(f"serving alone {prec} request {r['j']} n={mesh.n} k={r['k']}")
        prob = B.problem_from_mesh(ctx, mesh, r["L"], k=r["k"], guard=r["guard"], precision=precision)
        fp.append(prob.footprint())
        alone.append(prob.solve())
        prob.close()
    # room for the two largest requests at once: the others wait for memory, not only slots
    budget = sorted(fp)[-1] + sorted(fp)[-2]
    _case(f"serving mix {prec}: {len(reqs)} requests, budget {budget} B, 4 slots")
    srv = B.Server(ctx, hbm_budget_bytes=budget, max_slots=4)
    ids = [srv.submit_mesh(mesh, r["L"], k=r["k"], guard=r["guard"], precision=precision)
           for r, mesh in zip(reqs, meshes)]
    res = _wait_all(srv, ids)
    info = srv.info()
    srv.close()
    assert info["completed"] == len(reqs) and info["failed"] == 0
    assert info["peak_bytes"] <= budget
    assert info["peak_running"] >= 2          # solves overlapped
    for r, mesh, rid, (lam_a, X_a, st_a) in zip(reqs, meshes, ids, alone):
        lam_s, X_s, st_s = res[rid]
        # the same request gives the same result alone and in the mix
        np.testing.assert_allclose(lam_s, lam_a, rtol=1e-12, atol=0)
        assert np.abs(X_s - X_a).max() <= 1e-10 * np.abs(X_a).max()
        assert st_s["iterations"] == st_a["iterations"]
        assert st_s["latency_ms"] >= st_s["queue_ms"] >= 0.0
        # served solves replay their captured iteration graphs like solves alone
        assert st_s["graph_iterations"] >= st_s["iterations"] - 3 > 0, st_s
        # and both are the pencil's eigenpairs
        lam_ref, _ = o.reference_eigs(mesh.K, mesh.M, r["k"])
        np.testing.assert_allclose(lam_s, lam_ref, rtol=1e-10 if prec == "fp64" else 1e-9)
        assert _host_residuals(mesh, lam_s, X_s).max() <= 1.5e-8
        G = X_s.T @ (mesh.M @ X_s)
        assert np.abs(G - np.eye(r["k"])).max() <= 1e-10


def test_server_errors_are_per_request(B, ctx):
    _case("serving errors")
    mesh, cfg = w.config_mesh("t16")
    srv = B.Server(ctx, hbm_budget_bytes=0, max_slots=2)
    good = srv.submit_mesh(mesh, cfg["L"], k=cfg["k"])
    # a column index out of range: found when the request is planned, reported by poll
    Kbad = mesh.K.copy()
    Kbad.indices = Kbad.indices.copy()
    Kbad.indices[3] = mesh.n + 5
    bad = srv.submit(Kbad, mesh.M, geom=(mesh.coords, mesh.cx, mesh.cy, cfg["L"]), k=cfg["k"])
    # s >= dim V^H
    too_big_k = srv.submit_mesh(mesh, cfg["L"], k=9)
    after = srv.submit_mesh(mesh, cfg["L"], k=cfg["k"], precision=B.PREC_FP64)
    with pytest.raises(B.BPJDError) as e:
        _wait_all(srv, [bad])
    assert e.value.code == B.ERR_CSR
    with pytest.raises(B.BPJDError) as e:
        _wait_all(srv, [too_big_k])
    assert e.value.code == B.ERR_DD
    res = _wait_all(srv, [good, after])
    lam_ref, _ = o.reference_eigs(mesh.K, mesh.M, cfg["k"])
    for rid in (good, after):
        np.testing.assert_allclose(res[rid][0], lam_ref, rtol=1e-9)
    with pytest.raises(B.BPJDError) as e:
        srv.poll(good)                        # released after its final poll
    assert e.value.code == B.ERR_ARG
    info = srv.info()
    assert info["completed"] == 4 and info["failed"] == 2
    srv.close()
    # a budget no request fits
    tiny = B.Server(ctx, hbm_budget_bytes=1 << 16, max_slots=2)
    rid = tiny.submit_mesh(mesh, cfg["L"], k=cfg["k"])
    with pytest.raises(B.BPJDError) as e:
        _wait_all(tiny, [rid])
    assert e.value.code == B.ERR_OVER_BUDGET
    tiny.close()


def test_served_wide_band_request_equals_alone(B, ctx):
    """A served h = 1/512 request (local half-bandwidth 68: the 96-row blocked window)
    next to small ones: the same result alone and in the mix, residuals recomputed on
    the host, M-orthonormal eigenvectors."""
    reqs = w.serving_requests(count=8)
    big = next(r for r in reqs if r["Nx"] == 512)
    small = [r for r in reqs if r["Nx"] == 64][:3]
    mix = [big] + small
    meshes = [w.request_mesh(r) for r in mix]
    alone = []
    for r, mesh in zip(mix, meshes):
        _case(f"serving alone request {r['j']} n={mesh.n} k={r['k']}")
        prob = B.problem_from_mesh(ctx, mesh, r["L"], k=r["k"], guard=r["guard"])
        alone.append(prob.solve())
        prob.close()
    _case("serving mix with a wide-band request")
    srv = B.Server(ctx, hbm_budget_bytes=0, max_slots=4)
    ids = [srv.submit_mesh(mesh, r["L"], k=r["k"], guard=r["guard"]) for r, mesh in zip(mix, meshes)]
    res = _wait_all(srv, ids)
    info = srv.info()
    srv.close()
    assert info["completed"] == len(mix) and info["failed"] == 0
    for r, mesh, rid, (lam_a, X_a, st_a) in zip(mix, meshes, ids, alone):
        lam_s, X_s, st_s = res[rid]
        np.testing.assert_allclose(lam_s, lam_a, rtol=1e-12, atol=0)
        assert np.abs(X_s - X_a).max() <= 1e-10 * np.abs(X_a).max()
        assert st_s["converged"] and st_s["iterations"] == st_a["iterations"]
        assert _host_residuals(mesh, lam_s, X_s).max() <= 1.5e-8
        np.testing.assert_allclose(X_s.T @ (mesh.M @ X_s), np.eye(r["k"]), atol=1e-10)

"""The boundary's resource and error contracts on the GPU (through the C ABI):

* every device byte comes from the context's allocator (here PyTorch's caching
  allocator): the blocks a problem holds add up to its footprint, a solve
  allocates nothing, destroying the problem hands every block back, and the
  results equal those of a hipMalloc context bit for bit;
* a server takes its whole budget as one block from that allocator when it is
  created, and admits and reaps requests without further allocation calls;
* the last error is kept per context.
"""
import threading

import numpy as np
import pytest

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


def _case(msg):
    print(f"\n[gpu case] {msg}", flush=True)


def _rounded(nbytes):
    return (max(nbytes, 8) + 4095) // 4096 * 4096


@pytest.mark.parametrize("name,prec", [("c1", "mixed"), ("t64", "fp64")])
def test_caller_allocator_sees_every_device_byte(B, name, prec):
    _case(f"caller allocator {name} {prec}")
    mesh, cfg = w.config_mesh(name)
    s = cfg["k"] + cfg["guard"]
    X0 = None if cfg["seed_block"] is None else w.seeded_block(mesh.n, s, cfg["seed_block"])
    kw = dict(k=cfg["k"], guard=cfg["guard"], X_init=X0,
              precision=B.PREC_FP64 if prec == "fp64" else B.PREC_MIXED)
    plain = B.Context(0)
    ref = B.problem_from_mesh(plain, mesh, cfg["L"], **kw)
    lam0, X0r, st0 = ref.solve()
    ref.close()
    plain.close()

    ctx = B.Context(0, allocator="torch")
    A = ctx.allocator
    prob = B.problem_from_mesh(ctx, mesh, cfg["L"], **kw)
    n_blocks, held = A.allocs, A.live_bytes
    assert n_blocks > 0 and A.frees == 0
    assert sum(_rounded(b) for b in A.live.values()) == prob.footprint()
    for _ in range(2):
        lam, X, st = prob.solve()
        assert A.allocs == n_blocks and A.live_bytes == held          # a solve allocates nothing
        assert st["iterations"] == st0["iterations"]
        assert np.array_equal(lam, lam0) and np.array_equal(X, X0r)
    prob.close()
    assert A.live_bytes == 0 and A.frees == n_blocks
    ctx.close()


def test_server_block_from_caller_allocator(B):
    _case("server block from the caller's allocator")
    ctx = B.Context(0, allocator="torch")
    A = ctx.allocator
    reqs = w.serving_requests(count=4, h_choices=(64,))
    meshes = [w.request_mesh(r) for r in reqs]
    alone = []
    for r, mesh in zip(reqs, meshes):
        p = B.problem_from_mesh(ctx, mesh, r["L"], k=r["k"], guard=r["guard"])
        alone.append(p.solve())
        p.close()
    assert A.live_bytes == 0
    budget = 256 << 20
    srv = B.Server(ctx, hbm_budget_bytes=budget, max_slots=3)
    assert A.live_bytes == budget                  # the whole budget, taken once
    n_allocs = A.allocs
    ids = [srv.submit_mesh(mesh, r["L"], k=r["k"], guard=r["guard"]) for r, mesh in zip(reqs, meshes)]
    out = {}
    while len(out) < len(ids):
        for i in ids:
            if i not in out:
                res = srv.poll(i)
                if res is not None:
                    out[i] = res
    assert A.allocs == n_allocs                    # admission and reaping allocate nothing
    for i, (lam, X, st) in zip(ids, alone):
        np.testing.assert_allclose(out[i][0], lam, rtol=1e-12)
        np.testing.assert_allclose(np.abs(out[i][1]), np.abs(X), atol=1e-10)
    info = srv.info()
    assert info["peak_bytes"] <= budget
    srv.close()
    assert A.live_bytes == 0
    ctx.close()


def test_last_error_is_per_context(B):
    _case("last error per context")
    mesh, cfg = w.config_mesh("t16")
    a, b = B.Context(0), B.Context(0)
    with pytest.raises(B.BPJDError):
        B.problem_from_mesh(a, mesh, cfg["L"], k=2, tol=0.0)
    assert "tol" in a.last_error()
    assert b.last_error() == ""
    # a failure on b from another thread is b's, and leaves a's message alone
    err = []

    def bad():
        try:
            B.problem_from_mesh(b, mesh, cfg["L"], k=2, precision=9)
        except B.BPJDError as e:
            err.append(e)
    t = threading.Thread(target=bad)
    t.start()
    t.join()
    assert err and "precision" in b.last_error()
    assert "tol" in a.last_error()
    a.close()
    b.close()

"""The allocation-free coarse eigenproblem (bpjd_coarse_eigen_noalloc) through the
C ABI against the existing entry points that compute the same thing with the
library's own workspace (bpjd_setup, then bpjd_coarse_eigenvalues): two calls in
a row on one context, the second with a smaller coarse space, each checked to the
FP64 tolerance; the eigenvectors satisfy K_H Y = M_H Y Lambda and Y^T M_H Y = I."""
import numpy as np
import pytest

from oracle import bpjd_oracle as o
from paper_2203_06327_amd import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_06327_amd import binding
    binding.lib()
    stream = torch.cuda.Stream()
    ctx = binding.Context(0, stream=stream.cuda_stream)
    yield torch, binding, ctx, stream
    ctx.close()


def _coarse_matrices(name):
    mesh, cfg = w.config_mesh(name)
    P = o.coarse_prolongation(mesh.coords, mesh.cx, mesh.cy)
    KH = (P.T @ (mesh.K @ P)).toarray()
    MH = (P.T @ (mesh.M @ P)).toarray()
    KH, MH = 0.5 * (KH + KH.T), 0.5 * (MH + MH.T)
    rows, cols = np.nonzero(MH)
    return mesh, cfg, KH, MH, int(np.max(np.abs(rows - cols)))


def _existing(B, ctx, mesh, cfg):
    prob = B.problem_from_mesh(ctx, mesh, cfg["L"], k=cfg["k"], guard=cfg["guard"], precision=B.PREC_FP64)
    prob.setup()
    lam = prob.coarse_eigenvalues()
    prob.close()
    return lam


def test_noalloc_matches_setup_on_two_sizes(env):
    torch, B, ctx, stream = env
    for name in ("c2", "c1"):                  # n_H = 225, then 9
        print(f"\n[gpu case] coarse eigen noalloc {name}", flush=True)
        mesh, cfg, KH, MH, bw = _coarse_matrices(name)
        n = KH.shape[0]
        dev = torch.device("cuda", 0)
        with torch.cuda.stream(stream):
            Kd = torch.from_numpy(KH).to(dev)
            Md = torch.from_numpy(MH).to(dev)
            lam_d = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
            Y_d = torch.full((n, n), float("nan"), dtype=torch.float64, device=dev)
            info = torch.full((1,), -1, dtype=torch.int32, device=dev)
        stream.synchronize()
        B.coarse_eigen_noalloc(ctx, Kd, Md, bw, lam_d, Y_d, info)
        stream.synchronize()
        assert int(info.cpu()[0]) == 0
        lam = lam_d.cpu().numpy()
        Y = Y_d.cpu().numpy()
        ref = _existing(B, ctx, mesh, cfg)
        err = np.max(np.abs(lam - ref) / np.abs(ref))
        print(f"  n_H={n} bw={bw} max rel diff to bpjd_setup's {err:.3e}", flush=True)
        assert err < 1e-11
        np.testing.assert_allclose(Y.T @ MH @ Y, np.eye(n), atol=1e-10)
        R = KH @ Y - (MH @ Y) * lam[None, :]
        assert np.abs(R).max() <= 1e-10 * np.abs(KH).max() * max(1.0, np.abs(Y).max())


def test_noalloc_rejects_sizes_beyond_its_scratch(env):
    torch, B, ctx, stream = env
    dev = torch.device("cuda", 0)
    n = 321
    A = torch.eye(n, dtype=torch.float64, device=dev)
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Y = torch.empty((n, n), dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    with pytest.raises(B.BPJDError) as e:
        B.coarse_eigen_noalloc(ctx, A, A, 0, lam, Y, info)
    assert e.value.code == B.ERR_ARG and "320" in str(e.value)
    assert "320" in ctx.last_error()

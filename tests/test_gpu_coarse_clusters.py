"""Clustered eigenvalues in the dense symmetric eigensolver of the coarse problem
(Section 3, eq. EigenvalueCoarse), through the allocation-free entry point with
caller-given matrices: K_H = Q diag(lambda) Q^T with a known spectrum (a closed form
by construction) and M_H = I.  The spectrum holds a run of 24 eigenvalues closer than
the solver's cluster gap (orthonormalised and rotated in memory, chunks wider than 16),
a run of 12 and an exactly threefold eigenvalue (held in LDS), and isolated values.
Eigenvalues must match the constructed ones; eigenvectors must be orthonormal with a
small residual (inside a cluster the vectors are not unique, so they are not compared
one by one)."""
import numpy as np
import pytest

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


def _spectrum(n):
    runs = [100.0 + 0.5 * np.arange(24), 400.0 + 0.3 * np.arange(12), np.full(3, 700.0)]
    members = np.concatenate(runs)
    iso = [x for x in np.arange(1.0, 2000.0, 4.0) if np.min(np.abs(members - x)) > 3.0]
    lam = np.sort(np.concatenate([members, np.array(iso[: n - members.size])]))
    assert lam.size == n
    return lam, runs


def test_coarse_eigensolver_clusters(env):
    torch, B, ctx, stream = env
    n = 200
    lam_ref, runs = _spectrum(n)
    tn = np.max(np.abs(lam_ref))
    gap = 1e-3 * tn                     # the solver groups consecutive gaps below this
    cut = np.nonzero(np.diff(lam_ref) > gap)[0] + 1
    sizes = sorted((len(r) for r in np.split(lam_ref, cut) if len(r) > 1), reverse=True)
    assert sizes == [24, 12, 3]         # one chunk wider than 16 columns, two within
    rng = np.random.default_rng(61)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    K = (Q * lam_ref[None, :]) @ Q.T
    K = 0.5 * (K + K.T)
    M = np.eye(n)
    print(f"\n[gpu case] coarse eigensolver clusters n={n} runs 24/12/3 gap {gap:.3f}", flush=True)
    dev = torch.device("cuda", 0)
    with torch.cuda.stream(stream):
        Kd = torch.from_numpy(K).to(dev)
        Md = torch.from_numpy(M).to(dev)
        lam_d = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
        Y_d = torch.full((n, n), float("nan"), dtype=torch.float64, device=dev)
        info = torch.full((1,), -1, dtype=torch.int32, device=dev)
    stream.synchronize()
    B.coarse_eigen_noalloc(ctx, Kd, Md, 0, lam_d, Y_d, info)
    stream.synchronize()
    assert int(info.cpu()[0]) == 0
    lam = lam_d.cpu().numpy()
    Y = Y_d.cpu().numpy()
    err = np.max(np.abs(lam - lam_ref))
    print(f"  max |lambda - constructed| {err:.3e} (|T| {tn:.1f})", flush=True)
    assert err <= 1e-12 * tn
    orth = np.abs(Y.T @ Y - np.eye(n)).max()
    res = np.abs(K @ Y - Y * lam[None, :]).max()
    print(f"  |Y^T Y - I| {orth:.3e}, |K Y - Y Lambda| {res:.3e}", flush=True)
    assert orth <= 1e-12
    assert res <= 1e-12 * tn
    # each run's eigenvectors span the constructed invariant subspace
    for run in runs:
        idx = np.nonzero(np.isin(lam_ref, run))[0]
        Qr = Q[:, idx]
        Yr = Y[:, idx]
        proj = Yr - Qr @ (Qr.T @ Yr)
        assert np.abs(proj).max() <= 1e-9, (run[0], np.abs(proj).max())

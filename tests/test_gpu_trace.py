"""The JSON-lines trace (environment variable BPJD_TRACE): planning stages, one record
per residual read-back, and a solve summary that agree with the returned statistics."""
import json

import numpy as np
import pytest

from paper_2203_06327_amd import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2203_06327_amd import binding
    binding.lib()
    return binding


def test_trace_records_planning_iterations_and_solve(B, tmp_path, monkeypatch):
    print("\n[gpu case] trace c1 mixed", flush=True)
    path = tmp_path / "trace.jsonl"
    ctx = B.Context(0)
    mesh, cfg = w.config_mesh("c1")
    monkeypatch.setenv("BPJD_TRACE", str(path))
    prob = B.problem_from_mesh(ctx, mesh, cfg["L"], k=cfg["k"], guard=cfg["guard"], precision=B.PREC_MIXED)
    monkeypatch.delenv("BPJD_TRACE")
    lam, X, st = prob.solve()
    prob.close()
    ctx.close()
    recs = [json.loads(line) for line in path.read_text().splitlines() if line.strip()]
    stages = [r["stage"] for r in recs if r["event"] == "create"]
    assert stages[:2] == ["read_csr", "union_pattern"] and "allocate_upload" in stages
    assert all(r["ms"] >= 0 for r in recs if r["event"] == "create")
    its = [r for r in recs if r["event"] == "iteration"]
    assert sorted({r["it"] for r in its}) == list(range(st["iterations"] + 1))
    last = its[-1]
    assert last["it"] == st["iterations"] and last["rho_max"] == pytest.approx(st["max_residual"], rel=1e-6)
    assert np.allclose(last["lambda"][: cfg["k"]], lam, rtol=1e-14)
    rr = [r for r in recs if r["event"] == "rayleigh_ritz"]
    assert len(rr) == st["iterations"] and all(len(r["theta"]) == r["m"] for r in rr)
    solve = [r for r in recs if r["event"] == "solve"]
    assert len(solve) == 1 and solve[0]["iterations"] == st["iterations"] and solve[0]["converged"]

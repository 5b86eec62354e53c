#!/usr/bin/env python
"""Throughput of the two-level BPJD eigensolver on one MI355X.

One step = one complete solve of the workload (device numeric setup:
Galerkin coarse operators, coarse eigenproblem, start block; then outer
iterations of Algorithm 3.1 until every wanted pair has relative residual
<= 1e-8), with K, M and the decomposition already resident in HBM.  The
default workload is the 261,121-dof Laplacian (unit square, P1, h = 1/512,
16 x 16 subdomains, overlap 4h, first 8 eigenpairs) solved with FP32 local
solves (mixed precision); the plain FP64 solve of the same problem is timed
beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "eigenpairs/sec at residual 1e-8 (batched mixed vs plain FP64); p50/p99 latency"
PEAK = {"hbm_GBs": 8000.0, "fp32_TFs": 157.3, "fp64_TFs": 78.6}


def local_solve_flops(nl: np.ndarray, bw: np.ndarray, s: int) -> float:
    """Algorithmic flops of one batched local LDL^T factor + solve launch.

    Per (subdomain, shift): at step j the a_j = min(w, n_l - 1 - j) rows below the
    pivot take a_j(a_j+1)/2 window updates (one FMA = 2 flops each) and a_j
    multiplier scalings; forward and backward substitution cost 2 a_j flops each,
    plus one division per row.
    """
    total = 0.0
    for n, w in zip(nl.tolist(), bw.tolist()):
        j = np.arange(n)
        a = np.minimum(w, n - 1 - j).astype(np.float64)
        total += float(np.sum(a * (a + 1) + a + 4 * a + 2))
    return total * s


def spmm_bytes(n: int, nnz: int, ncols: int) -> float:
    """Algorithmic HBM bytes of one fused [K;M] X launch: row pointers, column
    indices, (K, M) value pairs, the X block once, KX and MX written once."""
    return 4.0 * (n + 1) + 4.0 * nnz + 16.0 * nnz + 8.0 * n * ncols + 16.0 * n * ncols


def time_solves(prob, steps: int, warmup: int, torch, k: int, n: int):
    lam_d = torch.empty(k, dtype=torch.float64, device="cuda")
    X_d = torch.empty((n, k), dtype=torch.float64, device="cuda")
    from paper_2203_06327_amd import binding as B
    for _ in range(warmup):
        prob.solve(lam_d, X_d, mem=B.MEM_DEVICE)
    torch.cuda.synchronize()
    lat, stats = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        _, _, st = prob.solve(lam_d, X_d, mem=B.MEM_DEVICE)
        lat.append(time.perf_counter() - ts)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, np.array(lat), stats, lam_d.cpu().numpy(), X_d


def cpu_baseline(mesh, cfg, gpu_iters: int, sample_iters: int):
    """The FP64 oracle on the host cores: structural + coarse + local setup and
    `sample_iters` outer iterations, extrapolated to a full solve with the
    iteration count of the same algorithm (the GPU FP64 run's count)."""
    from oracle import bpjd_oracle as o
    t0 = time.perf_counter()
    dd = o.build_dd(mesh, cfg["L"])
    cs = o.coarse_setup(mesh.K, mesh.M, dd.P)
    ls = o.local_setup(mesh.K, mesh.M, dd.subs)
    t1 = time.perf_counter()
    o.bpjd(mesh.K, mesh.M, dd, cfg["k"], cfg["guard"], tol=1e-8, max_iter=sample_iters, setups=(cs, ls))
    t2 = time.perf_counter()
    t_setup = t1 - t0
    t_iter = (t2 - t1) / max(1, sample_iters)
    est = t_setup + gpu_iters * t_iter
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": cfg["k"] / est, "unit": "eigenpairs/s", "cores": threads, "kind": "oracle",
        "sample": (f"setup + {sample_iters} outer iterations of the FP64 oracle on the same workload "
                   f"({t_setup:.1f} s setup, {t_iter:.1f} s/iteration), extrapolated to {gpu_iters} iterations "
                   f"= {est:.1f} s per solve"),
    }


COUNTERS = os.path.join(ROOT, "profiles", "local_band_mfma_c2_counters.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2203_06327_amd", "csrc", "precond.hip")


def source_hash(path: str) -> str:
    import hashlib
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def counter_traffic(config: str):
    """HBM bytes per launch of the local solve kernel from the committed counter
    summary: FETCH_SIZE + WRITE_SIZE per dispatch, each scaled by the factor a plain
    copy kernel of known size gives for the same counter.  None when the summary is
    missing, covers another workload, or was taken on another version of the kernel
    source."""
    if not os.path.exists(COUNTERS):
        return None
    vals = {}
    with open(COUNTERS) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                key, val = line.split("=", 1)
                vals[key.strip()] = val.strip()
    try:
        if vals.get("workload") != config or vals.get("kernel_source_sha256") != source_hash(KERNEL_SRC):
            return None
        fetch = float(vals["fetch_kib_per_dispatch"]) * 1024.0 * float(vals["copy_fetch_factor"])
        write = float(vals["write_kib_per_dispatch"]) * 1024.0 * float(vals["copy_write_factor"])
    except (KeyError, ValueError):
        return None
    return fetch + write


def copy_calibration(torch):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE
    counters: 512 MiB read and 512 MiB written per launch, three launches."""
    nbytes = 512 << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-breakdown", action="store_true", help="skip the untimed per-phase profile solve")
    ap.add_argument("--cpu-sample-iters", type=int, default=2)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain copy of known size (for scaling memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: multi-GPU runs are not part of this build (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    from paper_2203_06327_amd import binding as B
    from paper_2203_06327_amd import workloads as w

    mesh, cfg = w.config_mesh(args.config)
    k, s = cfg["k"], cfg["k"] + cfg["guard"]
    print(f"[bench] {args.config}: n={mesh.n} nnz={mesh.K.nnz} k={k}", file=sys.stderr, flush=True)
    ctx = B.Context(0)
    # timed solves: only the local-solve phase carries HIP events (two per iteration)
    prob = B.problem_from_mesh(ctx, mesh, cfg["L"], k=k, guard=cfg["guard"], tol=1e-8, precision=B.PREC_MIXED,
                               profile=2)
    secs, lat, stats, lam, X_d = time_solves(prob, args.steps, args.warmup, torch, k, mesh.n)
    print(f"[bench] mixed: {secs / args.steps * 1e3:.1f} ms/solve, iterations {stats[-1]['iterations']}",
          file=sys.stderr, flush=True)
    value = k * args.steps / secs
    st = stats[-1]
    i_local = B.PHASES.index("local")
    local_ms = sum(x["phase_ms"][i_local] for x in stats)
    local_n = sum(x["phase_count"][i_local] for x in stats)
    local_avg_ms = local_ms / max(1, local_n)

    # per-phase breakdown from one extra, untimed solve with every phase timed
    ph = cnt = None
    if not args.no_breakdown:
        probp = B.problem_from_mesh(ctx, mesh, cfg["L"], k=k, guard=cfg["guard"], tol=1e-8,
                                    precision=B.PREC_MIXED, profile=1)
        _, _, stp = probp.solve(torch.empty(k, dtype=torch.float64, device="cuda"),
                                torch.empty((mesh.n, k), dtype=torch.float64, device="cuda"), mem=B.MEM_DEVICE)
        torch.cuda.synchronize()
        ph = dict(zip(B.PHASES, stp["phase_ms"]))
        cnt = dict(zip(B.PHASES, stp["phase_count"]))
        probp.close()

    fp64 = None
    if not args.no_fp64:
        prob64 = B.problem_from_mesh(ctx, mesh, cfg["L"], k=k, guard=cfg["guard"], tol=1e-8,
                                     precision=B.PREC_FP64, profile=2)
        secs64, lat64, stats64, lam64, _ = time_solves(prob64, max(1, args.steps // 2), 1, torch, k, mesh.n)
        fp64 = {"value": k * len(lat64) / secs64, "ms_per_solve": 1e3 * secs64 / len(lat64),
                "iterations": stats64[-1]["iterations"], "max_residual": stats64[-1]["max_residual"],
                "local_avg_launch_ms": sum(x["phase_ms"][i_local] for x in stats64)
                / max(1, sum(x["phase_count"][i_local] for x in stats64))}
        print(f"[bench] fp64: {fp64['ms_per_solve']:.1f} ms/solve, iterations {fp64['iterations']}",
              file=sys.stderr, flush=True)
        gpu_iters = stats64[-1]["iterations"]
        prob64.close()
    else:
        gpu_iters = st["iterations"]

    # dominant kernel of the mixed solve (the batched local LDL^T factor + solve) and its
    # roofline: algorithmic flops per launch over the average launch time measured with
    # HIP events on the library's stream inside the timed solves
    nl, bw = prob.local_sizes()
    local_flops = local_solve_flops(nl, bw, s)
    roofline = {"bound": "alu", "achieved": local_flops / (local_avg_ms * 1e-3) / 1e12,
                "peak": PEAK["fp32_TFs"], "unit": "TFLOP/s", "traffic": None,
                "kernel": "local_band_mfma_kernel<float>", "avg_launch_ms": local_avg_ms,
                "launches_timed": local_n, "algorithmic_per_launch": local_flops}
    roofline["frac"] = roofline["achieved"] / roofline["peak"]
    roofline["traffic"] = counter_traffic(args.config)
    roof_spmm = None
    if ph is not None:
        spmm_avg_ms = ph["spmm"] / max(1, cnt["spmm"])
        sb = spmm_bytes(mesh.n, mesh.K.nnz, s)
        roof_spmm = {"bound": "hbm", "achieved": sb / (spmm_avg_ms * 1e-3) / 1e9, "peak": PEAK["hbm_GBs"],
                     "unit": "GB/s", "kernel": "spmm_km_kernel", "avg_launch_ms": spmm_avg_ms,
                     "algorithmic_per_launch": sb, "source": "untimed profiled solve"}
        roof_spmm["frac"] = roof_spmm["achieved"] / roof_spmm["peak"]

    # correctness of the returned pairs against the paper's printed values where they exist
    check = {}
    if args.config == "c2":
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from conftest import load_table1
        t1 = load_table1()[:k, 2]
        check["max_abs_err_vs_table1"] = float(np.max(np.abs(lam / np.pi ** 2 - t1)))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(mesh, cfg, gpu_iters, args.cpu_sample_iters)

    out = {
        "metric": METRIC, "value": value, "unit": "eigenpairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * secs / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"{args.config}: {cfg['desc']}", "n": mesh.n, "k": k, "s": s,
                   "n_sub": prob.n_sub, "n_coarse": prob.n_coarse, "precision": "mixed (FP32 local solves)",
                   "subspace": "UU", "stop": "max relative residual <= 1e-8"},
        "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "iterations": st["iterations"], "max_residual": st["max_residual"],
        "fp64": fp64, "phase_ms_per_solve": ph, "phase_launches": cnt,
        "roofline": roofline, "roofline_spmm": roof_spmm, "cpu_baseline": cpu, **check,
    }
    print(json.dumps(out), flush=True)
    prob.close()
    ctx.close()


if __name__ == "__main__":
    main()

#!/usr/bin/env python
"""Throughput of the two-level BPJD eigensolver on one MI355X.

One step = one complete solve of the workload: the whole hot path, i.e. the
device numeric setup (Galerkin coarse operators, coarse eigenproblem, start
block, local extraction) and the outer iterations of Algorithm 3.1 until every
wanted pair has relative residual <= 1e-8, with K, M and the decomposition
already resident in HBM.  The default workload is the largest configuration:
the 1,056,759-dof Laplacian on [0,1] x [0,1.01] (P1, h = 1/1024, 32 x 32
subdomains, overlap 4h, first 12 eigenpairs with one guard vector) solved with
FP32 local solves (mixed precision); beside it: the plain FP64 solve of the same
problem, the whole job from device-resident CSR (problem creation included) and
from host CSR to host eigenpairs, the per-phase roofline, the served mix of 256
requests and the FP64 oracle on the host.  Prints one JSON line.
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


def local_kernel_name(band: int, slots: int) -> str:
    """The FP32 local solver the library picks: the blocked MFMA solver with a 64-row
    window up to half-bandwidth 48 and a 96-row window up to 80 (at most 8 lower
    entries per local row), the wide blocked solver (192-row window) for bands 49..176
    with up to 20 lower entries, the windowed LDS solver otherwise."""
    if slots <= 8 and band <= 48:
        return "local_band_mfma_kernel<float, 0, 4>"
    if slots <= 8 and band <= 80:
        return "local_band_mfma_kernel<float, 0, 6>"
    if 49 <= band <= 176 and slots <= 20:
        return "local_band_wide_kernel<0>"
    return "local_ldlt_kernel<float>"


# kernel of each SpMM lane layout (bpjd_stats.spmm_form)
SPMM_KERNELS = {1: "spmm_km_pair_kernel", 2: "spmm_km_kernel", 3: "spmm_km_flat_kernel"}


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


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(mesh, cfg, gpu_iters: int, sample_subs: int = 64):
    """The FP64 oracle on the host cores, timed on a bounded sample of the same workload
    and scaled to one solve: its numeric setup (Galerkin coarse operators and the full
    coarse eigenproblem, plus the local matrices of `sample_subs` subdomains scaled to all
    of them) and one outer iteration (the global steps in full, the local solves of the
    sampled subdomains scaled to all), times the GPU run's iteration count.  The
    decomposition itself (coarse prolongation, subdomain sets) is host planning on both
    sides and is not timed.  cores = process CPU time / wall time over the sample."""
    from oracle import bpjd_oracle as o
    k, s = cfg["k"], cfg["k"] + cfg["guard"]
    if getattr(mesh, "P", None) is not None:          # plate: the oracle's own BFS spaces
        from oracle import bfs_space as bs
        Nc = cfg["N"] // cfg["coarse"]
        dd = o.DD(bs.coarse_space(cfg["N"], Nc, mesh.vert, mesh.kind), bs.local_spaces(cfg["N"], Nc, cfg["L"], mesh.vert))
    else:
        P = o.coarse_prolongation(mesh.coords, mesh.cx, mesh.cy)
        # the subdomains of the first sqrt(sample) x sqrt(sample) coarse cells
        q = int(np.sqrt(sample_subs))
        nx, ny = len(mesh.cx) - 1, len(mesh.cy) - 1
        cxs, cys = mesh.cx[:min(q, nx) + 1], mesh.cy[:min(q, ny) + 1]
        subs = o.subdomain_sets(mesh.coords, cxs, cys, mesh.K, mesh.M, cfg["L"], cfg.get("shape", "square"))
        dd = o.DD(P, subs)
    n_sub_all = cfg.get("n_sub_all") or len(dd.subs)
    sample = dd.subs[:sample_subs]
    scale = n_sub_all / len(sample)
    w0, c0 = time.perf_counter(), sum(os.times()[:2])
    cs = o.coarse_setup(mesh.K, mesh.M, dd.P)
    t1 = time.perf_counter()
    ls = o.local_setup(mesh.K, mesh.M, sample)
    t2 = time.perf_counter()
    # one outer iteration of the oracle's Algorithm 3.1 as it stands, with the local solves
    # of the sampled subdomains (the residual of the next iteration included)
    sub_dd = o.DD(dd.P, sample)
    o.bpjd(mesh.K, mesh.M, sub_dd, k, cfg["guard"], tol=1e-300, max_iter=1, setups=(cs, ls))
    t3 = time.perf_counter()
    # the local solves of that iteration alone, to scale them to every subdomain
    X = dd.P @ cs.Y[:, :s]
    lam = cs.lamH[:s].copy()
    F = (mesh.M @ X) * lam[None, :] - mesh.K @ X
    t4 = time.perf_counter()
    o.local_term(F, lam, ls)
    t5 = time.perf_counter()
    wall, cpu = time.perf_counter() - w0, sum(os.times()[:2]) - c0
    t_setup = (t1 - w0) + scale * (t2 - t1)
    t_local = t5 - t4
    t_iter = (t3 - t2) + (scale - 1.0) * t_local
    est = t_setup + gpu_iters * t_iter
    return {
        "value": k / est, "unit": "eigenpairs/s", "cores": max(1, int(round(cpu / wall))), "kind": "oracle",
        "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
        "sample": (f"FP64 oracle, {wall:.1f} s wall / {cpu:.1f} s CPU: numeric setup ({t1 - w0:.2f} s coarse, "
                   f"local matrices of {len(sample)} of {n_sub_all} subdomains {t2 - t1:.2f} s) and one outer "
                   f"iteration of its Algorithm 3.1 with the local solves of those subdomains ({t3 - t2:.2f} s, of "
                   f"which local solves {t_local:.2f} s for {len(sample)} subdomains x {s} shifts); scaled to "
                   f"all subdomains and {gpu_iters} iterations = {est:.1f} s per solve"),
    }


KERNEL_SRC = os.path.join(ROOT, "paper_2203_06327_amd", "csrc", "precond.hip")
KERNEL_REGION = ("// Local solves, blocked:", "// Local extraction (numeric setup)")


def counters_path(config: str) -> str:
    return os.path.join(ROOT, "profiles", f"local_band_mfma_{config}_counters.txt")


def source_hash(path: str) -> str:
    """First 16 hex digits of the sha256 of the blocked local solver's source: the text
    of precond.hip from the comment that opens the blocked solver (its helpers, tile
    traits and kernel) up to the next section."""
    import hashlib
    text = open(path, encoding="utf-8").read()
    a = text.index(KERNEL_REGION[0])
    b = text.index(KERNEL_REGION[1], a)
    return hashlib.sha256(text[a:b].encode("utf-8")).hexdigest()[:16]


def counter_traffic(config: str):
    """HBM bytes per launch of the local solve kernel from the committed counter
    summary: FETCH_SIZE + WRITE_SIZE per dispatch, each scaled by the factor a plain
    copy kernel of known size gives for the same counter.  None when the summary is
    missing, covers another workload, or was taken on another version of the kernel
    source."""
    path = counters_path(config)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
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


def phase_ideal(n: int, nnz: int, s: int, sum_nl: int, nnzP: int, nH: int, local_flops: float):
    """Algorithmic cost of one outer iteration per phase, in ms at the MI355X peaks (HBM
    8 TB/s; FP32 157.3 TFLOP/s for the local solves): the bytes each phase must move
    at least once (FP64 blocks, CSR arrays) or the local solver's flops.
      spmm: one fused [K; M] T launch;  residual: K X, M X read, F written (24 n s);
      coarse: F read, P^T (12 B per entry), Y and Y^T read (16 n_H^2);
      gather_scatter: F gathered (8 + 4 B per local entry and shift), z written and read
        back in FP32 (4 + 4 B), the index arrays, Z written (8 n s), P read;
      ortho: two CGS passes (Gram of [X P] (2s columns) with T, T -= [X P] C) and two
        CholQR passes (Gram of T with M T, T, K T, M T right-multiplied in place);
      rr: Gram of W with K W (3s + 3s columns), [X P], K[X P], M[X P] <- (W, K W, M W) C.
    """
    B = 8e12 / 1e3     # bytes per ms
    n8 = 8.0 * n
    ph = {
        "spmm": spmm_bytes(n, nnz, s) / B,
        "residual": 24.0 * n * s / B,
        "coarse": (n8 * s + 12.0 * nnzP + 16.0 * nH * nH) / B,
        "gather_scatter": ((8 + 4 + 4 + 4) * s * sum_nl + 8.0 * sum_nl + n8 * s + 12.0 * nnzP) / B,
        "ortho": (2 * n8 * (2 * s + s + 2 * s + s + s) + 2 * n8 * (2 * s + 6 * s)) / B,
        "rr": (n8 * 6 * s + n8 * (9 * s + 6 * s)) / B,
        "local": local_flops / (PEAK["fp32_TFs"] * 1e12) * 1e3,
    }
    return ph


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


def build_served_meshes(count: int, workers: int = 8):
    """Meshes of the served mix, assembled on the host by a pool of threads of this
    process (no child process is ever started, so a profiler's preloaded library
    never sees a fork)."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_2203_06327_amd import workloads as w
    reqs = w.serving_requests(count)
    with ThreadPoolExecutor(max_workers=workers) as pool:
        meshes = list(pool.map(w.request_mesh, reqs))
    return reqs, meshes


def _wait(srv, ids, done_at=None):
    out = {}
    pending = list(ids)
    while pending:
        left = []
        for i in pending:
            r = srv.poll(i, raise_noconv=False)
            if r is None:
                left.append(i)
            else:
                out[i] = r
                if done_at is not None:
                    done_at[i] = time.perf_counter()
        pending = left
        if pending:
            time.sleep(0.0005)
    return out


def serving_bench(B, ctx, reqs, meshes, budget: int, slots: int, rate_frac: float = 0.7, log_path=None):
    """The served mix three ways: plain FP64 solves one request at a time (host CSR in,
    eigenpairs in host memory), the mixed-precision server with every request
    submitted at once (saturated throughput mu), and the server under Poisson
    arrivals at rate_frac * mu (latency percentiles)."""
    ks = np.array([r["k"] for r in reqs])
    total_k = int(ks.sum())
    # (i) plain FP64, one request at a time
    t0 = time.perf_counter()
    plain = []
    log = open(log_path, "w") if log_path else None     # per-request times of this leg
    for j, (r, mesh) in enumerate(zip(reqs, meshes)):
        ts = time.perf_counter()
        prob = B.problem_from_mesh(ctx, mesh, r["L"], k=r["k"], guard=r["guard"], precision=B.PREC_FP64)
        tc = time.perf_counter()
        lam, _, st = prob.solve(raise_noconv=False)
        plain.append((lam, st))
        prob.close()
        if log:
            log.write(f"{j}\t{r['Nx']}\t{mesh.n}\t{r['k']}\t{st['iterations']}\t{st['converged']}\t"
                      f"{1e3 * (tc - ts):.1f}\t{1e3 * (time.perf_counter() - tc):.1f}\t{st['max_band']}\n")
            log.flush()
        if (j + 1) % 16 == 0:
            print(f"[bench] plain FP64: {j + 1} requests, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                  flush=True)
    t_plain = time.perf_counter() - t0
    print(f"[bench] served mix, plain FP64 one at a time: {t_plain:.2f} s", file=sys.stderr, flush=True)
    # (i') the same one at a time with FP32 local solves: separates the precision gain
    # from the batching gain
    t0 = time.perf_counter()
    for r, mesh in zip(reqs, meshes):
        prob = B.problem_from_mesh(ctx, mesh, r["L"], k=r["k"], guard=r["guard"], precision=B.PREC_MIXED)
        prob.solve(raise_noconv=False)
        prob.close()
    t_mixed1 = time.perf_counter() - t0
    print(f"[bench] served mix, mixed one at a time: {t_mixed1:.2f} s", file=sys.stderr, flush=True)

    # (ii) server, burst: all requests at t = 0
    srv = B.Server(ctx, hbm_budget_bytes=budget, max_slots=slots)
    t0 = time.perf_counter()
    ids = [srv.submit_mesh(mesh, r["L"], k=r["k"], guard=r["guard"], precision=B.PREC_MIXED)
           for r, mesh in zip(reqs, meshes)]
    res = _wait(srv, ids)
    t_burst = time.perf_counter() - t0
    info_burst = srv.info()
    srv.close()
    mu = len(reqs) / t_burst
    print(f"[bench] served mix, server burst: {t_burst:.2f} s", file=sys.stderr, flush=True)
    rel = max(float(np.max(np.abs(res[i][0] - p[0]) / np.abs(p[0]))) for i, p in zip(ids, plain))
    rmax = max(res[i][2]["max_residual"] for i in ids)
    unconverged = sum(1 for i in ids if not res[i][2]["converged"]) + sum(1 for p in plain if not p[1]["converged"])

    # (iii) server, Poisson arrivals at rate_frac * mu
    rate = rate_frac * mu
    gaps = np.random.default_rng(2203).exponential(1.0 / rate, size=len(reqs))
    arrive = np.cumsum(gaps) - gaps[0]
    srv = B.Server(ctx, hbm_budget_bytes=budget, max_slots=slots)
    t0 = time.perf_counter()
    ids2 = []
    done_at, out2 = {}, {}
    for j, (r, mesh) in enumerate(zip(reqs, meshes)):
        while time.perf_counter() - t0 < arrive[j]:
            ready = _poll_some(srv, ids2, out2, done_at)
            if not ready:
                time.sleep(0.0002)
        ids2.append(srv.submit_mesh(mesh, r["L"], k=r["k"], guard=r["guard"], precision=B.PREC_MIXED))
    out2.update(_wait(srv, [i for i in ids2 if i not in out2], done_at))
    t_poisson = time.perf_counter() - t0
    info_p = srv.info()
    srv.close()
    lat = np.array([out2[i][2]["latency_ms"] for i in ids2])
    qms = np.array([out2[i][2]["queue_ms"] for i in ids2])
    print(f"[bench] served mix, Poisson arrivals: {t_poisson:.2f} s", file=sys.stderr, flush=True)
    return {
        "workload": (f"{len(reqs)} requests: -div(a grad u) = lambda u on [0,1]x[0,r], r~U[1,2], a piecewise "
                     f"constant on 4x4 blocks, log-uniform in [0.1,10], P1, h in 1/64..1/512, k in 4..16 "
                     f"(guard 2), H=1/8, delta=2h"),
        "requests": len(reqs), "eigenpairs": total_k, "dofs_total": int(sum(m.n for m in meshes)),
        "hbm_budget_bytes": budget, "slots": slots,
        "plain_fp64_one_at_a_time": {"value": total_k / t_plain, "unit": "eigenpairs/s", "wall_s": t_plain},
        "mixed_one_at_a_time": {"value": total_k / t_mixed1, "unit": "eigenpairs/s", "wall_s": t_mixed1},
        "served_mixed_burst": {"value": total_k / t_burst, "unit": "eigenpairs/s", "wall_s": t_burst,
                               "requests_per_s": mu, "peak_running": info_burst["peak_running"],
                               "peak_bytes": info_burst["peak_bytes"]},
        "speedup_vs_plain_fp64": t_plain / t_burst,
        "speedup_batching_vs_mixed_one_at_a_time": t_mixed1 / t_burst,
        "served_mixed_poisson": {"arrival_rate_per_s": rate, "value": total_k / t_poisson, "unit": "eigenpairs/s",
                                 "wall_s": t_poisson, "p50_ms": float(np.percentile(lat, 50)),
                                 "p99_ms": float(np.percentile(lat, 99)),
                                 "queue_p50_ms": float(np.percentile(qms, 50)),
                                 "queue_p99_ms": float(np.percentile(qms, 99)),
                                 "peak_running": info_p["peak_running"], "peak_bytes": info_p["peak_bytes"]},
        "max_rel_eig_diff_served_vs_plain_fp64": rel, "max_residual_served": rmax,
        "unconverged": unconverged,
    }


def _poll_some(srv, ids, out, done_at):
    got = False
    for i in ids:
        if i not in out:
            r = srv.poll(i, raise_noconv=False)
            if r is not None:
                out[i] = r
                done_at[i] = time.perf_counter()
                got = True
    return got


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-breakdown", action="store_true", help="skip the untimed per-phase profile solve")
    ap.add_argument("--no-whole-job", action="store_true",
                    help="skip the whole-job legs (problem creation from device-resident and from host CSR)")
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the served mix: the first N of the 256-request workload "
                         "(0: skip the serving measurement)")
    ap.add_argument("--serve-only", action="store_true", help="only the served-mix measurement")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0, help="HBM budget of the server")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-log", default=None, help="file for per-request times of the plain FP64 serving leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain copy of known size (for scaling memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the multi-GPU path is designed, not built (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    served = None
    if args.serve_requests > 0 and not args.copy_calibration:
        # host assembly of the served meshes, before anything touches the GPU
        t0 = time.perf_counter()
        served = build_served_meshes(args.serve_requests)
        print(f"[bench] served mix: {len(served[0])} meshes assembled in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    from paper_2203_06327_amd import binding as B
    from paper_2203_06327_amd import workloads as w

    if args.serve_only:
        if served is None:
            print("--serve-only needs --serve-requests > 0", file=sys.stderr)
            sys.exit(2)
        ctx = B.Context(0)
        serving = serving_bench(B, ctx, served[0], served[1], int(args.serve_budget_gb * (1 << 30)),
                                args.serve_slots, log_path=args.serve_log)
        print(json.dumps({"metric": METRIC, "n_gpus": 1, "data": "synthetic", "serving": serving}), flush=True)
        ctx.close()
        return

    plate = args.config in w.PLATE_CONFIGS
    if plate:          # clamped plate, BFS elements: the caller's coarse space and local sets
        mesh, cfg = w.config_plate(args.config)
    else:
        mesh, cfg = w.config_mesh(args.config)
    k, s = cfg["k"], cfg["k"] + cfg["guard"]
    print(f"[bench] {args.config}: n={mesh.n} nnz={mesh.K.nnz} k={k}", file=sys.stderr, flush=True)
    ctx = B.Context(0)
    stop = B.STOP_PAPER if cfg.get("stop") == "paper" else B.STOP_RESIDUAL
    shape = B.CELL_TRIANGLE if cfg.get("shape") == "triangle" else B.CELL_SQUARE

    def make(K=None, M=None, **kw):
        K = mesh.K if K is None else K
        M = mesh.M if M is None else M
        if plate:
            return B.Problem(ctx, K, M, dd=(mesh.P, mesh.subs), k=k, guard=cfg["guard"],
                             tol=cfg.get("tol", 1e-8), **kw)
        return B.Problem(ctx, K, M, geom=(mesh.coords, mesh.cx, mesh.cy, cfg["L"], shape), k=k, guard=cfg["guard"],
                         tol=cfg.get("tol", 1e-8), stop_rule=stop, **kw)

    # timed solves: only the local-solve phase carries HIP events (two per iteration)
    prob = make(precision=B.PREC_MIXED, profile=2)
    secs, lat, stats, lam, X_d = time_solves(prob, args.steps, args.warmup, torch, k, mesh.n)
    print(f"[bench] mixed: {secs / args.steps * 1e3:.1f} ms/solve, iterations {stats[-1]['iterations']}",
          file=sys.stderr, flush=True)
    value = k * args.steps / secs
    st = stats[-1]
    i_local = B.PHASES.index("local")
    local_ms = sum(x["phase_ms"][i_local] for x in stats)
    local_n = sum(x["phase_count"][i_local] for x in stats)
    local_avg_ms = local_ms / max(1, local_n)
    nl, bw = prob.local_sizes()
    local_flops = local_solve_flops(nl, bw, s)

    # per-phase breakdown from one extra, untimed solve with every phase timed, and the
    # roofline of the whole iteration: sum over phases of the time at the peaks / measured
    ph = cnt = roof_phases = None
    if not args.no_breakdown:
        probp = make(precision=B.PREC_MIXED, profile=1)
        _, _, stp = probp.solve(torch.empty(k, dtype=torch.float64, device="cuda"),
                                torch.empty((mesh.n, k), dtype=torch.float64, device="cuda"), mem=B.MEM_DEVICE)
        torch.cuda.synchronize()
        ph = dict(zip(B.PHASES, stp["phase_ms"]))
        cnt = dict(zip(B.PHASES, stp["phase_count"]))
        probp.close()
        its = stp["iterations"]
        Pn = getattr(mesh, "P", None)
        nnzP = Pn.nnz if Pn is not None else 3 * mesh.n
        ideal = phase_ideal(mesh.n, mesh.K.nnz, s, int(nl.sum()), nnzP, prob.n_coarse, local_flops)
        ideal_ms = {q: v * its for q, v in ideal.items()}
        meas = {q: ph[q] for q in ideal}
        roof_phases = {"ideal_ms_per_solve": ideal_ms, "measured_ms_per_solve": meas,
                       "frac": sum(ideal_ms.values()) / sum(meas.values()),
                       "frac_with_setup": sum(ideal_ms.values()) / (sum(meas.values()) + ph["setup"]),
                       "iterations": its,
                       "bound": "each phase at its own peak (HBM 8 TB/s, FP32 157.3 TFLOP/s for the local solves)"}

    fp64 = None
    prob64 = None
    if not args.no_fp64:
        try:
            prob64 = make(precision=B.PREC_FP64, profile=2)
        except B.BPJDError as e:       # e.g. an FP64 local window that does not fit in LDS
            if e.code != B.ERR_DD:
                raise
            fp64 = {"skipped": str(e)}
            print(f"[bench] fp64 comparison not available: {e}", file=sys.stderr, flush=True)
    if prob64 is not None:
        secs64, lat64, stats64, lam64, _ = time_solves(prob64, max(1, args.steps // 2), 1, torch, k, mesh.n)
        fp64 = {"value": k * len(lat64) / secs64, "ms_per_solve": 1e3 * secs64 / len(lat64),
                "iterations": stats64[-1]["iterations"], "max_residual": stats64[-1]["max_residual"],
                "local_avg_launch_ms": sum(x["phase_ms"][i_local] for x in stats64)
                / max(1, sum(x["phase_count"][i_local] for x in stats64)),
                "max_rel_eig_diff_vs_mixed": float(np.max(np.abs(lam64 - lam) / np.abs(lam64)))}
        print(f"[bench] fp64: {fp64['ms_per_solve']:.1f} ms/solve, iterations {fp64['iterations']}",
              file=sys.stderr, flush=True)
        gpu_iters = stats64[-1]["iterations"]
        prob64.close()
    else:
        gpu_iters = st["iterations"]

    whole_dev = host_inclusive = None
    if not args.no_whole_job:
        # the whole job with K and M resident in HBM: problem creation from device CSR (the
        # host plans the structure: it reads the pattern back), setup, solve, eigenpairs in
        # HBM, release
        Kd, Md = B.DeviceCSR(mesh.K), B.DeviceCSR(mesh.M)
        lam_w = torch.empty(k, dtype=torch.float64, device="cuda")
        X_w = torch.empty((mesh.n, k), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        reps = 3                     # median of the repetitions (a device allocation can stall once)
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            pr = make(K=Kd, M=Md, precision=B.PREC_MIXED)
            pr.solve(lam_w, X_w, mem=B.MEM_DEVICE)
            pr.close()
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        dev_ms = float(np.median(times))
        whole_dev = {"ms_per_solve": dev_ms, "value": k / (dev_ms * 1e-3), "unit": "eigenpairs/s",
                     "runs_ms": [round(x, 1) for x in times],
                     "span": "bpjd_problem_create from device-resident CSR (host planning included) to eigenpairs "
                             "in device memory, mixed; median of the runs"}
        print(f"[bench] whole job, device-resident inputs: {dev_ms:.1f} ms/solve", file=sys.stderr, flush=True)
        del Kd, Md
        # from host CSR to eigenpairs in host memory (PCIe transfers included)
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            pr = make(precision=B.PREC_MIXED)
            pr.solve()
            pr.close()
            times.append((time.perf_counter() - t0) * 1e3)
        host_ms = float(np.median(times))
        host_inclusive = {"ms_per_solve": host_ms, "value": k / (host_ms * 1e-3), "unit": "eigenpairs/s",
                          "runs_ms": [round(x, 1) for x in times],
                          "span": "bpjd_problem_create from host CSR to eigenpairs in host memory, mixed; median of "
                                  "the runs"}
        print(f"[bench] host-inclusive: {host_ms:.1f} ms/solve", file=sys.stderr, flush=True)

    # dominant kernel of the mixed solve (the batched local LDL^T factor + solve) and its
    # roofline: algorithmic flops per launch over the average launch time measured with
    # HIP events on the library's stream inside the timed solves
    slots = 20 if plate else 4   # lower entries per local row, diagonal included
    roofline = {"bound": "alu", "achieved": local_flops / (local_avg_ms * 1e-3) / 1e12,
                "peak": PEAK["fp32_TFs"], "unit": "TFLOP/s", "traffic": None,
                "kernel": local_kernel_name(int(bw.max()), slots), "avg_launch_ms": local_avg_ms,
                "launches_timed": local_n, "algorithmic_per_launch": local_flops}
    roofline["frac"] = roofline["achieved"] / roofline["peak"]
    roofline["traffic"] = counter_traffic(args.config)
    roof_spmm = None
    if ph is not None:
        spmm_avg_ms = ph["spmm"] / max(1, cnt["spmm"])
        sb = spmm_bytes(mesh.n, mesh.K.nnz, s)
        roof_spmm = {"bound": "hbm", "achieved": sb / (spmm_avg_ms * 1e-3) / 1e9, "peak": PEAK["hbm_GBs"],
                     "unit": "GB/s", "kernel": SPMM_KERNELS.get(stp.get("spmm_form"), "unknown"),
                     "avg_launch_ms": spmm_avg_ms, "algorithmic_per_launch": sb, "source": "untimed profiled solve"}
        roof_spmm["frac"] = roof_spmm["achieved"] / roof_spmm["peak"]

    # correctness of the returned pairs against the paper's printed values where they exist
    check = {}
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from conftest import load_golden_table
    if args.config == "c2":
        check["max_abs_err_vs_table1"] = float(np.max(np.abs(lam / np.pi ** 2 - load_golden_table("table1.txt")[:k, 2])))
    if "table1_col" in cfg:
        check["max_abs_err_vs_table1"] = float(np.max(np.abs(lam - load_golden_table("table1.txt")[:k, cfg["table1_col"]])))
    if "table3_col" in cfg:
        check["max_abs_err_vs_table3"] = float(np.max(np.abs(lam - load_golden_table("table3.txt")[:k, cfg["table3_col"]])))
    if args.config == "c3":
        ref = np.array([float(line.split()[1]) for line in open(os.path.join(ROOT, "tests", "golden", "c3_reference.txt"))
                        if not line.startswith("#")])[:k]
        check["max_rel_err_vs_oracle_reference"] = float(np.max(np.abs(lam - ref) / ref))

    serving = None
    if served is not None:
        serving = serving_bench(B, ctx, served[0], served[1], int(args.serve_budget_gb * (1 << 30)),
                                args.serve_slots, log_path=args.serve_log)

    cpu = None
    if not args.no_cpu_baseline:
        cfg_cpu = dict(cfg, n_sub_all=prob.n_sub)
        cpu = cpu_baseline(mesh, cfg_cpu, gpu_iters)
        print(f"[bench] cpu baseline: {cpu['sample']}", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": value, "unit": "eigenpairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * secs / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"{args.config}: {cfg['desc']}", "n": mesh.n, "k": k, "s": s,
                   "n_sub": prob.n_sub, "n_coarse": prob.n_coarse, "precision": "mixed (FP32 local solves)",
                   "subspace": "UU",
                   "stop": ("sum |dlambda| < %g" % cfg["tol"]) if stop == B.STOP_PAPER
                   else f"max relative residual <= {cfg.get('tol', 1e-8):g}"},
        "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "iterations": st["iterations"], "max_residual": st["max_residual"], "stop_value": st["stop_value"],
        "fp64": fp64, "whole_job_device_inputs": whole_dev, "host_inclusive": host_inclusive,
        "phase_ms_per_solve": ph, "phase_launches": cnt, "roofline": roofline, "roofline_phases": roof_phases,
        "roofline_spmm": roof_spmm, "cpu_baseline": cpu, "serving": serving, **check,
    }
    print(json.dumps(out), flush=True)
    prob.close()
    ctx.close()


if __name__ == "__main__":
    main()

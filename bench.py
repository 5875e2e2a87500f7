"""Throughput benchmark of the batched eigensolver on one MI355X.

A step is one solve (eigenvalues + eigenvectors) of the batch-512 FP32 n=64
workload: half Gaussian symmetric (G+G^T)/2, half covariance X^T X/(4n), 10%
of the matrices with a planted eigenvalue pair 1e-6 apart.  Inputs are resident
in HBM before timing starts.  The same run times n=32 and n=48 (reported under
"per_n"), a short serving loop (p50/p99 latency), and the binary64 oracle on
the host cores ("cpu_baseline").

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector (and FP32 MFMA) peak
BATCH = 512


def flop_model(n):
    """Algorithmic flops of one n x n solve (fixed model, no deflation credit):
    4/3 n^3 tridiagonalization + 2 n^3 back-transform + sum over merges of
    2 m (m1^2 + m2^2) back-multiplication + 54 m^2 secular/Loewner work."""
    merges = []

    def walk(d, j):
        lo, hi = (j * n) >> d, ((j + 1) * n) >> d
        if hi - lo <= 2:
            return
        s = ((2 * j + 1) * n) >> (d + 1)
        merges.append((hi - lo, s - lo, hi - s))
        walk(d + 1, 2 * j)
        walk(d + 1, 2 * j + 1)

    walk(0, 0)
    gemm = sum(2 * m * (m1 * m1 + m2 * m2) for m, m1, m2 in merges)
    sec = sum(54 * m * m for m, _, _ in merges)
    return 4.0 / 3.0 * n ** 3 + 2.0 * n ** 3 + gemm + sec


def time_solver(bed, torch, A, steps, warmup):
    """Returns (ms per step by wall clock, ms per launch by HIP events)."""
    b, n = A.shape[0], A.shape[1]
    lam = torch.empty(b, n, device=A.device, dtype=A.dtype)
    Q = torch.empty_like(A)
    info = torch.empty(b, dtype=torch.int32, device=A.device)
    flat, lflat = A.view(-1), lam.view(-1)
    qflat = Q.view(-1)
    nl = [n] * b
    for _ in range(warmup):
        bed.syevd_packed(nl, flat, lam=lflat, Q=qflat, info=info)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        bed.syevd_packed(nl, flat, lam=lflat, Q=qflat, info=info)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    ev = e0.elapsed_time(e1) / steps
    return wall, ev, lam, Q, info


def parity_sample(oracle, A_np, lam, Q, info, count=16):
    """Oracle check of sampled outputs of the timed launch."""
    from tests.parity import compare_batch
    idx = np.linspace(0, A_np.shape[0] - 1, count).astype(int)
    lam_o, Q_o, _ = oracle.syevd(A_np[idx].astype(np.float64))
    worst, fails = compare_batch(A_np[idx], lam[idx], Q[idx], lam_o, Q_o, np.float32,
                                 info=info[idx])
    return {"sampled": int(count), "failures": len(fails),
            "max_lambda_err_rel": float(worst.get("lam", 0.0)),
            "max_residual": float(worst.get("res", 0.0)),
            "max_orthogonality": float(worst.get("orth", 0.0))}


def cpu_baseline(oracle, A_np, budget_s):
    """The binary64 oracle (single thread, as committed) on a bounded sample."""
    A64 = A_np.astype(np.float64)
    done, t0 = 0, time.perf_counter()
    while True:
        chunk = A64[done % A64.shape[0]: done % A64.shape[0] + 16]
        oracle.syevd(chunk)
        done += chunk.shape[0]
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": done / el, "unit": "eigendecomps/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} matrices of the n={A_np.shape[1]} FP32 workload (promoted to "
                      f"FP64), {el:.1f} s single-threaded"}


def serving_leg(bed, torch, requests, qps, seed=5000):
    """Open-loop Poisson trace through the continuous-batching server."""
    from paper_2604_27325_amd import workloads
    arr, counts, ns = workloads.serving_trace(seed=seed, requests=requests, qps=qps)
    bufs = []
    for i in range(requests):
        A = torch.from_numpy(workloads.serving_matrices(seed + 1 + i, int(counts[i]), int(ns[i])))
        bufs.append(A.to("cuda"))
    outs = [(torch.empty(b.shape[0], b.shape[1], device="cuda"), torch.empty_like(b)) for b in bufs]
    torch.cuda.synchronize()
    srv = bed.Server(streams=4)
    tickets = []
    t0 = time.perf_counter()
    for i in range(requests):
        while time.perf_counter() - t0 < arr[i]:
            pass
        tk = None
        while tk is None:
            tk = srv.submit(bufs[i], outs[i][0], outs[i][1])
        tickets.append(tk)
    srv.drain()
    el = time.perf_counter() - t0
    lats = []
    for tk in tickets:
        done, lat = srv.poll(tk)
        lats.append(lat)
    srv.close()
    lats = np.asarray(lats)
    mats = int(np.sum(counts))
    return {"requests": requests, "qps_offered": qps, "matrices": mats,
            "matrices_per_s": mats / el, "p50_ms": float(np.percentile(lats, 50) / 1e3),
            "p99_ms": float(np.percentile(lats, 99) / 1e3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--serve-qps", type=float, default=1000.0)
    ap.add_argument("--only-n", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver shards by matrix with no "
              "cross-GPU step, so multi-GPU runs are not part of this benchmark",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_27325_amd as bed
    from paper_2604_27325_amd import workloads

    bed.load_library()
    per_n = {}
    main_res = None
    sizes = [args.only_n] if args.only_n else [32, 48, 64]
    for n in sizes:
        A_np, _, _ = workloads.paper_scale(n)
        A = torch.from_numpy(A_np).to("cuda")
        wall, ev, lam, Q, info = time_solver(bed, torch, A, args.steps, args.warmup)
        F = flop_model(n)
        per_n[str(n)] = {"eigendecomps_per_s": BATCH / (wall * 1e-3), "ms_per_step": wall,
                         "kernel_ms": ev, "tflops_model": BATCH * F / (ev * 1e-3) / 1e12,
                         "flops_per_matrix": F}
        if n == sizes[-1]:
            main_res = (n, A_np, wall, ev, lam.cpu().numpy(), Q.cpu().numpy(), info.cpu().numpy())

    n, A_np, wall, ev, lam, Q, info = main_res
    F = flop_model(n)
    achieved = BATCH * F / (ev * 1e-3) / 1e12
    import oracle
    parity = parity_sample(oracle, A_np, lam, Q, info)
    cpu = None if args.no_cpu else cpu_baseline(oracle, A_np, args.cpu_seconds)
    serving = None if args.no_serve else serving_leg(bed, torch, args.serve_requests,
                                                     args.serve_qps)
    line = {
        "metric": "eigendecomps/sec at n=64 fp32 batch 512 (n=32, n=48 under per_n; "
                  "p50/p99 under serving)",
        "value": BATCH / (wall * 1e-3),
        "unit": "eigendecomps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch {BATCH} FP32 symmetric n={n}: half Gaussian (G+G^T)/2, "
                               "half covariance X^T X/(4n), 10% planted 1e-6 eigenpairs",
                   "batch": BATCH, "n": n},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "k_syevd_uniform<float,64,256>",
                     "flops_per_launch": BATCH * F, "kernel_ms": ev},
        "cpu_baseline": cpu,
        "per_n": per_n,
        "parity": parity,
        "serving": serving,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

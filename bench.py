"""Throughput benchmark of the batched eigensolver on one MI355X.

A step is one solve (eigenvalues + eigenvectors) of the batch-512 FP32 n=64
workload: half Gaussian symmetric (G+G^T)/2, half covariance X^T X/(4n), 10%
of the matrices with a planted eigenvalue pair 1e-6 apart.  Inputs are resident
in HBM before timing starts.  The same run also measures

  per_n         the batch-512 workload at n=32 and n=48;
  uneven        4096 matrices with n ~ U{4..64}: autotuned plan replayed from a
                HIP graph vs one plain launch per distinct n;
  backward      batch 1024, n=32 forward + backward (eigengaps >= 1e-3);
  serving       a Poisson trace of requests (1-256 matrices, n in {8,..,64})
                through the continuous-batching server at 0.5 and 0.9 of the
                closed-loop saturation rate, vs plain sequential launches;
  cpu_baseline  the binary64 oracle on the host cores, on a bounded sample.

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

# MI355X FP32 vector peak: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2 (dual
# issue / packed FP32) x 2.4 GHz = 157.3 TFLOP/s; FP32 MFMA has the same figure.
PEAK_FP32_TFLOPS = 157.3
BATCH = 512


def nmax_of(n):
    """Size class of the solver's team for order n."""
    return 16 if n <= 16 else (32 if n <= 32 else 64)


def threads_of(n):
    """Threads per matrix of the default schedule for order n."""
    return {16: 64, 32: 256, 64: 512}[nmax_of(n)]


def merge_tree(n):
    """(m, m1, m2) of every merge of the dyadic tearing tree of size n."""
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
    return merges


def flop_model(n):
    """Algorithmic flops of one n x n solve (fixed model, no deflation credit):
    4/3 n^3 tridiagonalization + 2 n^3 back-transform + sum over merges of
    2 m (m1^2 + m2^2) back-multiplication + 54 m^2 secular/Loewner work."""
    merges = merge_tree(n)
    gemm = sum(2 * m * (m1 * m1 + m2 * m2) for m, m1, m2 in merges)
    sec = sum(54 * m * m for m, _, _ in merges)
    return 4.0 / 3.0 * n ** 3 + 2.0 * n ** 3 + gemm + sec


def backward_flops(n):
    """dA = Q (diag(dlam) + sym(F o Q^T dQ)) Q^T: three n x n x n products."""
    return 6.0 * n ** 3


def profiled_traffic(name):
    """HBM bytes per launch from the committed counter summary profiles/<name>.md,
    or None when the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name + ".md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if " = " in line:
            k, v = line.split(" = ", 1)
            kv[k.strip()] = v.strip()
    try:
        h = hashlib.sha256()
        for src in kv["kernel_sources"].split():
            with open(os.path.join(ROOT, "paper_2604_27325_amd", "csrc", src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != kv["kernel_sources_sha256"]:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def timed(torch, fn, steps, warmup, stream=None, per_step=False):
    """(wall ms per step, event ms per step) of `steps` calls of fn() after
    `warmup` untimed ones, events on `stream` (torch's current stream if None).
    per_step: also return the per-call event times (ms), one event pair per call."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = stream or torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if per_step else None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for i in range(steps):
        if per_step:
            evs[i].record(stream)
        fn()
    if per_step:
        evs[steps].record(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    if per_step:
        each = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
        return wall, e0.elapsed_time(e1) / steps, each
    return wall, e0.elapsed_time(e1) / steps


def time_solver(bed, torch, A, steps, warmup):
    """Returns (ms per step by wall clock, ms per launch by HIP events, outputs)."""
    b, n = A.shape[0], A.shape[1]
    lam = torch.empty(b, n, device=A.device, dtype=A.dtype)
    Q = torch.empty_like(A)
    info = torch.empty(b, dtype=torch.int32, device=A.device)
    flat, lflat, qflat = A.view(-1), lam.view(-1), Q.view(-1)
    nl = [n] * b
    wall, ev, each = timed(torch, lambda: bed.syevd_packed(nl, flat, lam=lflat, Q=qflat,
                                                            info=info),
                           steps, warmup, per_step=True)
    return wall, ev, each, lam, Q, info


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(oracle, A64, budget_s, threads):
    """Matrices/s of the oracle over `threads` host threads (the ctypes calls
    release the interpreter lock, so threads run the C code in parallel), one
    16-matrix chunk of the workload per task, for about budget_s seconds."""
    import concurrent.futures
    import itertools
    chunks = [A64[i:i + 16] for i in range(0, A64.shape[0], 16)]
    it = itertools.cycle(chunks)
    done, t0 = 0, time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        while True:
            batch = [next(it) for _ in range(threads)]
            list(ex.map(oracle.syevd, batch))
            done += sum(c.shape[0] for c in batch)
            el = time.perf_counter() - t0
            if el >= budget_s:
                return done / el, done, el


def cpu_baseline(oracle, A_np, budget_s):
    """The binary64 oracle as committed, on the host cores of this run: all
    cores (the reported value, cores = threads used) and one thread, each on a
    bounded sample of the same workload; LAPACK (numpy eigh, binary64) on the
    same matrices as context."""
    A64 = A_np.astype(np.float64)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    threads = max(1, min(avail, 16))
    v1, d1, e1 = _oracle_rate(oracle, A64, budget_s / 2, 1)
    vn, dn, en = _oracle_rate(oracle, A64, budget_s / 2, threads)
    t0 = time.perf_counter()
    reps = 0
    while time.perf_counter() - t0 < 1.0:
        np.linalg.eigh(A64[:64])
        reps += 1
    lapack = reps * 64 / (time.perf_counter() - t0)
    return {"value": vn, "unit": "eigendecomps/s", "cores": threads, "kind": "oracle",
            "sample": f"{dn} matrices of the batch-512 n={A_np.shape[1]} FP32 workload "
                      f"(promoted to FP64) in {en:.1f} s on {threads} threads; "
                      f"{d1} in {e1:.1f} s on one thread",
            "single_thread_value": v1, "nproc": os.cpu_count(), "affinity_cpus": avail,
            "cpu_model": cpu_model(),
            "context_numpy_eigh_binary64": lapack}


def eigenvalues_leg(bed, torch, A, A_np, oracle, steps, warmup):
    """Eigenvalues only (Sec. 2.3.5: vectors are formed only when required) on
    the timed workload: per-launch time, rate, and the oracle's eigenvalues on
    sampled matrices."""
    b, n = A.shape[0], A.shape[1]
    lam = torch.empty(b * n, device=A.device, dtype=A.dtype)
    info = torch.empty(b, dtype=torch.int32, device=A.device)
    flat, nl = A.view(-1), [n] * b
    wall, ev, each = timed(torch, lambda: bed.syevd_packed(nl, flat, lam=lam, info=info,
                                                            want_vectors=False),
                           steps, warmup, per_step=True)
    from tests.parity import compare_batch
    lam = lam.view(b, n).cpu().numpy()
    idx = np.linspace(0, b - 1, 16).astype(int)
    lam_o = oracle.syevd(A_np[idx].astype(np.float64))[0]
    worst, fails = compare_batch(A_np[idx], lam[idx], None, lam_o, None, np.float32,
                                 info=info.cpu().numpy()[idx])
    err = float(worst.get("lam", 0.0))
    return {"eigendecomps_per_s": b / (wall * 1e-3), "ms_per_step": wall, "kernel_ms": ev,
            "launch_us_median": float(np.median(each) * 1e3),
            "launch_us_p10": float(np.percentile(each, 10) * 1e3),
            "launch_us_p90": float(np.percentile(each, 90) * 1e3),
            "sampled": 16, "failures": len(fails), "max_lambda_err_rel": err,
            "info_nonzero": int((info.cpu().numpy() != 0).sum())}


def leaf_leg(bed, torch, steps, warmup, sizes=(32, 64)):
    """Per-launch time of the batch-512 solve with leaves of at most 2, 4 or 8
    elements (Sec. 2.2: the divide step may stop early and hand small blocks to
    Jacobi); the default cutoff is 4."""
    from paper_2604_27325_amd import workloads
    out = {}
    for n in sizes:
        A = torch.from_numpy(workloads.paper_scale(n)[0]).to("cuda")
        flat, nl = A.view(-1), [n] * A.shape[0]
        lam = torch.empty(A.shape[0] * n, device="cuda")
        Q = torch.empty_like(flat)
        row = {}
        for leaf in (2, 4, 8):
            plan = bed.Plan(torch.float32, nl, tune={"leaf": leaf})
            _, ev, each = timed(torch, lambda: plan.run(flat, lam, Q), steps, warmup, per_step=True)
            row[str(leaf)] = {"kernel_us": ev * 1e3, "launch_us_median": float(np.median(each) * 1e3)}
            plan.close()
        out[str(n)] = row
    return out


def uneven_leg(bed, torch, steps, warmup):
    """4096 FP32 matrices, n ~ U{4..64}: autotuned persistent plan replayed from
    a HIP graph, against one plain bed_syevd launch per distinct n."""
    from paper_2604_27325_amd import workloads
    ns, mats = workloads.uneven()
    ns_list = [int(v) for v in ns]
    _, flat = workloads.pack(mats)
    A = torch.from_numpy(flat).to("cuda")
    lam = torch.empty(int(ns.sum()), device="cuda")
    Q = torch.empty_like(A)
    info = torch.empty(len(ns_list), dtype=torch.int32, device="cuda")
    tune = bed.autotune(torch.float32, ns_list, A, lam, Q)
    plan = bed.Plan(torch.float32, ns_list, tune=tune)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.run(A, lam, Q, info, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.run(A, lam, Q, info, stream=s)
    torch.cuda.synchronize()
    wall_g, ev_g = timed(torch, g.replay, steps, warmup)
    wall_p, ev_p = timed(torch, lambda: plan.run(A, lam, Q, info), steps, warmup)
    # per-size plain launches on contiguous per-n buffers, eagerly and replayed
    # from one graph (device work only, without the host's launch cost)
    groups = {}
    for i, n in enumerate(ns_list):
        groups.setdefault(n, []).append(mats[i])
    per = []
    for n, ms in sorted(groups.items()):
        An = torch.from_numpy(np.stack(ms)).to("cuda")
        per.append((An, torch.empty(An.shape[0], n, device="cuda"), torch.empty_like(An)))

    def plain(stream=None):
        for An, ln, Qn in per:
            bed.syevd_packed([An.shape[1]] * An.shape[0], An.view(-1), lam=ln.view(-1),
                             Q=Qn.view(-1), stream=stream)

    wall_s, ev_s = timed(torch, plain, steps, warmup)
    with torch.cuda.stream(s):
        plain(stream=s)
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=s):
        plain(stream=s)
    torch.cuda.synchronize()
    wall_sg, ev_sg = timed(torch, g2.replay, steps, warmup)
    flops = sum(flop_model(n) for n in ns_list)
    b = len(ns_list)
    return {"matrices": b, "distinct_n": len(groups), "schedule": tune,
            "graph": {"eigendecomps_per_s": b / (wall_g * 1e-3), "ms_per_step": wall_g,
                      "kernel_ms": ev_g, "tflops_model": flops / (ev_g * 1e-3) / 1e12},
            "plan_eager": {"eigendecomps_per_s": b / (wall_p * 1e-3), "ms_per_step": wall_p},
            "per_size_plain": {"eigendecomps_per_s": b / (wall_s * 1e-3), "ms_per_step": wall_s,
                               "launches": len(groups)},
            "per_size_plain_graph": {"eigendecomps_per_s": b / (wall_sg * 1e-3),
                                     "ms_per_step": wall_sg, "kernel_ms": ev_sg},
            "speedup_vs_per_size": wall_s / wall_g,
            "speedup_vs_per_size_graph": wall_sg / wall_g}


def backward_leg(bed, torch, steps, warmup):
    """Batch 1024 FP32 n=32 (eigengaps >= 1e-3): forward, backward, both."""
    from paper_2604_27325_amd import workloads
    A_np, dlam_np, dQ_np, _ = workloads.differentiation()
    A = torch.from_numpy(A_np).to("cuda")
    dlam, dQ = torch.from_numpy(dlam_np).to("cuda"), torch.from_numpy(dQ_np).to("cuda")
    lam, Q = bed.syevd(A)
    dA = torch.empty_like(A)
    b, n = A.shape[0], A.shape[1]
    nl = [n] * b

    def fwd():
        bed.syevd_packed(nl, A.view(-1), lam=lam.view(-1), Q=Q.view(-1))

    def bwd():
        bed.syevd_backward(lam, Q, dlam, dQ, out=dA)

    def both():
        fwd()
        bwd()

    wall_f, ev_f = timed(torch, fwd, steps, warmup)
    wall_b, ev_b = timed(torch, bwd, steps, warmup)
    wall_fb, _ = timed(torch, both, steps, warmup)
    # device time: the calls replayed from HIP graphs (an eager call of the
    # short backward kernel is paced by the host's launch cost)
    g_b, g_fb = _graph_of(torch, bwd), _graph_of(torch, both)
    wall_gb, ev_gb = timed(torch, g_b.replay, steps, warmup)
    wall_gfb, ev_gfb = timed(torch, g_fb.replay, steps, warmup)
    ev_gb /= GRAPH_REPS
    ev_gfb /= GRAPH_REPS
    return {"batch": b, "n": n,
            "forward_ms": wall_f, "backward_ms": wall_b, "backward_eager_event_ms": ev_b,
            "forward_backward_ms": wall_fb,
            "backward_kernel_ms": ev_gb, "forward_backward_graph_ms": ev_gfb,
            "eigendecomps_per_s_fwd_bwd": b / (ev_gfb * 1e-3),
            "backward_tflops": b * backward_flops(n) / (ev_gb * 1e-3) / 1e12}


GRAPH_REPS = 10


def _graph_of(torch, fn, reps=GRAPH_REPS):
    """reps calls of fn() captured in one HIP graph on a side stream (after one
    eager warm-up); a replay's time divided by reps is the device time of one
    call without the launch cost of a graph per call."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(reps):
            fn()
    torch.cuda.synchronize()
    return g


def spectral_leg(bed, torch, steps, warmup):
    """Matrix square root of batch 1024 FP32 covariance matrices n = 32 (the
    meta-layer use): decomposition + Q sqrt(Lambda) Q^T forward, and the
    divided-difference backward, replayed from HIP graphs."""
    from paper_2604_27325_amd import workloads
    A_np, _, dQ_np, _ = workloads.differentiation()
    A = torch.from_numpy(A_np).to("cuda")
    dF = torch.from_numpy(dQ_np).to("cuda")
    b, n = A.shape[0], A.shape[1]
    lam, Q = bed.syevd(A)
    F, dA = torch.empty_like(A), torch.empty_like(A)
    nl = [n] * b

    def fwd():
        bed.syevd_packed(nl, A.view(-1), lam=lam.view(-1), Q=Q.view(-1))
        bed.spectral_apply(lam, Q, "sqrt", out=F)

    def bwd():
        bed.spectral_backward(lam, Q, dF, "sqrt", out=dA)

    def both():
        fwd()
        bwd()

    _, ev_f = timed(torch, _graph_of(torch, fwd).replay, steps, warmup)
    _, ev_b = timed(torch, _graph_of(torch, bwd).replay, steps, warmup)
    _, ev_fb = timed(torch, _graph_of(torch, both).replay, steps, warmup)
    ev_f, ev_b, ev_fb = ev_f / GRAPH_REPS, ev_b / GRAPH_REPS, ev_fb / GRAPH_REPS
    return {"batch": b, "n": n, "function": "sqrt", "forward_ms": ev_f,
            "backward_ms": ev_b, "forward_backward_ms": ev_fb,
            "matrices_per_s_fwd_bwd": b / (ev_fb * 1e-3)}


class _ServeData:
    """Per-request input views into per-n pools and private output buffers."""

    def __init__(self, torch, counts, ns, seed):
        from paper_2604_27325_amd import workloads
        pool_sz = 1024
        self.pools = {}
        for n in sorted(set(int(v) for v in ns)):
            self.pools[n] = torch.from_numpy(
                workloads.serving_matrices(seed + n, pool_sz, n)).to("cuda")
        rng = np.random.default_rng(seed)
        lam_tot = int(np.sum(counts.astype(np.int64) * ns))
        q_tot = int(np.sum(counts.astype(np.int64) * ns * ns))
        self.lam_all = torch.empty(lam_tot, device="cuda")
        self.q_all = torch.empty(q_tot, device="cuda")
        self.req = []
        ol = oq = 0
        for c, n in zip(counts.tolist(), ns.tolist()):
            off = int(rng.integers(0, pool_sz - c + 1))
            A = self.pools[n][off:off + c]
            lam = self.lam_all[ol:ol + c * n].view(c, n)
            Q = self.q_all[oq:oq + c * n * n].view(c, n, n)
            self.req.append((A, lam, Q))
            ol += c * n
            oq += c * n * n


def _serve_server(bed, data, arrivals, streams=4, producer=None):
    """Open loop through the server (arrivals=None: closed loop, all at t=0).
    Latency = arrival -> completion observed by the server's scheduler.
    `producer` is the stream the requests name as the producer of their input
    (None: torch's current stream)."""
    srv = bed.Server(streams=streams)
    R = len(data.req)
    arr = np.zeros(R) if arrivals is None else arrivals
    tickets, sub = [], np.zeros(R)
    t0 = time.perf_counter()
    for i in range(R):
        while time.perf_counter() - t0 < arr[i]:
            pass
        A, lam, Q = data.req[i]
        tk = srv.submit(A, lam, Q, stream=producer)
        while tk is None:
            tk = srv.submit(A, lam, Q, stream=producer)
        sub[i] = time.perf_counter() - t0
        tickets.append(tk)
    srv.drain()
    el = time.perf_counter() - t0
    lats = np.empty(R)
    for i, tk in enumerate(tickets):
        done, lat_us = srv.poll(tk)
        lats[i] = (sub[i] - arr[i]) * 1e3 + lat_us * 1e-3
    srv.close()
    return el, lats


def _serve_plain(bed, torch, data, arrivals):
    """The same trace as plain sequential bed_syevd calls on one stream;
    latency = arrival -> completion event observed on the host."""
    R = len(data.req)
    s = torch.cuda.Stream()
    evs = [None] * R
    done_t = np.zeros(R)
    head = 0
    t0 = time.perf_counter()

    def reap(upto):
        nonlocal head
        while head < upto and evs[head].query():
            done_t[head] = time.perf_counter() - t0
            head += 1

    with torch.cuda.stream(s):
        for i in range(R):
            while time.perf_counter() - t0 < arrivals[i]:
                reap(i)
            A, lam, Q = data.req[i]
            bed.syevd_packed([A.shape[1]] * A.shape[0], A.reshape(-1), lam=lam.reshape(-1),
                             Q=Q.reshape(-1), stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
            evs[i] = ev
            reap(i)
        while head < R:
            reap(R)
    el = time.perf_counter() - t0
    return el, (done_t - arrivals) * 1e3


def serving_leg(bed, torch, requests, fracs=(0.5, 0.9), seed=5000):
    """Saturation rates of the server and of plain sequential launches from
    closed loops, then open-loop Poisson traces at 0.5 and 0.9 of the server's
    rate and at 0.5 of the plain path's (a load both can sustain), each through
    the server and through plain sequential launches."""
    from paper_2604_27325_amd import workloads
    _, counts, ns = workloads.serving_trace(seed=seed, requests=requests, qps=1.0)
    data = _ServeData(torch, counts, ns, seed + 1)
    mats = int(np.sum(counts))
    _serve_server(bed, data, None)  # warm-up
    el, _ = _serve_server(bed, data, None)
    r_sat = requests / el
    el_p, _ = _serve_plain(bed, torch, data, np.zeros(requests))
    r_plain = requests / el_p
    out = {"requests": requests, "matrices": mats, "saturation_requests_per_s": r_sat,
           "saturation_matrices_per_s": mats / el,
           "plain_saturation_requests_per_s": r_plain,
           "plain_saturation_matrices_per_s": mats / el_p, "loads": []}
    offered = [(f, f * r_sat, "server saturation") for f in fracs] + \
        [(0.5, 0.5 * r_plain, "plain saturation")]
    for f, qps, of in offered:
        arr, _, _ = workloads.serving_trace(seed=seed, requests=requests, qps=qps)
        el_s, lat_s = _serve_server(bed, data, arr)
        el_p, lat_p = _serve_plain(bed, torch, data, arr)
        out["loads"].append({
            "fraction_of": of, "fraction": f, "qps_offered": qps,
            "server": {"matrices_per_s": mats / el_s, "p50_ms": float(np.percentile(lat_s, 50)),
                       "p99_ms": float(np.percentile(lat_s, 99))},
            "plain_sequential": {"matrices_per_s": mats / el_p,
                                 "p50_ms": float(np.percentile(lat_p, 50)),
                                 "p99_ms": float(np.percentile(lat_p, 99))}})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the batch-512 legs (no uneven / backward / serving)")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--only-n", type=int, default=0)
    ap.add_argument("--no-big", action="store_true", help="skip the n = 128 entry of per_n")
    ap.add_argument("--main-only", action="store_true",
                    help="only the timed batch-512 solves and their parity sample (profiler "
                         "runs: no other launch of the same kernel)")
    ap.add_argument("--only-leg", choices=["uneven", "backward", "spectral", "serving", "leaf"],
                    default=None, help="run only this leg (for profiler passes); no JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also launch one 256 MiB device copy (HBM counter calibration)")
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
    if args.only_leg:
        leg = {"uneven": lambda: uneven_leg(bed, torch, args.steps, args.warmup),
               "backward": lambda: backward_leg(bed, torch, args.steps, args.warmup),
               "spectral": lambda: spectral_leg(bed, torch, args.steps, args.warmup),
               "serving": lambda: serving_leg(bed, torch, args.serve_requests),
               "leaf": lambda: leaf_leg(bed, torch, args.steps, args.warmup)}[args.only_leg]()
        print(f"[bench] {args.only_leg}: {json.dumps(leg)}", flush=True)
        return
    if args.copy_calibration:
        src = torch.ones(64 << 20, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {src.numel() * 4} bytes read, "
              f"{dst.numel() * 4} bytes written", flush=True)
    per_n = {}
    main_res = None
    sizes = [args.only_n] if args.only_n else [32, 48, 64]
    for n in sizes:
        A_np, _, _ = workloads.paper_scale(n)
        A = torch.from_numpy(A_np).to("cuda")
        wall, ev, each, lam, Q, info = time_solver(bed, torch, A, args.steps, args.warmup)
        F = flop_model(n)
        per_n[str(n)] = {"eigendecomps_per_s": BATCH / (wall * 1e-3), "ms_per_step": wall,
                         "kernel_ms": ev, "tflops_model": BATCH * F / (ev * 1e-3) / 1e12,
                         "flops_per_matrix": F,
                         "launch_us_median": float(np.median(each) * 1e3),
                         "launch_us_p10": float(np.percentile(each, 10) * 1e3),
                         "launch_us_p90": float(np.percentile(each, 90) * 1e3)}
        print(f"[bench] n={n}: {per_n[str(n)]['eigendecomps_per_s']:.4g} matrices/s, "
              f"kernel {ev * 1e3:.1f} us", flush=True)
        if n == 64 and not args.main_only:
            # the same solve with one team per CU (batch = number of CUs): one
            # matrix's chain latency with nothing sharing its CU
            cus = torch.cuda.get_device_properties(0).multi_processor_count
            A1 = A[:cus].contiguous()
            _, ev1, each1, _, _, _ = time_solver(bed, torch, A1, args.steps, args.warmup)
            per_n[str(n)]["one_team_per_cu"] = {
                "batch": cus, "kernel_ms": ev1,
                "launch_us_median": float(np.median(each1) * 1e3),
                "batch_512_over_this": float(np.median(each) / np.median(each1))}
            print(f"[bench] n=64 one team per CU (batch {cus}): {ev1 * 1e3:.1f} us", flush=True)
        if n == sizes[-1]:
            main_res = (n, A_np, wall, ev, lam.cpu().numpy(), Q.cpu().numpy(), info.cpu().numpy())

    if not args.only_n and not args.no_big and not args.main_only:
        # 64 < n <= 128: one more tearing step above the n <= 64 kernels
        nb = 128
        A_np_b, _, _ = workloads.paper_scale(nb)
        A_b = torch.from_numpy(A_np_b).to("cuda")
        wall_b, ev_b, each_b, lam_b, Q_b, info_b = time_solver(bed, torch, A_b,
                                                              max(args.steps // 4, 10),
                                                              max(args.warmup // 4, 3))
        import oracle as _orc
        F_b = flop_model(nb)
        per_n[str(nb)] = {"eigendecomps_per_s": BATCH / (wall_b * 1e-3), "ms_per_step": wall_b,
                          "kernel_ms": ev_b, "tflops_model": BATCH * F_b / (ev_b * 1e-3) / 1e12,
                          "flops_per_matrix": F_b,
                          "launch_us_median": float(np.median(each_b) * 1e3),
                          "launch_us_p10": float(np.percentile(each_b, 10) * 1e3),
                          "launch_us_p90": float(np.percentile(each_b, 90) * 1e3),
                          "kernels": "reduce + tear, Householder product, halves on the n <= 64 kernels, top merge",
                          "parity": parity_sample(_orc, A_np_b, lam_b.cpu().numpy(),
                                                  Q_b.cpu().numpy(), info_b.cpu().numpy())}
        print(f"[bench] n={nb}: {per_n[str(nb)]['eigendecomps_per_s']:.4g} matrices/s, "
              f"{ev_b * 1e3:.1f} us per solve", flush=True)
        del A_b, lam_b, Q_b

    n, A_np, wall, ev, lam, Q, info = main_res
    F = flop_model(n)
    achieved = BATCH * F / (ev * 1e-3) / 1e12
    import oracle
    parity = parity_sample(oracle, A_np, lam, Q, info)
    evals = None
    if not args.main_only:
        A = torch.from_numpy(A_np).to("cuda")
        evals = eigenvalues_leg(bed, torch, A, A_np, oracle, args.steps, args.warmup)
        print(f"[bench] n={n} eigenvalues only: {evals['eigendecomps_per_s']:.4g} matrices/s, "
              f"kernel {evals['kernel_ms'] * 1e3:.1f} us", flush=True)
    uneven = backward = serving = spectral = leaves = None
    if not args.no_extra and not args.main_only:
        leaves = leaf_leg(bed, torch, max(args.steps // 2, 10), max(args.warmup // 2, 3))
        print(f"[bench] leaf cutoff: {json.dumps(leaves)}", flush=True)
        uneven = uneven_leg(bed, torch, max(args.steps // 4, 10), max(args.warmup // 4, 3))
        print(f"[bench] uneven: graph {uneven['graph']['eigendecomps_per_s']:.4g} matrices/s, "
              f"{uneven['speedup_vs_per_size']:.2f}x per-size launches", flush=True)
        backward = backward_leg(bed, torch, args.steps, args.warmup)
        print(f"[bench] backward: {backward['backward_kernel_ms'] * 1e3:.1f} us", flush=True)
        spectral = spectral_leg(bed, torch, args.steps, args.warmup)
        print(f"[bench] spectral sqrt: fwd {spectral['forward_ms'] * 1e3:.1f} us, bwd "
              f"{spectral['backward_ms'] * 1e3:.1f} us", flush=True)
        if not args.no_serve:
            serving = serving_leg(bed, torch, args.serve_requests)
            print(f"[bench] serving: saturation {serving['saturation_matrices_per_s']:.4g} "
                  "matrices/s", flush=True)
    cpu = None if (args.no_cpu or args.main_only) else cpu_baseline(oracle, A_np, args.cpu_seconds)
    line = {
        "metric": "eigendecomps/sec at n=64 fp32 batch 512 (n=32, n=48 under per_n; "
                  "p50/p99 latency under serving)",
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
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": profiled_traffic(f"k_syevd_uniform_f32_n{n}_b{BATCH}"),
                     "kernel": (f"k_syevd_uniform<float, {nmax_of(n)}, {threads_of(n)}>" if n <= 64
                                else "k_big_reduce, k_big_qh, k_syevd_tri, k_big_merge (one solve)"),
                     "flops_per_launch": BATCH * F, "kernel_ms": ev},
        "latency": None if "one_team_per_cu" not in per_n.get(str(n), {}) else {
            "one_matrix_chain_us": per_n[str(n)]["one_team_per_cu"]["kernel_ms"] * 1e3,
            "launch_us": ev * 1e3,
            "frac": per_n[str(n)]["one_team_per_cu"]["kernel_ms"] / ev,
            "note": "two matrices per CU at batch 512: frac 1 would mean the second one "
                    "costs nothing beyond one matrix's dependent chain"},
        "cpu_baseline": cpu,
        "per_n": per_n,
        "parity": parity,
        "eigenvalues_only": evals,
        "leaf_cutoff": leaves,
        "uneven": uneven,
        "backward": backward,
        "spectral": spectral,
        "serving": serving,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

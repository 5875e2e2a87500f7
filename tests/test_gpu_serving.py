"""Continuous-batching server: results in a mix are bitwise equal to solo
solves, admission by slots and memory, overlap of steps on the device."""
import time

import numpy as np
import pytest

from paper_2604_27325_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2604_27325_amd as bed  # noqa: E402

DEV = torch.device("cuda:0")


def make_requests(count, seed=5000):
    arr, counts, ns = workloads.serving_trace(seed=seed, requests=count, qps=5000.0, cmax=64)
    reqs = []
    for i in range(count):
        A = torch.from_numpy(workloads.serving_matrices(seed + 1 + i, int(counts[i]), int(ns[i])))
        reqs.append(A.to(DEV))
    return reqs


def test_mixed_results_equal_solo():
    reqs = make_requests(60)
    solo = [bed.syevd(A) for A in reqs]
    torch.cuda.synchronize()
    srv = bed.Server(streams=4)
    outs, tickets = [], []
    for A in reqs:
        lam = torch.empty(A.shape[0], A.shape[1], device=DEV)
        Q = torch.empty_like(A)
        info = torch.empty(A.shape[0], dtype=torch.int32, device=DEV)
        tk = srv.submit(A, lam, Q, info)
        assert tk is not None
        outs.append((lam, Q, info))
        tickets.append(tk)
    srv.drain()
    for tk, (lam, Q, info), (lam_s, Q_s) in zip(tickets, outs, solo):
        done, lat = srv.poll(tk)
        assert done and lat > 0
        assert torch.equal(lam, lam_s) and torch.equal(Q, Q_s)
        assert int(info.abs().sum()) == 0
    srv.close()


def test_admission_by_inflight_limit_and_memory():
    reqs = make_requests(8, seed=6000)
    srv = bed.Server(streams=1, max_inflight=reqs[0].shape[0])
    lam = torch.empty(reqs[0].shape[0], reqs[0].shape[1], device=DEV)
    Q = torch.empty_like(reqs[0])
    first = srv.submit(reqs[0], lam, Q)
    assert first is not None
    # a second request cannot fit until the first completes
    lam2 = torch.empty(reqs[1].shape[0], reqs[1].shape[1], device=DEV)
    Q2 = torch.empty_like(reqs[1])
    refused = srv.submit(reqs[1], lam2, Q2)
    srv.drain()
    if refused is None:
        assert srv.submit(reqs[1], lam2, Q2) is not None  # admitted after completion
    srv.drain()
    srv.close()
    tiny = bed.Server(streams=2, mem_budget=64)
    assert tiny.submit(reqs[2], torch.empty(reqs[2].shape[:2], device=DEV),
                       torch.empty_like(reqs[2])) is None
    tiny.close()


def test_latency_and_throughput_reported():
    reqs = make_requests(200, seed=7000)
    outs = [(torch.empty(A.shape[0], A.shape[1], device=DEV), torch.empty_like(A)) for A in reqs]
    torch.cuda.synchronize()
    srv = bed.Server(streams=4)
    t0 = time.perf_counter()
    tickets = [srv.submit(A, o[0], o[1]) for A, o in zip(reqs, outs)]
    srv.drain()
    el = time.perf_counter() - t0
    lats = np.array([srv.poll(tk)[1] for tk in tickets])
    srv.close()
    mats = sum(A.shape[0] for A in reqs)
    print(f"[serving] {mats / el:.0f} matrices/s p50 {np.percentile(lats, 50):.0f} us "
          f"p99 {np.percentile(lats, 99):.0f} us", flush=True)
    assert np.all(lats > 0)

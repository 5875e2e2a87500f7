"""Deflation on the GPU, counted by the instrumented copy of the solver
(include/bed_probe.h, the same kernel code with counters): on the batch-512
workload, the matrices with a planted eigenvalue pair 1e-6 apart (relative gap
about 1e-7 to 5e-7, at the binary32 deflation tolerance 8u max(|d|, rho z^T z))
take type-2 deflations (a Givens rotation of two close poles), and the
eigenvalues of that instrumented run still match the oracle."""
import ctypes
import os

import numpy as np
import pytest

import oracle
from paper_2604_27325_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2604_27325_amd as bed  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE = os.path.join(ROOT, "paper_2604_27325_amd", "_lib", "libbed_probe.so")


@pytest.mark.parametrize("n", [32, 64])
def test_type2_deflation_fires_on_planted_pairs(n):
    bed.load_library()
    lib = ctypes.CDLL(PROBE)
    vp = ctypes.c_void_p
    lib.bed_probe_phases.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp]
    A_np, planted, _ = workloads.paper_scale(n)
    b = A_np.shape[0]
    A = torch.from_numpy(A_np).to("cuda")
    lam = torch.empty(b, n, device="cuda")
    Q = torch.empty_like(A)
    marks = torch.zeros(b * 64, dtype=torch.int64, device="cuda")
    steps = torch.zeros(b * 16, dtype=torch.int64, device="cuda")
    defl = torch.zeros(b * 2, dtype=torch.int64, device="cuda")
    threads = 128 if n <= 32 else 512
    st = lib.bed_probe_phases(0, threads, n, b, vp(A.data_ptr()), vp(lam.data_ptr()),
                              vp(Q.data_ptr()), vp(marks.data_ptr()), vp(steps.data_ptr()),
                              vp(defl.data_ptr()), vp(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    d = defl.view(b, 2).cpu().numpy()
    mask = np.zeros(b, dtype=bool)
    mask[planted] = True
    t2_planted = d[mask, 1]
    t2_other = d[~mask, 1]
    print(f"[deflation n={n}] type 1 per matrix {d[:, 0].mean():.2f}; type 2: planted "
          f"{t2_planted.mean():.3f} ({int((t2_planted > 0).sum())}/{mask.sum()} matrices), "
          f"others {t2_other.mean():.3f}", flush=True)
    assert (t2_planted > 0).mean() >= 0.5        # most planted pairs rotate
    assert t2_planted.mean() > 5 * max(t2_other.mean(), 1e-3)
    assert d[:, 0].sum() > 0                     # type 1 occurs too
    lam_o, _, _ = oracle.syevd(A_np.astype(np.float64))
    err = np.abs(lam.cpu().numpy() - lam_o).max(axis=1) / np.abs(lam_o).max(axis=1)
    assert err.max() <= 1e-5

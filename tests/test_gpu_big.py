"""Orders 64 < n <= 128 (binary32, uniform batches): one tearing step above the
n <= 64 kernels and the top merge on a 512-thread team, against the binary64
oracle under the same parity rules as n <= 64."""
import numpy as np
import pytest

import oracle
from paper_2604_27325_amd import workloads
from tests.parity import compare_batch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2604_27325_amd as bed  # noqa: E402

DEV = torch.device("cuda:0")


def check(A_np, label, vectors=True):
    A = torch.from_numpy(np.ascontiguousarray(A_np)).to(DEV)
    b, n = A_np.shape[0], A_np.shape[1]
    print(f"[{label}] batch {b} n={n} vectors={vectors}", flush=True)
    lam, Q, info = bed.syevd_packed([n] * b, A.view(-1), want_vectors=vectors)
    torch.cuda.synchronize()
    lam = lam.view(b, n).cpu().numpy()
    Q = Q.view(b, n, n).cpu().numpy() if vectors else None
    lam_o, Q_o, _ = oracle.syevd(A_np.astype(np.float64))
    worst, fails = compare_batch(A_np, lam, Q, lam_o, Q_o if vectors else None, np.float32,
                                 info=info.cpu().numpy())
    print(f"  worst {worst}", flush=True)
    assert not fails, f"{label}: {len(fails)} failing matrices, first {fails[:3]}"


@pytest.mark.parametrize("n", [65, 66, 80, 96, 97, 127, 128])
def test_gaussian_and_covariance(n):
    rng = np.random.default_rng(8000 + n)
    A = np.concatenate([workloads.gaussian_sym(rng, 8, n), workloads.covariance(rng, 8, n)])
    check(A.astype(np.float32), f"n={n}")


@pytest.mark.parametrize("n", [65, 96, 128])
def test_planted_pairs_deflate(n):
    """Planted eigenvalue pairs 1e-6 apart (type-2 deflation at the top merge
    or in the halves) and repeated eigenvalues."""
    A, idx, _ = workloads.paper_scale(n, batch=64, planted_frac=0.5)
    rng = np.random.default_rng(8100 + n)
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    w = np.repeat(np.linspace(-1.0, 1.0, n // 4 + 1), 4)[:n]  # fourfold eigenvalues
    rep = ((V * w) @ V.T).astype(np.float32)
    check(np.concatenate([A[idx][:24], rep[None]]), f"planted n={n}")


@pytest.mark.parametrize("n", [65, 100, 128])
def test_eigenvalues_only(n):
    rng = np.random.default_rng(8200 + n)
    A = np.concatenate([workloads.gaussian_sym(rng, 8, n), workloads.covariance(rng, 8, n)])
    check(A.astype(np.float32), f"eigenvalues n={n}", vectors=False)


def test_full_batch_512_n128_sampled():
    """The batch-512 n = 128 workload (the bench's shape), sampled outputs
    against the oracle."""
    A_np, _, _ = workloads.paper_scale(128)
    A = torch.from_numpy(A_np).to(DEV)
    lam, Q, info = bed.syevd(A, return_info=True)
    torch.cuda.synchronize()
    idx = np.linspace(0, 511, 16).astype(int)
    lam_o, Q_o, _ = oracle.syevd(A_np[idx].astype(np.float64))
    worst, fails = compare_batch(A_np[idx], lam.cpu().numpy()[idx], Q.cpu().numpy()[idx], lam_o,
                                 Q_o, np.float32, info=info.cpu().numpy()[idx])
    print(f"[batch 512 n=128] worst {worst}", flush=True)
    assert not fails, fails[:3]
    assert int(info.abs().sum()) == 0


def test_workspace_grows_and_results_repeat():
    """Calls of growing and shrinking size on one stream (the workspace is
    reused or grown), each bitwise equal to a fresh call."""
    rng = np.random.default_rng(8300)
    outs = []
    for n, b in ((70, 3), (128, 40), (90, 1), (128, 40)):
        A = torch.from_numpy(workloads.gaussian_sym(rng, b, n).astype(np.float32)).to(DEV)
        outs.append((A, bed.syevd(A)))
    torch.cuda.synchronize()
    l1, q1 = outs[1][1]
    l3, q3 = outs[3][1]
    assert not torch.equal(outs[1][0], outs[3][0]) or (torch.equal(l1, l3) and torch.equal(q1, q3))
    for A, (lam, Q) in outs:
        l2, q2 = bed.syevd(A)
        assert torch.equal(lam, l2) and torch.equal(Q, q2)


def test_nonfinite_input_reports_info_minus_one():
    rng = np.random.default_rng(8400)
    A_np = workloads.gaussian_sym(rng, 3, 100).astype(np.float32)
    A_np[1, 50, 7] = np.nan
    A = torch.from_numpy(A_np).to(DEV)
    lam, Q, info = bed.syevd(A, return_info=True)
    info = info.cpu().numpy()
    assert list(info) == [0, -1, 0]
    assert torch.isnan(lam[1]).all() and torch.isnan(Q[1]).all()
    assert torch.isfinite(lam[0]).all() and torch.isfinite(Q[2]).all()


def test_nonfinite_input_eigenvalues_only():
    """The binary32 reduction path (eigenvalues only) flags a NaN matrix the
    same way and leaves its neighbours intact."""
    rng = np.random.default_rng(8401)
    A_np = workloads.gaussian_sym(rng, 4, 128).astype(np.float32)
    A_np[2, 120, 3] = np.inf  # lower triangle (the only one read)
    A = torch.from_numpy(A_np).to(DEV)
    lam, _, info = bed.syevd_packed([128] * 4, A.view(-1), want_vectors=False)
    lam = lam.view(4, 128)
    info = info.cpu().numpy()
    assert list(info) == [0, 0, -1, 0]
    assert torch.isnan(lam[2]).all()
    lam_o, _, _ = oracle.syevd(A_np[[0, 1, 3]].astype(np.float64))
    err = np.abs(lam[[0, 1, 3]].cpu().numpy() - lam_o).max() / np.abs(lam_o).max()
    assert err < 1e-5, err


def test_unsupported_forms_fail_loudly():
    A = torch.zeros(2, 100, 100, dtype=torch.float64, device=DEV)
    with pytest.raises(bed.BedError) as ei:
        bed.syevd(A)
    assert ei.value.status == 2  # BED_ERR_UNSUPPORTED (binary64 above 64)
    flat = torch.zeros(100 * 100 + 10 * 10, device=DEV)
    with pytest.raises(bed.BedError) as ei:
        bed.syevd_packed([100, 10], flat)
    assert ei.value.status == 2  # mixed batch with n > 64


def test_graph_capture_and_replay():
    """After a first call on a stream (which sizes its workspace), the
    launches of an n = 100 solve (reduction, Householder product, halves, top
    merge) can be captured in a HIP graph; every replay, with eager work in
    between, gives the eager result bitwise."""
    rng = np.random.default_rng(8500)
    A = torch.from_numpy(workloads.gaussian_sym(rng, 40, 100).astype(np.float32)).to(DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ref_l, ref_q = bed.syevd(A, stream=s)  # sizes the workspace of stream s
    torch.cuda.synchronize()
    lam = torch.empty_like(ref_l)
    Q = torch.empty_like(ref_q)
    info = torch.empty(40, dtype=torch.int32, device=DEV)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bed.syevd_packed([100] * 40, A.view(-1), lam=lam.view(-1), Q=Q.view(-1), info=info,
                         stream=s)
    for rep in range(3):
        lam.fill_(-1.0)
        Q.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = (A * 2.0).sum().item()  # eager work between replays
        assert torch.equal(lam, ref_l) and torch.equal(Q, ref_q), f"replay {rep}"


def test_graph_capture_eigenvalues_only():
    """The eigenvalues-only chain (binary32 reduction, halves, top merge) of
    an odd order captured in a HIP graph: every replay equals the eager
    result bitwise."""
    rng = np.random.default_rng(8501)
    A = torch.from_numpy(workloads.gaussian_sym(rng, 24, 101).astype(np.float32)).to(DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ref, _, _ = bed.syevd_packed([101] * 24, A.view(-1), want_vectors=False, stream=s)
    torch.cuda.synchronize()
    lam = torch.empty_like(ref)
    info = torch.empty(24, dtype=torch.int32, device=DEV)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bed.syevd_packed([101] * 24, A.view(-1), lam=lam, info=info, want_vectors=False, stream=s)
    for rep in range(3):
        lam.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = (A * 2.0).sum().item()
        assert torch.equal(lam, ref), f"replay {rep}"


def test_graph_keeps_workspace_when_stream_grows():
    """A graph captured at n = 100 keeps its workspace after a larger eager
    call (n = 128, more matrices) on the capture stream has grown that
    stream's workspace: replays after the growth still equal the eager
    result bitwise, and so does the larger call."""
    rng = np.random.default_rng(8502)
    A = torch.from_numpy(workloads.gaussian_sym(rng, 16, 100).astype(np.float32)).to(DEV)
    A2 = torch.from_numpy(workloads.gaussian_sym(rng, 48, 128).astype(np.float32)).to(DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ref_l, ref_q = bed.syevd(A, stream=s)
    torch.cuda.synchronize()
    lam = torch.empty_like(ref_l)
    Q = torch.empty_like(ref_q)
    info = torch.empty(16, dtype=torch.int32, device=DEV)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bed.syevd_packed([100] * 16, A.view(-1), lam=lam.view(-1), Q=Q.view(-1), info=info,
                         stream=s)
    ref2_l, ref2_q = bed.syevd(A2)  # default stream: its own workspace
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        l2, q2 = bed.syevd(A2, stream=s)  # grows the capture stream's workspace
    torch.cuda.synchronize()
    assert torch.equal(l2, ref2_l) and torch.equal(q2, ref2_q)
    for rep in range(2):
        lam.fill_(-1.0)
        Q.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(lam, ref_l) and torch.equal(Q, ref_q), f"replay {rep}"


def test_in_place_q_over_a():
    """Q == A (in place) at n = 128: the reduction reads A before the
    Householder product is written over it; the result equals the
    out-of-place solve bitwise."""
    rng = np.random.default_rng(8600)
    A = torch.from_numpy(workloads.gaussian_sym(rng, 6, 128).astype(np.float32)).to(DEV)
    lam_r, Q_r = bed.syevd(A)
    B = A.clone()
    lam = torch.empty(6 * 128, device=DEV)
    bed.syevd_packed([128] * 6, B.view(-1), lam=lam, Q=B.view(-1))
    torch.cuda.synchronize()
    assert torch.equal(lam.view(6, 128), lam_r) and torch.equal(B, Q_r)


def test_every_order_65_to_128():
    """Every order above 64, two matrices each (one Gaussian, one covariance),
    eigenvectors and eigenvalues only: all tearing splits n1 = n2 and
    n2 = n1 + 1 with children of 32 .. 64."""
    for n in range(65, 129):
        rng = np.random.default_rng(8700 + n)
        A = np.concatenate([workloads.gaussian_sym(rng, 1, n), workloads.covariance(rng, 1, n)])
        check(A.astype(np.float32), f"n={n}")
        check(A.astype(np.float32), f"eigenvalues n={n}", vectors=False)

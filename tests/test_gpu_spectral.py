"""Spectral matrix functions on the GPU against the binary64 oracle (through the
C-ABI): the kernels alone on the GPU's own decomposition, and end to end
(decomposition + function, autograd backward) on positive definite inputs."""
import numpy as np
import pytest

import oracle
from paper_2604_27325_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2604_27325_amd as bed  # noqa: E402

DEV = torch.device("cuda:0")
FNS = [("sqrt", 0.0), ("invsqrt", 0.0), ("exp", 0.0), ("log", 0.0), ("pow", 0.7)]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def spd(seed, batch, n, dtype=np.float32):
    rng = np.random.default_rng(seed)
    return workloads.covariance(rng, batch, n, m=2 * n).astype(dtype)


@pytest.mark.parametrize("fn,p", FNS)
@pytest.mark.parametrize("n", [5, 32, 64])
def test_apply_and_backward_kernels_alone(fn, p, n):
    """Same (lambda, Q) on both sides: the kernels' arithmetic only."""
    A = spd(800 + n, 64, n)
    lam, Q = bed.syevd(torch.from_numpy(A).to(DEV))
    F = bed.spectral_apply(lam, Q, fn, p).cpu().numpy()
    rng = np.random.default_rng(900 + n)
    dF = rng.standard_normal((64, n, n)).astype(np.float32)
    dA = bed.spectral_backward(lam, Q, torch.from_numpy(dF).to(DEV), fn, p).cpu().numpy()
    l64, q64 = lam.cpu().numpy().astype(np.float64), Q.cpu().numpy().astype(np.float64)
    F_o = oracle.spectral_apply(l64, q64, fn, p)
    dA_o = oracle.spectral_backward(l64, q64, dF.astype(np.float64), fn, p)
    ef = max(rel(F[b], F_o[b]) for b in range(64))
    eb = max(rel(dA[b], dA_o[b]) for b in range(64))
    print(f"[spectral {fn} n={n}] apply {ef:.3g} backward {eb:.3g}", flush=True)
    assert ef <= 1e-5 and eb <= 2e-5


@pytest.mark.parametrize("fn,p", FNS)
def test_end_to_end_fp32_and_autograd(fn, p):
    """f(A) and its gradient through the autograd function, against the
    oracle's own decomposition (covariance inputs, well separated spectra)."""
    n = 32
    A = spd(1000, 128, n)
    At = torch.from_numpy(A).to(DEV).requires_grad_(True)
    F = bed.matrix_function(At, fn, p)
    rng = np.random.default_rng(1001)
    dF = rng.standard_normal((128, n, n)).astype(np.float32)
    (F * torch.from_numpy(dF).to(DEV)).sum().backward()
    lo, qo, _ = oracle.syevd(A.astype(np.float64))
    F_o = oracle.spectral_apply(lo, qo, fn, p)
    G_o = oracle.spectral_backward(lo, qo, dF.astype(np.float64), fn, p)
    F_g, G_g = F.detach().cpu().numpy(), At.grad.cpu().numpy()
    ef = max(rel(F_g[b], F_o[b]) for b in range(128))
    eg = max(rel(G_g[b], G_o[b]) for b in range(128))
    print(f"[matrix_function {fn}] F {ef:.3g} grad {eg:.3g}", flush=True)
    assert ef <= 1e-5 and eg <= 1e-4


def test_fp64_and_mixed_sizes():
    ns = [3, 17, 64, 40, 1]
    rng = np.random.default_rng(1100)
    mats = [workloads.covariance(rng, 1, n, m=2 * n)[0] for n in ns]
    _, flat = workloads.pack(mats)
    lam, Q, _ = bed.syevd_packed(ns, torch.from_numpy(flat).to(DEV))
    dF = rng.standard_normal(flat.shape[0])
    F = bed.spectral_apply(lam, Q, "sqrt", n_list=ns).cpu().numpy()
    dA = bed.spectral_backward(lam, Q, torch.from_numpy(dF).to(DEV), "sqrt",
                               n_list=ns).cpu().numpy()
    lh, qh = lam.cpu().numpy(), Q.cpu().numpy()
    oA = oL = 0
    for n, M in zip(ns, mats):
        q = qh[oA:oA + n * n].reshape(n, n)
        l = lh[oL:oL + n]
        F_o = oracle.spectral_apply(l, q, "sqrt")
        d_o = oracle.spectral_backward(l, q, dF[oA:oA + n * n].reshape(n, n), "sqrt")
        assert rel(F[oA:oA + n * n].reshape(n, n), F_o) <= 1e-13
        assert rel(dA[oA:oA + n * n].reshape(n, n), d_o) <= 1e-12
        assert rel(F_o @ F_o, M) <= 1e-12  # the decomposition itself is right
        oA += n * n
        oL += n

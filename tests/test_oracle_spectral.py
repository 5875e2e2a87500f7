"""Pins of the oracle's spectral matrix functions (CPU): closed forms and
identities (sqrt(A)^2 = A, A^{-1/2} A A^{-1/2} = I, A^2, diagonal inputs),
independent library algorithms for special cases (scipy's Pade expm, Schur
sqrtm and logm), and binary64 finite differences for the backward."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_2604_27325_amd import workloads

FNS = [("sqrt", 0.0), ("invsqrt", 0.0), ("exp", 0.0), ("log", 0.0), ("pow", 0.7), ("pow", 2.0)]


def spd(seed, n, batch=4):
    rng = np.random.default_rng(seed)
    return workloads.covariance(rng, batch, n, m=2 * n)


def apply_oracle(A, fn, p=0.0):
    lam, Q, _ = oracle.syevd(A)
    return oracle.spectral_apply(lam, Q, fn, p)


@pytest.mark.parametrize("n", [1, 2, 5, 16, 33])
def test_closed_forms(n):
    A = spd(100 + n, n)
    I = np.eye(n)
    S = apply_oracle(A, "sqrt")
    assert np.abs(S @ S - A).max() <= 1e-12 * np.abs(A).max()
    W = apply_oracle(A, "invsqrt")
    assert np.abs(W @ A @ W - I).max() <= 1e-10
    P2 = apply_oracle(A, "pow", 2.0)
    assert np.abs(P2 - A @ A).max() <= 1e-12 * np.abs(A @ A).max()
    assert np.abs(apply_oracle(A, "pow", 0.5) - S).max() <= 1e-12 * np.abs(S).max()
    d = np.random.default_rng(n).uniform(0.5, 2.0, size=n)
    D = np.diag(d)[None]
    assert np.allclose(apply_oracle(D, "exp")[0], np.diag(np.exp(d)), rtol=1e-14, atol=0)
    assert np.allclose(apply_oracle(D, "log")[0], np.diag(np.log(d)), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("n", [3, 12, 32])
def test_against_library_algorithms(n):
    A = spd(200 + n, n, batch=3)
    for b in range(3):
        lam, Q, _ = oracle.syevd(A[b])
        for fn, ref in (("exp", sla.expm(A[b])), ("sqrt", sla.sqrtm(A[b]).real),
                        ("log", sla.logm(A[b]).real)):
            F = oracle.spectral_apply(lam, Q, fn)
            assert np.abs(F - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max()), fn


@pytest.mark.parametrize("fn,p", FNS)
@pytest.mark.parametrize("n", [4, 16])
def test_backward_matches_finite_differences(fn, p, n):
    rng = np.random.default_rng(300 + n)
    A = spd(300 + n, n, batch=1)[0]
    dF = rng.standard_normal((n, n))
    lam, Q, _ = oracle.syevd(A)
    G = oracle.spectral_backward(lam, Q, dF, fn, p)
    assert np.allclose(G, G.T, atol=1e-12 * np.abs(G).max())
    h = 1e-6
    for _ in range(4):
        E = rng.standard_normal((n, n))
        E = 0.5 * (E + E.T)
        E /= np.linalg.norm(E)
        lp, Qp, _ = oracle.syevd(A + h * E)
        lm, Qm, _ = oracle.syevd(A - h * E)
        fd = (np.sum(dF * oracle.spectral_apply(lp, Qp, fn, p)) -
              np.sum(dF * oracle.spectral_apply(lm, Qm, fn, p))) / (2 * h)
        an = np.sum(G * E)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_backward_equal_eigenvalues_use_the_derivative():
    """A = c I (all eigenvalues equal): dA = f'(c) sym(dF)."""
    n, c = 6, 1.7
    rng = np.random.default_rng(7)
    dF = rng.standard_normal((n, n))
    lam, Q, _ = oracle.syevd(c * np.eye(n))
    G = oracle.spectral_backward(lam, Q, dF, "sqrt")
    assert np.allclose(G, 0.5 / np.sqrt(c) * 0.5 * (dF + dF.T), atol=1e-14)

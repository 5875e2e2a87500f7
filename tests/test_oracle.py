"""Pins for the binary64 oracle: each check compares the oracle with something
other than itself (closed forms, special matrices with known spectra, the
cyclic-Jacobi brute force, LAPACK, exact identities of the note)."""
import os

import numpy as np
import pytest

import oracle
from tests.jacobi_ref import jacobi_eigh
from paper_2604_27325_amd import workloads

U = 2.0 ** -53
HERE = os.path.dirname(os.path.abspath(__file__))


def angle(u, v):
    """sin of the angle between two vectors, sign-invariant, FP64 renormalized
    (never sqrt(1 - c^2))."""
    u = u / np.linalg.norm(u)
    v = v / np.linalg.norm(v)
    return np.linalg.norm(u - (v @ u) * v)


def check_decomp(A, lam, Q, tol):
    A = np.tril(A) + np.tril(A, -1).T
    n = A.shape[0]
    nrm = max(np.linalg.norm(A), 1e-300)
    assert np.all(np.diff(lam) >= 0)
    assert np.linalg.norm(A @ Q - Q * lam) / nrm <= tol
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= tol
    # sign canonical: largest-|.| entry of each column positive
    idx = np.argmax(np.abs(Q), axis=0)
    assert np.all(Q[idx, np.arange(n)] > 0)


# ---------------------------------------------------------------- closed forms
def test_2x2_closed_form():
    rng = np.random.default_rng(11)
    for _ in range(200):
        a, b, c = rng.standard_normal(3) * 10.0 ** rng.integers(-3, 3, size=3)
        A = np.array([[a, 0.0], [b, c]])  # lower triangle only
        lam, Q, info = oracle.syevd(A)
        mid, rad = 0.5 * (a + c), np.hypot(0.5 * (a - c), b)
        exp = np.array([mid - rad, mid + rad])
        assert info == 0
        np.testing.assert_allclose(lam, exp, rtol=0, atol=8 * U * (abs(mid) + rad))
        for j in range(2):  # (b, lam - a) spans the eigenvector when b != 0
            if abs(b) > 1e-8 * rad:
                v = np.array([b, exp[j] - a]) if abs(exp[j] - a) >= abs(exp[j] - c) else \
                    np.array([exp[j] - c, b])
                assert angle(Q[:, j], v) < 1e-12


def _smith3(A):
    """Smith (1961) trigonometric eigenvalues of a symmetric 3x3 matrix."""
    q = np.trace(A) / 3.0
    p1 = A[0, 1] ** 2 + A[0, 2] ** 2 + A[1, 2] ** 2
    p2 = (A[0, 0] - q) ** 2 + (A[1, 1] - q) ** 2 + (A[2, 2] - q) ** 2 + 2 * p1
    p = np.sqrt(p2 / 6.0)
    B = (A - q * np.eye(3)) / p
    r = np.clip(np.linalg.det(B) / 2.0, -1.0, 1.0)
    phi = np.arccos(r) / 3.0
    l1 = q + 2 * p * np.cos(phi)
    l3 = q + 2 * p * np.cos(phi + 2 * np.pi / 3)
    return np.sort([l3, 3 * q - l1 - l3, l1])


def test_3x3_smith():
    rng = np.random.default_rng(12)
    for _ in range(200):
        A = workloads.gaussian_sym(rng, 1, 3)[0]
        lam, Q, info = oracle.syevd(A)
        np.testing.assert_allclose(lam, _smith3(A), rtol=0, atol=1e-12 * np.abs(lam).max())
        check_decomp(A, lam, Q, 30 * U * 3)


@pytest.mark.parametrize("n", [3, 4, 5, 8, 13, 16, 31, 48, 64])
@pytest.mark.parametrize("bsign", [1.0, -1.0])
def test_toeplitz_tridiagonal(n, bsign):
    a0, b0 = 0.7, 0.45 * bsign
    k = np.arange(1, n + 1)
    exp = np.sort(a0 + 2 * b0 * np.cos(k * np.pi / (n + 1)))
    lam, Q, capped = oracle.tridiag_eig(np.full(n, a0), np.full(n - 1, b0))
    assert capped == 0
    np.testing.assert_allclose(lam, exp, rtol=0, atol=20 * n * U)
    T = np.diag(np.full(n, a0)) + np.diag(np.full(n - 1, b0), 1) + np.diag(np.full(n - 1, b0), -1)
    lam2, Q2, info = oracle.syevd(T)
    np.testing.assert_allclose(lam2, exp, rtol=0, atol=20 * n * U)
    for j in range(n):  # v_k(i) ∝ sin(i k pi/(n+1)) for eigenvalue a + 2b cos(k pi/(n+1))
        kk = np.argmin(np.abs(a0 + 2 * b0 * np.cos(k * np.pi / (n + 1)) - exp[j]))
        v = np.sin(np.arange(1, n + 1) * k[kk] * np.pi / (n + 1))
        assert angle(Q[:, j], v) < 1e-11
        assert angle(Q2[:, j], v) < 1e-11


@pytest.mark.parametrize("n", [2, 5, 16, 33, 64])
def test_rank_one(n):
    rng = np.random.default_rng(13 + n)
    u = rng.standard_normal(n)
    A = np.outer(u, u)
    st = oracle.Stats()
    lam, Q, info = oracle.syevd(A, stats=st)
    s = u @ u
    np.testing.assert_allclose(lam[-1], s, rtol=20 * n * U)
    assert np.max(np.abs(lam[:-1])) <= 20 * n * U * s
    assert angle(Q[:, -1], u) < 1e-13
    check_decomp(A, lam, Q, 20 * n * U)


@pytest.mark.parametrize("n", [1, 2, 7, 64])
def test_diagonal_exact(n):
    rng = np.random.default_rng(14)
    d = rng.permutation(np.arange(n, dtype=np.float64) - n / 3)
    lam, Q, info = oracle.syevd(np.diag(d))
    assert np.array_equal(lam, np.sort(d))
    P = np.zeros((n, n))
    P[np.argsort(d, kind="stable"), np.arange(n)] = 1.0
    assert np.array_equal(Q, P)


@pytest.mark.parametrize("n", [3, 16, 64])
def test_scaled_identity(n):
    lam, Q, info = oracle.syevd(2.5 * np.eye(n))
    assert np.all(lam == 2.5)
    check_decomp(2.5 * np.eye(n), lam, Q, 10 * n * U)


def test_wilkinson_w21():
    n = 21
    T = np.diag(np.abs(np.arange(n) - 10.0)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    st = oracle.Stats()
    lam, Q, info = oracle.syevd(T, stats=st)
    wj, Vj = jacobi_eigh(T)
    np.testing.assert_allclose(lam, wj, rtol=0, atol=1e-13 * 11)
    check_decomp(T, lam, Q, 10 * n * U)
    # the top pair is nearly degenerate: compare the 2-D invariant subspace
    P = Q[:, -2:] @ Q[:, -2:].T
    Pj = Vj[:, -2:] @ Vj[:, -2:].T
    assert np.linalg.norm(P - Pj, 2) < 1e-10


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 8, 11, 16, 24, 33, 48, 64, 65, 97, 128])
def test_vs_cyclic_jacobi(n):
    rng = np.random.default_rng(100 + n)
    for kind in ("gauss", "cov"):
        A = (workloads.gaussian_sym(rng, 1, n) if kind == "gauss" else
             workloads.covariance(rng, 1, n))[0]
        lam, Q, info = oracle.syevd(A)
        wj, Vj = jacobi_eigh(A)
        nrm = np.abs(wj).max()
        assert info == 0
        np.testing.assert_allclose(lam, wj, rtol=0, atol=1e-13 * nrm)
        gaps = np.full(n, np.inf)
        if n > 1:
            g = np.diff(wj)
            gaps = np.minimum(np.concatenate([[np.inf], g]), np.concatenate([g, [np.inf]]))
        gaps = np.minimum(gaps, nrm)
        for j in range(n):
            if gaps[j] > 1e-6 * nrm:
                assert angle(Q[:, j], Vj[:, j]) * gaps[j] / nrm < 1e-13
        check_decomp(A, lam, Q, 10 * max(n, 1) * U * 10)


def test_vs_lapack_batches():
    A = workloads.plain_fp64()
    lam, Q, info = oracle.syevd(A)
    assert np.all(info == 0)
    w = np.linalg.eigvalsh(A)
    np.testing.assert_allclose(lam, w, rtol=0, atol=1e-13 * np.abs(w).max())
    for b in range(A.shape[0]):
        check_decomp(A[b], lam[b], Q[b], 10 * 16 * U * 10)
    Ac, _, _ = workloads.paper_scale(32, batch=16)
    lam, Q, info = oracle.syevd(Ac.astype(np.float64))
    w = np.linalg.eigvalsh(Ac.astype(np.float64))
    np.testing.assert_allclose(lam, w, rtol=0, atol=1e-13 * np.abs(w).max())


def test_invariants_trace_frobenius():
    rng = np.random.default_rng(21)
    for n in (8, 37, 64):
        A = workloads.gaussian_sym(rng, 1, n)[0]
        lam, Q, info = oracle.syevd(A)
        assert abs(lam.sum() - np.trace(A)) <= 50 * n * U * np.abs(A).sum()
        assert abs(np.sum(lam ** 2) - np.sum(A * A)) <= 50 * n * U * np.sum(A * A)


def test_packed_mixed_sizes_and_nan():
    rng = np.random.default_rng(22)
    mats = [workloads.gaussian_sym(rng, 1, n)[0] for n in (5, 1, 64, 2, 17)]
    mats[3][1, 0] = np.nan
    ns, flat = workloads.pack(mats)
    lam, Q, info = oracle.syevd_packed(ns, flat)
    assert list(info) == [0, 0, 0, -1, 0]
    offA = offL = 0
    for M, n, inf in zip(mats, ns, info):
        l1, Q1 = lam[offL:offL + n], Q[offA:offA + n * n].reshape(n, n)
        if inf == -1:
            assert np.all(np.isnan(l1)) and np.all(np.isnan(Q1))
        else:
            l2, Q2, _ = oracle.syevd(M)
            assert np.array_equal(l1, l2) and np.array_equal(Q1, Q2)
        offA += n * n
        offL += n


# ---------------------------------------------------------------- Householder
@pytest.mark.parametrize("n", [1, 2, 3, 6, 16, 64])
def test_householder_factorization(n):
    rng = np.random.default_rng(30 + n)
    A = workloads.gaussian_sym(rng, 1, n)[0]
    a, b, V, tau = oracle.tridiag(A)
    QH = np.eye(n)
    for k in range(n - 2):
        QH = QH @ (np.eye(n) - tau[k] * np.outer(V[:, k], V[:, k]))
        assert V[k + 1, k] == 1.0 and np.all(V[: k + 1, k] == 0.0)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    assert np.linalg.norm(QH.T @ QH - np.eye(n)) <= 10 * n * U * 10
    assert np.linalg.norm(QH @ T @ QH.T - A) <= 10 * n * U * np.linalg.norm(A) * 10
    np.testing.assert_allclose(np.linalg.eigvalsh(T), np.linalg.eigvalsh(A), atol=1e-13 * n)


def test_householder_tridiagonal_input_unchanged():
    rng = np.random.default_rng(31)
    n = 12
    a0, b0 = rng.standard_normal(n), rng.standard_normal(n - 1)
    T = np.diag(a0) + np.diag(b0, 1) + np.diag(b0, -1)
    a, b, V, tau = oracle.tridiag(T)
    assert np.array_equal(a, a0) and np.array_equal(np.abs(b), np.abs(b0))
    assert np.all(tau == 0.0)


# ---------------------------------------------------------------- tearing (golden)
def _golden(name):
    vals = {}
    with open(os.path.join(HERE, "golden", name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            vals[key] = np.array([float(x) for x in rest])
    return vals


def test_tearing_identity_eq2_exact():
    g = _golden("tear_eq2_4x4.txt")
    T = g["T"].reshape(4, 4)
    T1, T2, v, beta = g["T1hat"].reshape(2, 2), g["T2hat"].reshape(2, 2), g["v"], g["beta"][0]
    blk = np.zeros((4, 4))
    blk[:2, :2], blk[2:, 2:] = T1, T2
    assert np.array_equal(blk + abs(beta) * np.outer(v, v), T)  # Eq. (2), bitwise
    # Eq. (4)-(5) with rows (not columns) of Q1, Q2: D + |beta| z z^T has T's spectrum
    d1, Q1 = np.linalg.eigh(T1)
    d2, Q2 = np.linalg.eigh(T2)
    z = np.concatenate([np.sign(beta) * Q1[-1, :], Q2[0, :]])
    M = np.diag(np.concatenate([d1, d2])) + abs(beta) * np.outer(z, z)
    np.testing.assert_allclose(np.linalg.eigvalsh(M), np.linalg.eigvalsh(T), atol=1e-14)
    assert abs(z @ z - 2.0) < 1e-15
    # the oracle's D&C on this T (one tear at the middle, two 2x2 leaves)
    lam, Q, capped = oracle.tridiag_eig(np.diag(T), np.diag(T, -1))
    np.testing.assert_allclose(lam, np.linalg.eigvalsh(T), atol=1e-14)


# ---------------------------------------------------------------- secular solver
def _random_secular(rng, k):
    d = np.sort(rng.standard_normal(k))
    while k > 1 and np.min(np.diff(d)) < 1e-3:
        d = np.sort(rng.standard_normal(k))
    z = rng.standard_normal(k)
    z *= np.sqrt(2.0) / np.linalg.norm(z)
    return d, z, abs(rng.standard_normal()) + 0.05


@pytest.mark.parametrize("k", [1, 2, 3, 5, 16, 33, 64])
def test_secular_interlacing_trace_lapack(k):
    rng = np.random.default_rng(40 + k)
    for _ in range(5):
        d, z, rho = _random_secular(rng, k)
        lam, origin, tau, iters, capped = oracle.secular(d, z, rho)
        assert capped == 0
        upper = np.concatenate([d[1:], [d[-1] + rho * (z @ z)]])
        assert np.all(lam > d) and np.all(lam < upper) or k == 1
        assert np.all(lam >= d) and np.all(lam <= upper)
        assert abs(lam.sum() - (d.sum() + rho * (z @ z))) <= 1e-12 * (np.abs(d).sum() + rho * 2)
        w = np.linalg.eigvalsh(np.diag(d) + rho * np.outer(z, z))
        np.testing.assert_allclose(lam, w, rtol=0, atol=1e-13 * np.abs(w).max())
        assert np.all((origin == np.arange(k)) | (origin == np.arange(k) + 1))


def test_secular_k1_k2_closed_forms():
    rng = np.random.default_rng(50)
    for _ in range(100):
        d0, z0, rho = rng.standard_normal(), rng.standard_normal(), abs(rng.standard_normal())
        lam, *_ = oracle.secular([d0], [z0], rho)
        np.testing.assert_allclose(lam[0], d0 + rho * z0 * z0, rtol=0,
                                   atol=32 * U * (abs(d0) + rho * z0 * z0))
        d = np.sort(rng.standard_normal(2))
        z = rng.standard_normal(2)
        lam, *_ = oracle.secular(d, z, rho)
        a11, a22, a12 = d[0] + rho * z[0] ** 2, d[1] + rho * z[1] ** 2, rho * z[0] * z[1]
        mid, rad = 0.5 * (a11 + a22), np.hypot(0.5 * (a11 - a22), a12)
        np.testing.assert_allclose(lam, [mid - rad, mid + rad], rtol=0,
                                   atol=1e-14 * (abs(mid) + rad))


def test_secular_residual_and_shape():
    """f(lam_j) vanishes and f is increasing between poles (the curve shape of
    the note's secular-equation figure)."""
    rng = np.random.default_rng(51)
    d, z, rho = _random_secular(rng, 20)
    lam, origin, tau, iters, capped = oracle.secular(d, z, rho)
    for j in range(20):
        delta = (d - d[origin[j]]) - tau[j]
        f = 1.0 + rho * np.sum(z * z / delta)
        assert abs(f) <= 1e-12 * (1 + rho * np.sum(np.abs(z * z / delta)))
    hs = np.linspace(d[3] + 1e-9, d[4] - 1e-9, 200)
    fs = [1 + rho * np.sum(z * z / (d - h)) for h in hs]
    assert np.all(np.diff(fs) > 0)


def test_secular_frobenius_bound_used_and_safe():
    rng = np.random.default_rng(52)
    d, z, rho = _random_secular(rng, 10)
    w = np.linalg.eigvalsh(np.diag(d) + rho * np.outer(z, z))
    fro = np.sqrt(np.sum(w ** 2))
    lam1, *_ = oracle.secular(d, z, rho, ub=fro - d[-1])
    lam2, *_ = oracle.secular(d, z, rho, ub=0.0)
    lam3, *_ = oracle.secular(d, z, rho, ub=1e-3 * (w[-1] - d[-1]))  # invalid bound: rejected
    for lam in (lam1, lam2, lam3):
        np.testing.assert_allclose(lam, w, rtol=0, atol=1e-13 * np.abs(w).max())


# ---------------------------------------------------------------- Loewner / merge
def test_lowner_recovers_z():
    rng = np.random.default_rng(60)
    for k in (2, 7, 30, 64):
        d, z, rho = _random_secular(rng, k)
        lam, origin, tau, iters, capped = oracle.secular(d, z, rho)
        zh = oracle.lowner(d, z, rho, origin, tau)
        np.testing.assert_allclose(zh, z, rtol=1e-10)


@pytest.mark.parametrize("m", [3, 8, 31, 64])
def test_rank1_eig_orthogonal_and_exact(m):
    rng = np.random.default_rng(70 + m)
    d = rng.standard_normal(m)
    z = rng.standard_normal(m)
    rho = 0.8
    lam, Uv, capped = oracle.rank1_eig(d, z, rho)
    M = np.diag(d) + rho * np.outer(z, z)
    np.testing.assert_allclose(lam, np.linalg.eigvalsh(M), atol=1e-13 * np.abs(lam).max())
    assert np.linalg.norm(Uv.T @ Uv - np.eye(m)) < 50 * m * U
    assert np.linalg.norm(M @ Uv - Uv * lam) < 50 * m * U * np.linalg.norm(M)


def test_rank1_eig_deflation_paths():
    rng = np.random.default_rng(71)
    m = 12
    d = np.sort(rng.standard_normal(m))
    d[5] = d[4]            # equal poles -> type 2 rotation
    d[9] = d[8] + 1e-17    # numerically equal -> type 2
    z = rng.standard_normal(m)
    z[2] = 0.0             # zero weight -> type 1
    z[7] = 1e-18
    st = oracle.Stats()
    lam, Uv, capped = oracle.rank1_eig(d, z, 0.6, stats=st)
    assert st.defl_type1 >= 2 and st.defl_type2 >= 2
    M = np.diag(d) + 0.6 * np.outer(z, z)
    np.testing.assert_allclose(lam, np.linalg.eigvalsh(M), atol=1e-14 * np.abs(lam).max() * 10)
    assert np.linalg.norm(Uv.T @ Uv - np.eye(m)) < 50 * m * U
    assert np.linalg.norm(M @ Uv - Uv * lam) < 50 * m * U * np.linalg.norm(M)


def test_deflate_rotation_is_exact_similarity():
    rng = np.random.default_rng(72)
    m = 9
    d = np.sort(rng.standard_normal(m))
    d[3] = d[2] + 1e-18
    d[6] = d[5]
    z = rng.standard_normal(m)
    z[0] = 1e-19
    rho = 0.7
    d2, z2, G, flag, tol = oracle.deflate(d, z, rho)
    assert flag[0] and flag.sum() >= 3
    assert np.linalg.norm(G.T @ G - np.eye(m)) < 10 * U * m
    M = np.diag(d) + rho * np.outer(z, z)
    M2 = np.diag(d2) + rho * np.outer(z2, z2)
    R = G.T @ M @ G - M2  # only the dropped couplings remain, each <= tol
    assert np.max(np.abs(R)) <= tol + 50 * U * np.abs(M).max()
    assert np.all(z2[flag] == 0.0)
    for i in np.flatnonzero(flag):  # deflated pair is an eigenpair of M2 up to tol
        e = np.zeros(m)
        e[i] = 1.0
        assert np.linalg.norm(M2 @ e - d2[i] * e) <= tol


# ---------------------------------------------------------------- backward
def _aligned_loss(A, Q0, dlam, dQ):
    lam, Q, _ = oracle.syevd(A)
    Q = Q * np.sign(np.sum(Q * Q0, axis=0))  # align eigenvector signs
    return lam @ dlam + np.sum(Q * dQ)


@pytest.mark.parametrize("n", [4, 8, 32])
def test_backward_vs_finite_differences(n):
    rng = np.random.default_rng(80 + n)
    for _ in range(3):
        while True:
            X = rng.standard_normal((2 * n, n))
            A = X.T @ X / (2 * n)
            if np.min(np.diff(np.linalg.eigvalsh(A))) > 1e-3:
                break
        lam, Q, _ = oracle.syevd(A)
        dlam, dQ = rng.standard_normal(n), rng.standard_normal((n, n))
        dA = oracle.syevd_backward(lam, Q, dlam, dQ)
        assert np.allclose(dA, dA.T, atol=1e-14 * np.abs(dA).max())
        for _ in range(4):
            E = rng.standard_normal((n, n))
            E = E + E.T
            E /= np.linalg.norm(E)
            h = 1e-6
            fd = (_aligned_loss(A + h * E, Q, dlam, dQ) - _aligned_loss(A - h * E, Q, dlam, dQ)) / (2 * h)
            an = np.sum(dA * E)
            assert abs(fd - an) <= 1e-5 * max(abs(an), np.linalg.norm(dA))


def test_backward_eigenvalue_only_and_guard():
    rng = np.random.default_rng(90)
    n = 6
    A = workloads.gaussian_sym(rng, 1, n)[0]
    lam, Q, _ = oracle.syevd(A)
    dlam = rng.standard_normal(n)
    dA = oracle.syevd_backward(lam, Q, dlam, None)
    np.testing.assert_allclose(dA, (Q * dlam) @ Q.T, atol=1e-14)  # d lam_i/dA = q_i q_i^T
    # degenerate spectrum: the guard zeroes every coupling, only diag(dlam) survives
    lam_d = np.full(n, 1.5)
    dA = oracle.syevd_backward(lam_d, Q, dlam, rng.standard_normal((n, n)))
    np.testing.assert_allclose(dA, (Q * dlam) @ Q.T, atol=1e-14)

"""Cyclic Jacobi eigensolver (Golub & Van Loan Alg. 8.5.3): an independent
brute-force checker for the oracle.  Shares nothing with the oracle beyond the
textbook 2x2 symmetric Schur step, which it implements on its own."""
import numpy as np


def _schur2(app, apq, aqq):
    if apq == 0.0 or abs(apq) < 1e-300 * max(abs(aqq - app), 1.0):
        return 1.0, 0.0
    th = (aqq - app) / (2.0 * apq)
    if abs(th) > 1e150:
        return 1.0, 0.5 / th
    t = (1.0 if th >= 0 else -1.0) / (abs(th) + np.hypot(1.0, th))
    c = 1.0 / np.hypot(1.0, t)
    return c, t * c


def jacobi_eigh(A, tol=1e-15, max_sweeps=60):
    """Returns (ascending eigenvalues, eigenvector columns) of symmetric A."""
    A = np.array(A, dtype=np.float64)
    A = np.tril(A) + np.tril(A, -1).T
    n = A.shape[0]
    V = np.eye(n)
    fro = np.linalg.norm(A)
    for _ in range(max_sweeps):
        off = np.sqrt(2.0 * np.sum(np.tril(A, -1) ** 2))
        if off <= tol * fro:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                c, s = _schur2(A[p, p], A[p, q], A[q, q])
                if s == 0.0:
                    continue
                Ap, Aq = A[:, p].copy(), A[:, q].copy()
                A[:, p], A[:, q] = c * Ap - s * Aq, s * Ap + c * Aq
                Ap, Aq = A[p, :].copy(), A[q, :].copy()
                A[p, :], A[q, :] = c * Ap - s * Aq, s * Ap + c * Aq
                Vp, Vq = V[:, p].copy(), V[:, q].copy()
                V[:, p], V[:, q] = c * Vp - s * Vq, s * Vp + c * Vq
    w = np.diag(A).copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]

"""Seeded synthetic workloads (inputs only; none of the solver's arithmetic).

The note measures on unspecified random matrices: 4x4 matrices over batch
sizes and batch 512 over dimensions (Fig. 1, Sec. 3.1), larger matrices at large
batch (Fig. 4) and error against dimension (Fig. 5).  The generators below
define those inputs concretely.  All randomness is numpy PCG64 from a fixed seed,
drawn in binary64 and rounded to the working dtype last.  numpy/LAPACK is used
only to *construct* matrices with a prescribed spectrum; it never produces an
expected value.

Shared by the tests, the benchmark and the oracle checks; imports nothing from
the solver or the oracle.
"""
import numpy as np

__all__ = [
    "gaussian_sym", "covariance", "plain_fp64", "paper_scale", "uneven",
    "differentiation", "serving_trace", "serving_matrices", "pack",
]


def gaussian_sym(rng, batch, n):
    """(G + G^T)/2 with G_ij ~ N(0, 1)."""
    G = rng.standard_normal((batch, n, n))
    return 0.5 * (G + np.swapaxes(G, 1, 2))


def covariance(rng, batch, n, m=None):
    """X^T X / m with X in R^{m x n}, X_ij ~ N(0, 1), m = 4n by default."""
    m = 4 * n if m is None else m
    X = rng.standard_normal((batch, m, n))
    return np.einsum("bki,bkj->bij", X, X) / m


def plain_fp64(seed=1001, batch=64, n=16):
    """Plain method, CPU-checkable: batch of Gaussian symmetric FP64 matrices."""
    rng = np.random.default_rng(seed)
    return gaussian_sym(rng, batch, n)


def paper_scale(n, seed=None, batch=512, planted_frac=0.1, planted_gap=1e-6):
    """Batch-512 FP32 workload at dimension n (the batch-512 dimension sweep).

    The first half are Gaussian symmetric, the second half covariance matrices
    X^T X/(4n).  A random 10% of the matrices get one planted eigenvalue pair:
    their binary64 eigendecomposition V diag(w) V^T has w[k+1] := w[k] + gap for
    a random k, the matrix is reassembled, symmetrized and rounded to FP32.
    Returns (A float32 (batch, n, n), planted index array, planted k array).
    """
    seed = {32: 2032, 48: 2048, 64: 2064}.get(n, 2000 + n) if seed is None else seed
    rng = np.random.default_rng(seed)
    half = batch // 2
    A = np.concatenate([gaussian_sym(rng, half, n), covariance(rng, batch - half, n)])
    n_plant = int(round(planted_frac * batch))
    idx = np.sort(rng.choice(batch, size=n_plant, replace=False))
    ks = rng.integers(0, n - 1, size=n_plant)
    for i, k in zip(idx, ks):
        w, V = np.linalg.eigh(A[i])
        w[k + 1] = w[k] + planted_gap
        B = (V * w) @ V.T
        A[i] = 0.5 * (B + B.T)
    return A.astype(np.float32), idx, ks


def uneven(seed=3000, batch=4096, nmin=4, nmax=64):
    """Uneven batch: n_b ~ U{nmin..nmax}; A = V diag(sort(10^U(-4,0))) V^T with V
    the eigenvectors of a covariance matrix X^T X/(4n).  Returns (n array int32,
    list of float32 matrices)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=batch).astype(np.int32)
    mats = []
    for n in ns:
        X = rng.standard_normal((4 * n, n))
        _, V = np.linalg.eigh(X.T @ X / (4 * n))
        lam = np.sort(10.0 ** rng.uniform(-4.0, 0.0, size=n))
        B = (V * lam) @ V.T
        mats.append((0.5 * (B + B.T)).astype(np.float32))
    return ns, mats


def differentiation(seed=4000, batch=1024, n=32, m=64, min_gap=1e-3):
    """FP32 covariance matrices X^T X/m (X m x n) with every binary64 eigengap
    >= min_gap (rejection resampling), plus upstream dlam, dQ ~ N(0,1) from
    seed+1.  Returns (A, dlam, dQ, rejected_count)."""
    rng = np.random.default_rng(seed)
    out, rejected = [], 0
    while len(out) < batch:
        X = rng.standard_normal((m, n))
        A = (X.T @ X / m).astype(np.float32)
        w = np.linalg.eigvalsh(A.astype(np.float64))
        if np.min(np.diff(w)) < min_gap:
            rejected += 1
            continue
        out.append(A)
    A = np.stack(out)
    rng2 = np.random.default_rng(seed + 1)
    dlam = rng2.standard_normal((batch, n)).astype(np.float32)
    dQ = rng2.standard_normal((batch, n, n)).astype(np.float32)
    return A, dlam, dQ, rejected


def serving_trace(seed=5000, requests=20000, qps=1000.0, cmin=1, cmax=256,
                  sizes=(8, 16, 24, 32, 40, 48, 56, 64)):
    """Poisson request stream: arrival times (s), matrix counts, one n each."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    counts = rng.integers(cmin, cmax + 1, size=requests).astype(np.int32)
    ns = rng.choice(np.asarray(sizes, dtype=np.int32), size=requests)
    return arrivals, counts, ns


def serving_matrices(seed, count, n):
    """Gaussian symmetric FP32 matrices of one serving request."""
    rng = np.random.default_rng(seed)
    return gaussian_sym(rng, count, n).astype(np.float32)


def pack(mats):
    """Packed batch-major layout: concatenated row-major matrices."""
    ns = np.asarray([m.shape[0] for m in mats], dtype=np.int32)
    flat = np.concatenate([np.ascontiguousarray(m).ravel() for m in mats]) if mats else \
        np.zeros(0, dtype=np.float32)
    return ns, flat

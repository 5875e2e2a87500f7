"""GPU-vs-oracle comparison rules for eigendecompositions.

Eigenvalues are compared in sorted order against the binary64 oracle run on
the same (working-precision) input.  Eigenvectors are compared by the angle
  theta_i = || u_i - (v_i^T u_i) v_i ||_2 ,
with u_i the GPU vector renormalized in binary64 and v_i the oracle vector
(never via sqrt(1 - c^2), which loses everything for FP32 columns).  Individual
vectors are only determined up to u * ||A|| / gap, so:
  R1  max |lam_gpu - lam_orc| <= tol_lam * ||A||_2
  R3  theta_i <= 1e-4 where relgap_i >= sep (well separated);
      theta_i * relgap_i <= tol_gap elsewhere outside clusters
  R4  clusters (relgap < clus): ||(I - V_c V_c^T) U_c||_2 <= tol_gap / relgap(cluster, rest)
  R5  ||A Q - Q Lam||_F / ||A||_F <= tol_res, ||Q^T Q - I||_F <= tol_res
plus the sign convention (largest-|.| entry of each column positive).
"""
import numpy as np

TOL = {
    np.float32: dict(lam=1e-5, sep=1e-2, clus=1e-6, gap=1e-6, res=1e-5, theta=1e-4),
    np.float64: dict(lam=1e-12, sep=1e-6, clus=1e-12, gap=1e-12, res=1e-13, theta=1e-4),
}


def _sym(A):
    A = np.asarray(A, dtype=np.float64)
    return np.tril(A) + np.tril(A, -1).T


def relgaps(lam, nrm):
    n = lam.shape[0]
    if n == 1:
        return np.array([np.inf])
    g = np.diff(lam)
    left = np.concatenate([[np.inf], g])
    right = np.concatenate([g, [np.inf]])
    return np.minimum(left, right) / max(nrm, 1e-300)


def compare_one(A, lam_g, Q_g, lam_o, Q_o, dtype, check_sign=True):
    """Returns a dict of measured quantities and a list of violated rules."""
    t = TOL[dtype]
    A = _sym(A)
    n = A.shape[0]
    lam_g = np.asarray(lam_g, dtype=np.float64)
    Q_g = None if Q_g is None else np.asarray(Q_g, dtype=np.float64)
    nrm = max(np.abs(lam_o).max(), 1e-300)
    bad = []
    out = {}
    err_lam = np.abs(lam_g - lam_o).max() / nrm
    out["lam"] = err_lam
    if not np.all(np.isfinite(lam_g)) or err_lam > t["lam"]:
        bad.append(f"R1 eigenvalue error {err_lam:.3g} > {t['lam']}")
    if Q_g is None:
        return out, bad
    U = Q_g / np.linalg.norm(Q_g, axis=0, keepdims=True)
    rg = relgaps(lam_o, nrm)
    theta = np.linalg.norm(U - Q_o * np.sum(Q_o * U, axis=0, keepdims=True), axis=0)
    out["theta_sep"] = float(np.max(theta[rg >= t["sep"]], initial=0.0))
    mid = (rg < t["sep"]) & (rg >= t["clus"])
    out["theta_gap"] = float(np.max(theta[mid] * rg[mid], initial=0.0))
    if out["theta_sep"] > t["theta"]:
        bad.append(f"R3 separated-vector angle {out['theta_sep']:.3g} > {t['theta']}")
    if out["theta_gap"] > t["gap"]:
        bad.append(f"R3 gap-scaled angle {out['theta_gap']:.3g} > {t['gap']}")
    # clusters: maximal runs of consecutive relative gaps below clus
    worst_c = 0.0
    i = 0
    while i < n:
        j = i
        while j + 1 < n and (lam_o[j + 1] - lam_o[j]) / nrm < t["clus"]:
            j += 1
        if j > i:
            idx = np.arange(i, j + 1)
            V = Q_o[:, idx]
            Uc = U[:, idx]
            outside = np.concatenate([lam_o[:i], lam_o[j + 1:]])
            if outside.size:
                gap_c = min(np.min(np.abs(outside - lam_o[i])), np.min(np.abs(outside - lam_o[j])))
                gap_c = max(gap_c / nrm, 1e-300)
                resid = np.linalg.norm(Uc - V @ (V.T @ Uc), 2)
                worst_c = max(worst_c, resid * gap_c)
                if resid > t["gap"] / gap_c:
                    bad.append(f"R4 cluster [{i},{j}] subspace {resid:.3g} > {t['gap'] / gap_c:.3g}")
        i = j + 1
    out["cluster"] = worst_c
    normA = max(np.linalg.norm(A), 1e-300)
    res = np.linalg.norm(A @ Q_g - Q_g * lam_g) / normA
    orth = np.linalg.norm(Q_g.T @ Q_g - np.eye(n))
    out["res"], out["orth"] = res, orth
    if res > t["res"] or orth > t["res"]:
        bad.append(f"R5 residual {res:.3g} / orthogonality {orth:.3g} > {t['res']}")
    if check_sign:
        idx = np.argmax(np.abs(Q_g), axis=0)
        top = np.abs(Q_g[idx, np.arange(n)])
        # only columns whose largest entry is unambiguous must agree
        srt = np.sort(np.abs(Q_g), axis=0)
        clear = (n == 1) | (srt[-1] - (srt[-2] if n > 1 else 0) > 1e-3 * top)
        if np.any((Q_g[idx, np.arange(n)] <= 0) & clear):
            bad.append("sign convention violated")
    return out, bad


def compare_batch(As, lam_g, Q_g, lam_o, Q_o, dtype, info=None):
    """As, lam_*, Q_* are sequences per matrix.  Returns (worst dict, failures)."""
    worst = {}
    fails = []
    for b in range(len(As)):
        out, bad = compare_one(As[b], lam_g[b], None if Q_g is None else Q_g[b], lam_o[b],
                               None if Q_o is None else Q_o[b], dtype)
        for k, v in out.items():
            worst[k] = max(worst.get(k, 0.0), v)
        if info is not None and int(info[b]) != 0:
            bad.append(f"info = {int(info[b])}")
        if bad:
            fails.append((b, bad))
    return worst, fails

"""Planted-mistake checks: each mutant of the oracle source (built on the CPU
into a temporary library) must fail the pin battery that the real oracle
passes.  This shows the pins are sensitive to dropped terms, wrong signs,
swapped indices and wrong orders anywhere along the path."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

from tests.jacobi_ref import jacobi_eigh
from paper_2604_27325_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bed_oracle.c")

MUTANTS = {
    "z_without_sigma": ("sigma * c->Q[(s - 1) * n + lo + i]", "c->Q[(s - 1) * n + lo + i]"),
    "tear_wrong_sign": ("    c->a[s] -= rho;", "    c->a[s] += rho;"),
    "householder_dropped_term": ("W[i * n + j] -= V[i * n + k] * w[j] + w[i] * V[j * n + k];",
                                 "W[i * n + j] -= V[i * n + k] * w[j];"),
    "householder_tau_sign": ("double t = (alpha - x0) / alpha;", "double t = (x0 - alpha) / alpha;"),
    "lowner_swapped_index": ("double lam_minus_di = -((d[i] - d[origin[j]]) - tau[j]);\n            p *=",
                             "double lam_minus_di = -((d[j] - d[origin[i]]) - tau[i]);\n            p *="),
    "bracket_update_swapped": ("        *U = h;\n    else\n        *L = h;",
                               "        *L = h;\n    else\n        *U = h;"),
    "backtransform_wrong_order": ("for (int k = n - 3; k >= 0; --k) {", "for (int k = 0; k <= n - 3; ++k) {"),
    "deflation_rotation_sign": ("G[row * m + last] = c * gl - s * gi;", "G[row * m + last] = c * gl + s * gi;"),
    "leaf_wrong_vector": ("        Q[2] = -s; Q[3] = c;", "        Q[2] = s; Q[3] = c;"),
    "secular_top_bracket": ("double top = rho * zz;", "double top = 0.5 * rho * zz;"),
}


def _build(src_text, tmp):
    c = os.path.join(tmp, "m.c")
    so = os.path.join(tmp, "m.so")
    with open(c, "w") as fh:
        fh.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-I",
                           os.path.join(ROOT, "oracle"), c, "-o", so, "-lm"])
    lib = ctypes.CDLL(so)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.orc_syevd.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_void_p]
    lib.orc_rank1_eig.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp,
                                  ctypes.c_void_p]
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _battery(lib):
    """True when every pin holds (closed form / Jacobi / LAPACK / exact)."""
    rng = np.random.default_rng(7)
    cases = [workloads.gaussian_sym(rng, 1, n)[0] for n in (3, 6, 16, 33)]
    cases.append(workloads.covariance(rng, 1, 24)[0])
    cases.append(np.outer(np.arange(1.0, 9.0), np.arange(1.0, 9.0)))          # rank one
    T = np.diag(np.full(12, 0.3)) + np.diag(np.full(11, -0.8), 1) + np.diag(np.full(11, -0.8), -1)
    cases.append(T)                                                             # Toeplitz
    for A in cases:
        n = A.shape[0]
        A = np.ascontiguousarray(A, dtype=np.float64)
        lam, Q = np.zeros(n), np.zeros((n, n))
        lib.orc_syevd(n, _p(A), _p(lam), _p(Q), None)
        w, V = jacobi_eigh(A)
        if not np.all(np.isfinite(lam)) or np.max(np.abs(lam - w)) > 1e-12 * np.abs(w).max():
            return False
        if np.linalg.norm(A @ Q - Q * lam) > 1e-12 * np.linalg.norm(A):
            return False
    d = np.array([-1.0, 0.2, 0.2, 0.5, 0.9, 0.9 + 1e-17, 1.3])   # equal poles: type-2 deflation
    z = np.array([0.4, -0.3, 0.6, 0.2, -0.5, 0.1, 0.3])
    lam, U = np.zeros(7), np.zeros((7, 7))
    lib.orc_rank1_eig(7, _p(d), _p(z), 0.7, 0.0, _p(lam), _p(U), None)
    M = np.diag(d) + 0.7 * np.outer(z, z)
    if np.linalg.norm(M @ U - U * lam) > 1e-13 or np.linalg.norm(U.T @ U - np.eye(7)) > 1e-13:
        return False
    return True


def test_unmutated_source_passes_battery():
    with tempfile.TemporaryDirectory() as tmp:
        assert _battery(_build(open(SRC).read(), tmp))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    with tempfile.TemporaryDirectory() as tmp:
        assert not _battery(_build(src.replace(old, new), tmp)), f"{name} slipped through"

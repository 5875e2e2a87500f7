"""binary64 CPU oracle for the batched divide-and-conquer eigensolver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2604_27325_amd``) never imports it and shares no code with it.

The C source (``bed_oracle.c``) follows the note's steps one by one: Householder
tridiagonalization (textbook, Golub & Van Loan Sec. 8.3), rank-one tearing
(Sec. 2.1, Eq. (1)-(3)), 2x2 Givens leaves (Sec. 2.2), the secular equation
(Sec. 2.3.1, Eq. (8)-(12)), hybrid-section (Sec. 2.3.2, Eq. (13)-(17)), Halley
(Sec. 2.3.3, Eq. (20)-(21)), Loewner/Gu-Eisenstat eigenvectors (Sec. 2.3.5,
Eq. (23)-(25)), back-multiplication (Eq. (4)) and the back-transform.  This
module only marshals numpy arrays through ctypes.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bed_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i32p = ctypes.POINTER(ctypes.c_int32)


class Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("merges", "roots", "evals", "halley", "capped", "defl_type1", "defl_type2")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


def build():
    """Compile the oracle with gcc (plain -O2, IEEE semantics, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, "-o", _SO, "-lm"]
    subprocess.check_call(cmd)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_SO)
    lib.orc_tridiag.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
    lib.orc_tridiag_eig.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.POINTER(Stats)]
    lib.orc_rank1_eig.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                  _dp, _dp, ctypes.POINTER(Stats)]
    lib.orc_secular.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                _dp, _ip, _dp, _ip]
    lib.orc_lowner.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, _ip, _dp, _dp]
    lib.orc_deflate.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, _dp, _ip,
                                ctypes.POINTER(Stats)]
    lib.orc_deflate.restype = ctypes.c_double
    lib.orc_syevd.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.POINTER(Stats)]
    lib.orc_syevd_batch.argtypes = [ctypes.c_int64, _i32p, _dp, _dp, _dp, _i32p,
                                    ctypes.POINTER(Stats)]
    lib.orc_syevd_batch.restype = ctypes.c_int64
    lib.orc_syevd_backward.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_double, _dp]
    _lib = lib
    return lib


def _d(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def tridiag(A):
    """Householder reduction of one matrix: returns a, b, V, tau."""
    lib = _load()
    A = _d(A)
    n = A.shape[0]
    a, b = np.zeros(n), np.zeros(max(n - 1, 1))
    V, tau = np.zeros((n, n)), np.zeros(max(n - 2, 1))
    lib.orc_tridiag(n, _ptr(A), _ptr(a), _ptr(b), _ptr(V), _ptr(tau))
    return a, b[: n - 1], V, tau[: max(n - 2, 0)]


def tridiag_eig(a, b, stats=None):
    """D&C eigendecomposition of the tridiagonal (a, b): lam, Q, capped."""
    lib = _load()
    a = _d(a)
    n = a.shape[0]
    b = _d(np.concatenate([np.asarray(b, dtype=np.float64).ravel(), [0.0]]))
    lam, Q = np.zeros(n), np.zeros((n, n))
    st = stats if stats is not None else Stats()
    capped = lib.orc_tridiag_eig(n, _ptr(a), _ptr(b), _ptr(lam), _ptr(Q), ctypes.byref(st))
    return lam, Q, capped


def rank1_eig(d, z, rho, ub_frob=0.0, stats=None):
    """Eigendecomposition of diag(d) + rho z z^T by one merge: lam, U, capped."""
    lib = _load()
    d, z = _d(d), _d(z)
    m = d.shape[0]
    lam, U = np.zeros(m), np.zeros((m, m))
    st = stats if stats is not None else Stats()
    capped = lib.orc_rank1_eig(m, _ptr(d), _ptr(z), float(rho), float(ub_frob), _ptr(lam),
                               _ptr(U), ctypes.byref(st))
    return lam, U, capped


def secular(d, z, rho, ub=0.0):
    """Secular roots for ascending poles d: lam, origin, tau, evals, capped."""
    lib = _load()
    d, z = _d(d), _d(z)
    k = d.shape[0]
    lam, tau = np.zeros(k), np.zeros(k)
    origin = np.zeros(k, dtype=np.intc)
    iters = np.zeros(k, dtype=np.intc)
    capped = lib.orc_secular(k, _ptr(d), _ptr(z), float(rho), float(ub), _ptr(lam),
                             _ptr(origin, _ip), _ptr(tau), _ptr(iters, _ip))
    return lam, origin, tau, iters, capped


def lowner(d, zsign, rho, origin, tau):
    """Gu-Eisenstat zhat of Eq. (25)."""
    lib = _load()
    d, zsign, tau = _d(d), _d(zsign), _d(tau)
    origin = np.ascontiguousarray(origin, dtype=np.intc)
    k = d.shape[0]
    zh = np.zeros(k)
    lib.orc_lowner(k, _ptr(d), _ptr(zsign), float(rho), _ptr(origin, _ip), _ptr(tau), _ptr(zh))
    return zh


def deflate(d, z, rho, stats=None):
    """Deflation of one merge: d', z', G, flag, tol (d ascending)."""
    lib = _load()
    d, z = _d(d).copy(), _d(z).copy()
    m = d.shape[0]
    G = np.zeros((m, m))
    flag = np.zeros(m, dtype=np.intc)
    st = stats if stats is not None else Stats()
    tol = lib.orc_deflate(m, _ptr(d), _ptr(z), float(rho), _ptr(G), _ptr(flag, _ip),
                          ctypes.byref(st))
    return d, z, G, flag.astype(bool), tol


def syevd(A, stats=None):
    """Full oracle on one matrix (n, n) or a uniform batch (b, n, n).

    Returns lam, Q, info with the library's conventions (lower triangle read,
    ascending eigenvalues, sign-canonical columns)."""
    A = _d(A)
    single = A.ndim == 2
    if single:
        A = A[None]
    b, n = A.shape[0], A.shape[1]
    lam, Q, info = syevd_packed(np.full(b, n, dtype=np.int32), A.reshape(-1), stats=stats)
    lam, Q = lam.reshape(b, n), Q.reshape(b, n, n)
    if single:
        return lam[0], Q[0], int(info[0])
    return lam, Q, info


def syevd_packed(n_list, A_packed, stats=None):
    """Packed batch (matrix b at sum n_c^2, eigenvalues at sum n_c)."""
    lib = _load()
    n_arr = np.ascontiguousarray(n_list, dtype=np.int32)
    A = _d(A_packed).ravel()
    tot2 = int(np.sum(n_arr.astype(np.int64) ** 2))
    tot1 = int(np.sum(n_arr.astype(np.int64)))
    assert A.shape[0] == tot2
    lam, Q = np.zeros(tot1), np.zeros(tot2)
    info = np.zeros(n_arr.shape[0], dtype=np.int32)
    st = stats if stats is not None else Stats()
    lib.orc_syevd_batch(n_arr.shape[0], _ptr(n_arr, _i32p), _ptr(A), _ptr(lam), _ptr(Q),
                        _ptr(info, _i32p), ctypes.byref(st))
    return lam, Q, info


def syevd_backward(lam, Q, dlam=None, dQ=None, eps=1e3 * 2.0 ** -53):
    """dA = Q (diag(dlam) + sym(F o Q^T dQ)) Q^T for one matrix or a batch."""
    lib = _load()
    lam, Q = _d(lam), _d(Q)
    single = lam.ndim == 1
    if single:
        lam, Q = lam[None], Q[None]
        dlam = None if dlam is None else _d(dlam)[None]
        dQ = None if dQ is None else _d(dQ)[None]
    b, n = lam.shape
    dA = np.zeros((b, n, n))
    for i in range(b):
        dl = None if dlam is None else _d(dlam[i])
        dq = None if dQ is None else _d(dQ[i])
        out = np.zeros((n, n))
        lib.orc_syevd_backward(n, _ptr(_d(lam[i])), _ptr(_d(Q[i])),
                               _ptr(dl) if dl is not None else None,
                               _ptr(dq) if dq is not None else None, float(eps), _ptr(out))
        dA[i] = out
    return dA[0] if single else dA


# ---------------------------------------------------------------------------
# Spectral matrix functions (the differentiable meta-layer use of Sec. 1):
# plain binary64 definitions on a given decomposition A = Q diag(lam) Q^T.
# ---------------------------------------------------------------------------
def _fn_value(fn, x, p):
    if fn == "sqrt":
        return np.sqrt(x)
    if fn == "invsqrt":
        return 1.0 / np.sqrt(x)
    if fn == "exp":
        return np.exp(x)
    if fn == "log":
        return np.log(x)
    if fn == "pow":
        return x ** p
    raise ValueError(fn)


def _fn_deriv(fn, x, p):
    if fn == "sqrt":
        return 0.5 / np.sqrt(x)
    if fn == "invsqrt":
        return -0.5 * x ** -1.5
    if fn == "exp":
        return np.exp(x)
    if fn == "log":
        return 1.0 / x
    if fn == "pow":
        return p * x ** (p - 1.0)
    raise ValueError(fn)


def spectral_apply(lam, Q, fn, p=0.0):
    """F = Q f(Lambda) Q^T, the definition, for one matrix or a batch."""
    lam, Q = _d(lam), _d(Q)
    f = _fn_value(fn, lam, p)
    return np.einsum("...ik,...k,...jk->...ij", Q, f, Q)


def spectral_backward(lam, Q, dF, fn, p=0.0):
    """dA = Q (K o Q^T sym(dF) Q) Q^T with K_ij = (f(l_i) - f(l_j))/(l_i - l_j)
    and K_ij = f'(l_i) where l_i == l_j (first-order perturbation of f(A),
    Daleckii-Krein), plain divided differences, one matrix or a batch."""
    lam, Q, dF = _d(lam), _d(Q), _d(dF)
    f = _fn_value(fn, lam, p)
    li, lj = lam[..., :, None], lam[..., None, :]
    d = li - lj
    eq = d == 0.0
    K = np.where(eq, _fn_deriv(fn, np.broadcast_to(li, d.shape), p),
                 (f[..., :, None] - f[..., None, :]) / np.where(eq, 1.0, d))
    S = 0.5 * (dF + np.swapaxes(dF, -1, -2))
    W = np.swapaxes(Q, -1, -2) @ S @ Q
    return Q @ (K * W) @ np.swapaxes(Q, -1, -2)

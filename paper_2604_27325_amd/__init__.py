"""Batched small symmetric eigendecomposition on MI355X (gfx950).

Thin ctypes binding over the C ABI in ``include/bed.h`` (library
``_lib/libbed.so``).  PyTorch supplies device memory and streams only: every
step of the solve runs in the library's HIP kernels.  There is no CPU fallback:
if the library is missing or no GPU is present, calls raise.

Method: Householder tridiagonalization + the batch-efficient divide-and-conquer
of Y. Song, "A Short Note on Batch-efficient Divide-and-Conquer Algorithm for
EigenDecomposition" (arXiv 2604.27325), Sec. 2.
"""
import ctypes
import os

__all__ = ["syevd", "syevals", "syevd_packed", "syevd_noalloc_packed", "spectral_apply",
           "spectral_backward", "matrix_function", "FUNCTIONS", "syevd_backward", "eigh", "SyevdFn", "Plan",
           "Server", "autotune", "tune_set", "cache_entries", "BedError", "library_path",
           "load_library", "Tune"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_lib", "libbed.so")
_lib = None

BED_F32, BED_F64 = 0, 1
_STATUS = {0: "BED_OK", 1: "BED_ERR_INVALID_ARG", 2: "BED_ERR_UNSUPPORTED", 3: "BED_ERR_HIP",
           4: "BED_ERR_NOMEM", 5: "BED_ERR_CAPTURE", 6: "BED_ERR_BUSY"}
BED_ERR_BUSY = 6


class BedError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Tune(ctypes.Structure):
    _fields_ = [("threads_big", ctypes.c_int32), ("threads_mid", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("order", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("leaf", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class ServerOpts(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("mem_budget", ctypes.c_int64), ("max_step", ctypes.c_int32),
                ("device", ctypes.c_int32)]


def library_path():
    return _LIB_PATH


def load_library():
    """Load libbed.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- loads the HIP runtime the library must share
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python -m paper_2604_27325_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32p = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)
    lib.bed_syevd.argtypes = [ctypes.c_int, i64, i32p, vp, vp, vp, vp, vp]
    lib.bed_syevals.argtypes = [ctypes.c_int, i64, i32p, vp, vp, vp, vp]
    lib.bed_syevd_noalloc.argtypes = [ctypes.c_int, i64, i32p, vp, vp, vp, vp, vp]
    lib.bed_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64, i32p,
                                    ctypes.POINTER(Tune), vp]
    lib.bed_plan_run.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.bed_plan_get_tune.argtypes = [vp, ctypes.POINTER(Tune)]
    lib.bed_plan_destroy.argtypes = [vp]
    lib.bed_plan_destroy.restype = None
    lib.bed_autotune.argtypes = [ctypes.c_int, i64, i32p, vp, vp, vp, vp, ctypes.POINTER(Tune)]
    lib.bed_spectral_apply.argtypes = [ctypes.c_int, i64, i32p, vp, vp, ctypes.c_int32,
                                       ctypes.c_double, vp, vp]
    lib.bed_spectral_backward.argtypes = [ctypes.c_int, i64, i32p, vp, vp, ctypes.c_int32,
                                          ctypes.c_double, vp, vp, vp]
    lib.bed_tune_set.argtypes = [ctypes.c_int, i64, i32p, ctypes.POINTER(Tune)]
    lib.bed_cache_entries.restype = ctypes.c_int32
    lib.bed_syevd_backward.argtypes = [ctypes.c_int, i64, i32p, vp, vp, vp, vp, vp,
                                       ctypes.c_double, vp]
    lib.bed_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ServerOpts)]
    lib.bed_server_submit.argtypes = [vp, ctypes.c_int, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                      vp, vp, vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.bed_server_poll.argtypes = [vp, ctypes.c_uint64, i32p, ctypes.POINTER(ctypes.c_double)]
    lib.bed_server_drain.argtypes = [vp]
    lib.bed_server_destroy.argtypes = [vp]
    lib.bed_server_destroy.restype = None
    lib.bed_status_string.restype = ctypes.c_char_p
    lib.bed_last_error.restype = ctypes.c_char_p
    lib.bed_version.restype = ctypes.c_int32
    _lib = lib
    return lib


def _check(status):
    if status != 0:
        raise BedError(status, _lib.bed_last_error().decode(errors="replace"))


def _dtype_code(dtype):
    import torch
    if dtype == torch.float32:
        return BED_F32
    if dtype == torch.float64:
        return BED_F64
    raise TypeError(f"unsupported dtype {dtype} (float32 or float64)")


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (the library has no CPU path)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _n_array(n_list):
    import numpy as np
    arr = np.ascontiguousarray(n_list, dtype=np.int32)
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def syevd_packed(n_list, A, lam=None, Q=None, info=None, stream=None, want_vectors=True):
    """Packed batch: A is a flat GPU tensor holding the row-major matrices one
    after another.  Returns (lam_flat, Q_flat or None, info int32)."""
    import torch
    lib = load_library()
    n_arr, n_ptr = _n_array(n_list)
    tot1 = int(n_arr.astype("int64").sum())
    tot2 = int((n_arr.astype("int64") ** 2).sum())
    if A.numel() != tot2:
        raise ValueError(f"A has {A.numel()} elements, packed sizes need {tot2}")
    dt = _dtype_code(A.dtype)
    lam = torch.empty(tot1, dtype=A.dtype, device=A.device) if lam is None else lam
    if want_vectors:
        Q = torch.empty(tot2, dtype=A.dtype, device=A.device) if Q is None else Q
    info = torch.empty(len(n_arr), dtype=torch.int32, device=A.device) if info is None else info
    if want_vectors:
        _check(lib.bed_syevd(dt, len(n_arr), n_ptr, _dev(A, "A"), _dev(lam, "lambda"),
                             _dev(Q, "Q"), _dev(info, "info"), _stream_ptr(stream)))
    else:
        _check(lib.bed_syevals(dt, len(n_arr), n_ptr, _dev(A, "A"), _dev(lam, "lambda"),
                               _dev(info, "info"), _stream_ptr(stream)))
    return lam, (Q if want_vectors else None), info


def syevd_noalloc_packed(n_list, A, lam, Q, info=None, stream=None):
    """bed_syevd_noalloc on a packed batch into caller-provided outputs (the
    library allocates nothing; calls on one GPU must not overlap in time)."""
    lib = load_library()
    n_arr, n_ptr = _n_array(n_list)
    _check(lib.bed_syevd_noalloc(_dtype_code(A.dtype), len(n_arr), n_ptr, _dev(A, "A"),
                                 _dev(lam, "lambda"), _dev(Q, "Q"),
                                 _dev(info, "info") if info is not None else None,
                                 _stream_ptr(stream)))


def syevd(A, return_info=False, stream=None):
    """Eigen-decomposition of a (batch, n, n) or (n, n) symmetric GPU tensor
    (lower triangle read).  Returns (lam ascending, Q) [, info]."""
    single = A.dim() == 2
    Ab = A.unsqueeze(0) if single else A
    if Ab.dim() != 3 or Ab.shape[1] != Ab.shape[2]:
        raise ValueError("A must be (batch, n, n) or (n, n)")
    Ab = Ab.contiguous()
    b, n = Ab.shape[0], Ab.shape[1]
    lam, Q, info = syevd_packed([n] * b, Ab.view(-1), stream=stream)
    lam, Q = lam.view(b, n), Q.view(b, n, n)
    if single:
        lam, Q, info = lam[0], Q[0], info[0]
    return (lam, Q, info) if return_info else (lam, Q)


def syevals(A, stream=None):
    """Eigenvalues only of a (batch, n, n) symmetric GPU tensor."""
    Ab = (A.unsqueeze(0) if A.dim() == 2 else A).contiguous()
    b, n = Ab.shape[0], Ab.shape[1]
    lam, _, info = syevd_packed([n] * b, Ab.view(-1), stream=stream, want_vectors=False)
    lam = lam.view(b, n)
    return lam[0] if A.dim() == 2 else lam


def syevd_backward(lam, Q, dlam=None, dQ=None, eps=0.0, n_list=None, stream=None, out=None):
    """dA = Q (diag(dlam) + sym(F o Q^T dQ)) Q^T (uniform (batch, n[, n]) tensors,
    or flat packed tensors with n_list).  `out` (Q's shape) receives dA."""
    import torch
    lib = load_library()
    if n_list is None:
        b, n = lam.shape[-2] if lam.dim() == 2 else 1, lam.shape[-1]
        n_list = [n] * b
    n_arr, n_ptr = _n_array(n_list)
    lam_c, Q_c = lam.contiguous(), Q.contiguous()
    dl = dlam.contiguous() if dlam is not None else None
    dq = dQ.contiguous() if dQ is not None else None
    dA = torch.empty_like(Q_c) if out is None else out
    if dA.shape != Q_c.shape or dA.dtype != Q_c.dtype:
        raise ValueError("out must have Q's shape and dtype")
    _check(lib.bed_syevd_backward(
        _dtype_code(Q.dtype), len(n_arr), n_ptr, _dev(lam_c, "lambda"), _dev(Q_c, "Q"),
        _dev(dl, "dlambda") if dl is not None else None,
        _dev(dq, "dQ") if dq is not None else None, _dev(dA, "dA"), float(eps),
        _stream_ptr(stream)))
    return dA


FUNCTIONS = {"sqrt": 0, "invsqrt": 1, "exp": 2, "log": 3, "pow": 4}


def _fn_code(fn):
    if fn not in FUNCTIONS:
        raise ValueError(f"unknown function {fn!r} (one of {sorted(FUNCTIONS)})")
    return FUNCTIONS[fn]


def _batch_shape(lam, Q, n_list):
    if n_list is None:
        b, n = (lam.shape[0] if lam.dim() == 2 else 1), lam.shape[-1]
        n_list = [n] * b
    return n_list


def spectral_apply(lam, Q, fn, p=0.0, n_list=None, stream=None, out=None):
    """F = Q f(Lambda) Q^T for a decomposition (uniform (batch, n[, n]) tensors,
    or flat packed tensors with n_list); fn in sqrt, invsqrt, exp, log, pow."""
    import torch
    lib = load_library()
    n_arr, n_ptr = _n_array(_batch_shape(lam, Q, n_list))
    lam_c, Q_c = lam.contiguous(), Q.contiguous()
    F = torch.empty_like(Q_c) if out is None else out
    _check(lib.bed_spectral_apply(_dtype_code(Q.dtype), len(n_arr), n_ptr, _dev(lam_c, "lambda"),
                                  _dev(Q_c, "Q"), _fn_code(fn), float(p), _dev(F, "F"),
                                  _stream_ptr(stream)))
    return F


def spectral_backward(lam, Q, dF, fn, p=0.0, n_list=None, stream=None, out=None):
    """dA = Q (K o Q^T sym(dF) Q) Q^T, K the divided differences of f."""
    import torch
    lib = load_library()
    n_arr, n_ptr = _n_array(_batch_shape(lam, Q, n_list))
    lam_c, Q_c, dF_c = lam.contiguous(), Q.contiguous(), dF.contiguous()
    dA = torch.empty_like(Q_c) if out is None else out
    _check(lib.bed_spectral_backward(_dtype_code(Q.dtype), len(n_arr), n_ptr,
                                     _dev(lam_c, "lambda"), _dev(Q_c, "Q"), _fn_code(fn),
                                     float(p), _dev(dF_c, "dF"), _dev(dA, "dA"),
                                     _stream_ptr(stream)))
    return dA


def _make_fn():
    import torch

    class SyevdFn(torch.autograd.Function):
        """Differentiable eigendecomposition: forward and backward both run in
        the library's kernels."""

        @staticmethod
        def forward(ctx, A, eps=0.0):
            lam, Q = syevd(A)
            ctx.save_for_backward(lam, Q)
            ctx.eps = eps
            return lam, Q

        @staticmethod
        def backward(ctx, dlam, dQ):
            lam, Q = ctx.saved_tensors
            single = lam.dim() == 1
            l2 = lam.unsqueeze(0) if single else lam
            q2 = Q.unsqueeze(0) if single else Q
            dl = None if dlam is None else (dlam.unsqueeze(0) if single else dlam)
            dq = None if dQ is None else (dQ.unsqueeze(0) if single else dQ)
            dA = syevd_backward(l2, q2, dl, dq, eps=ctx.eps)
            return (dA[0] if single else dA), None

    class MatrixFunctionFn(torch.autograd.Function):
        """F = f(A) for symmetric A through the library: the decomposition, then
        Q f(Lambda) Q^T; backward by the divided differences of f."""

        @staticmethod
        def forward(ctx, A, fn, p=0.0):
            lam, Q = syevd(A)
            ctx.save_for_backward(lam, Q)
            ctx.fn, ctx.p = fn, p
            single = lam.dim() == 1
            F = spectral_apply(lam.unsqueeze(0) if single else lam,
                               Q.unsqueeze(0) if single else Q, fn, p)
            return F[0] if single else F

        @staticmethod
        def backward(ctx, dF):
            lam, Q = ctx.saved_tensors
            single = lam.dim() == 1
            dA = spectral_backward(lam.unsqueeze(0) if single else lam,
                                   Q.unsqueeze(0) if single else Q,
                                   dF.unsqueeze(0) if single else dF, ctx.fn, ctx.p)
            return (dA[0] if single else dA), None, None

    SyevdFn.MatrixFunctionFn = MatrixFunctionFn
    return SyevdFn


class _LazyFn:
    _fn = None

    def __getattr__(self, name):
        if _LazyFn._fn is None:
            _LazyFn._fn = _make_fn()
        return getattr(_LazyFn._fn, name)


SyevdFn = _LazyFn()


def matrix_function(A, fn, p=0.0):
    """Differentiable f(A) = Q f(Lambda) Q^T of a symmetric (batch of) GPU
    matrix through the library; fn in sqrt, invsqrt, exp, log, pow."""
    _fn_code(fn)
    return SyevdFn.MatrixFunctionFn.apply(A, fn, p)


def eigh(A, eps=0.0):
    """Differentiable (lam, Q) = eigh(A) through the library."""
    return SyevdFn.apply(A, eps)


class Plan:
    """A reusable schedule for one (dtype, n[]) batch; run() allocates nothing
    and can be captured in a HIP graph."""

    def __init__(self, dtype, n_list, tune=None, stream=None):
        lib = load_library()
        self._n_arr, n_ptr = _n_array(n_list)
        self.dtype = dtype
        h = ctypes.c_void_p()
        t = None
        if tune is not None:
            t = Tune(**{k: int(tune.get(k, 0)) for k, _ in Tune._fields_}) \
                if isinstance(tune, dict) else tune
        _check(lib.bed_plan_create(ctypes.byref(h), _dtype_code(dtype), len(self._n_arr), n_ptr,
                                   ctypes.byref(t) if t is not None else None,
                                   _stream_ptr(stream)))
        self._h = h

    def tune(self):
        t = Tune()
        _check(_lib.bed_plan_get_tune(self._h, ctypes.byref(t)))
        return t.as_dict()

    def run(self, A, lam, Q=None, info=None, stream=None):
        _check(_lib.bed_plan_run(self._h, _dev(A, "A"), _dev(lam, "lambda"),
                                 _dev(Q, "Q") if Q is not None else None,
                                 _dev(info, "info") if info is not None else None,
                                 _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.bed_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(dtype, n_list, A, lam, Q, stream=None):
    """Times candidate schedules for this size mix; returns the winner (dict)."""
    lib = load_library()
    n_arr, n_ptr = _n_array(n_list)
    t = Tune()
    _check(lib.bed_autotune(_dtype_code(dtype), len(n_arr), n_ptr, _dev(A, "A"),
                            _dev(lam, "lambda"), _dev(Q, "Q"), _stream_ptr(stream),
                            ctypes.byref(t)))
    return t.as_dict()


def tune_set(dtype, n_list, tune):
    """Stores a schedule (dict or Tune) for this size mix in the process cache."""
    lib = load_library()
    n_arr, n_ptr = _n_array(n_list)
    t = Tune(**{k: int(tune.get(k, 0)) for k, _ in Tune._fields_}) if isinstance(tune, dict) \
        else tune
    _check(lib.bed_tune_set(_dtype_code(dtype), len(n_arr), n_ptr, ctypes.byref(t)))


def cache_entries():
    """Plans currently held by the convenience entry points' cache."""
    return int(load_library().bed_cache_entries())


class Server:
    """Continuous-batching eigendecomposition server (see bed_server_* in bed.h)."""

    def __init__(self, streams=4, max_inflight=0, mem_budget=0, max_step=4096, device=0):
        lib = load_library()
        o = ServerOpts(streams, max_inflight, mem_budget, max_step, device)
        h = ctypes.c_void_p()
        _check(lib.bed_server_create(ctypes.byref(h), ctypes.byref(o)))
        self._h = h

    def submit(self, A, lam, Q, info=None, stream=None):
        """A: (count, n, n) GPU tensor; returns a ticket or None when admission
        is refused (BED_ERR_BUSY).  The request's step waits for the work
        enqueued so far on `stream` (torch's current stream by default), the
        producer of A."""
        count, n = A.shape[0], A.shape[1]
        tk = ctypes.c_uint64()
        st = _lib.bed_server_submit(self._h, _dtype_code(A.dtype), count, n, _dev(A, "A"),
                                    _dev(lam, "lambda"), _dev(Q, "Q"),
                                    _dev(info, "info") if info is not None else None,
                                    _stream_ptr(stream), ctypes.byref(tk))
        if st == BED_ERR_BUSY:
            return None
        _check(st)
        return tk.value

    def poll(self, ticket):
        """Returns (done, latency_us)."""
        done = ctypes.c_int32()
        lat = ctypes.c_double()
        _check(_lib.bed_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(lat)))
        return bool(done.value), lat.value

    def drain(self):
        _check(_lib.bed_server_drain(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.bed_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Host-side checks of the C-ABI library (no GPU needed): it loads, and exports
every entry point that include/bed.h declares."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bed.h")
LIB = os.path.join(ROOT, "paper_2604_27325_amd", "_lib", "libbed.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bed_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2604_27325_amd import build
        build.build()
    import torch  # noqa: F401  (the library shares torch's HIP runtime)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("bed_syevd", "bed_plan_create", "bed_plan_run", "bed_plan_destroy",
                 "bed_syevd_backward", "bed_server_create", "bed_server_submit",
                 "bed_server_poll", "bed_status_string", "bed_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(bed_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for f in declared_functions():
        assert getattr(lib, f) is not None


def test_status_strings_and_version(lib):
    lib.bed_status_string.restype = ctypes.c_char_p
    lib.bed_version.restype = ctypes.c_int32
    assert lib.bed_status_string(0) == b"BED_OK"
    assert lib.bed_status_string(2) == b"BED_ERR_UNSUPPORTED"
    assert lib.bed_version() >= 100


def test_argument_validation_without_gpu(lib):
    """Validation happens before any HIP call, so it runs on a CPU-only host."""
    lib.bed_last_error.restype = ctypes.c_char_p
    i32 = ctypes.c_int32
    n = (i32 * 3)(4, 65, 8)
    assert lib.bed_syevd(0, ctypes.c_int64(3), n, None, None, None, None, None) == 2  # mixed, n > 64
    n = (i32 * 2)(129, 129)
    assert lib.bed_syevd(0, ctypes.c_int64(2), n, None, None, None, None, None) == 2  # n > 128
    n = (i32 * 2)(100, 100)
    assert lib.bed_syevd(1, ctypes.c_int64(2), n, None, None, None, None, None) == 2  # FP64 > 64
    assert lib.bed_syevd(0, ctypes.c_int64(2), n, None, None, None, None, None) == 1  # NULL A
    # the allocation-free entry point stops at n = 64 (above, a workspace is needed)
    assert lib.bed_syevd_noalloc(0, ctypes.c_int64(2), n, None, None, None, None, None) == 2
    n = (i32 * 2)(4, 0)
    assert lib.bed_syevd(0, ctypes.c_int64(2), n, None, None, None, None, None) == 1  # n < 1
    assert lib.bed_syevd(0, ctypes.c_int64(-1), n, None, None, None, None, None) == 1
    assert lib.bed_syevd(7, ctypes.c_int64(1), n, None, None, None, None, None) == 1  # dtype
    n = (i32 * 1)(4)
    assert lib.bed_syevd(0, ctypes.c_int64(1), n, None, None, None, None, None) == 1  # NULL A
    assert b"NULL" in lib.bed_last_error()
    mis = ctypes.c_void_p(0x1002)
    assert lib.bed_syevd(0, ctypes.c_int64(1), n, mis, mis, mis, None, None) == 1  # misaligned
    assert b"aligned" in lib.bed_last_error()
    assert lib.bed_syevd(0, ctypes.c_int64(0), None, None, None, None, None, None) == 0  # empty
    assert lib.bed_syevd_backward(1, ctypes.c_int64(1), (i32 * 1)(70), None, None, None, None,
                                  None, ctypes.c_double(0), None) == 2


def test_binding_fails_loudly_without_gpu_tensors():
    import torch
    import paper_2604_27325_amd as bed
    if torch.cuda.is_available():
        pytest.skip("host-only check")
    with pytest.raises((ValueError, RuntimeError)):
        bed.syevd(torch.eye(4))


def test_probe_library_exports_its_header():
    """The instrumented measurement copy (include/bed_probe.h) is its own library."""
    probe_h = os.path.join(ROOT, "include", "bed_probe.h")
    probe_so = os.path.join(ROOT, "paper_2604_27325_amd", "_lib", "libbed_probe.so")
    if not os.path.exists(probe_so):
        from paper_2604_27325_amd import build
        build.build()
    text = re.sub(r"/\*.*?\*/", "", open(probe_h).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(bed_[a-z_]+)\s*\(", text)))
    assert names == ["bed_probe_phases"]
    out = subprocess.run(["nm", "-D", "--defined-only", probe_so], capture_output=True, text=True,
                         check=True).stdout
    assert "bed_probe_phases" in set(re.findall(r"\sT\s(bed_\w+)", out))


def test_tune_rejects_unsupported_leaf_size(lib):
    """The leaf cutoff of the divide step is 2, 4 or 8, or 0 for the per-class
    default (checked before any HIP call)."""
    from paper_2604_27325_amd import Tune
    lib.bed_last_error.restype = ctypes.c_char_p
    i32 = ctypes.c_int32
    n = (i32 * 2)(8, 40)
    for leaf in (1, 3, 5, 16, -2):
        t = Tune(threads_big=512, threads_mid=128, leaf=leaf)
        assert lib.bed_tune_set(0, 2, n, ctypes.byref(t)) == 1  # BED_ERR_INVALID_ARG
        assert b"leaf" in lib.bed_last_error()

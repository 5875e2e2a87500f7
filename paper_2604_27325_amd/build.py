"""Build the HIP library libbed.so for gfx950 (cross-compiles without a GPU).

    python -m paper_2604_27325_amd.build        # or: from ... import build; build.build()

Objects go to paper_2604_27325_amd/_build/, the library to
paper_2604_27325_amd/_lib/libbed.so, and the instrumented measurement copy of
the solver (include/bed_probe.h) to paper_2604_27325_amd/_lib/libbed_probe.so.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIB_DIR, "libbed.so")
PROBE_LIB = os.path.join(LIB_DIR, "libbed_probe.so")
ARCH = os.environ.get("BED_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["bed_kernels.hip", "bed_backward.hip", "bed_api.cpp", "bed_backward_api.cpp",
           "bed_tune.cpp", "bed_server.cpp", "bed_noalloc.hip", "bed_spectral.hip", "bed_big.hip"]
PROBE_SOURCES = ["bed_probe.hip"]

# Every HIP translation unit is compiled with packed-FP32 instruction
# selection disabled (plain float code only).
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(line for line in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in line)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{msgs}")
    return obj, msgs


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-o", tmp] + objs + ["-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    os.makedirs(LIB_DIR, exist_ok=True)
    srcs = SOURCES + PROBE_SOURCES
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(srcs), 7)) as ex:
        results = dict(zip(srcs, ex.map(_compile, srcs)))
    for obj, msgs in results.values():
        if verbose and msgs.strip():
            print(msgs, file=sys.stderr)
    _link([results[s][0] for s in SOURCES], LIB)
    _link([results[s][0] for s in PROBE_SOURCES], PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

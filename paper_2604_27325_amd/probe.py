"""Phase and Householder-step timing of the solver (measurement tool).

Runs the instrumented copy of the uniform-batch kernel (libbed_probe.so,
include/bed_probe.h) on the batch-512 workload and prints, as markdown, the
mean time of every phase over the teams and the cycle breakdown of one
Householder step.

    python -m paper_2604_27325_amd.probe --n 64 [--threads 512] [--batch 256]
"""
import argparse
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
PROBE_LIB = os.path.join(_HERE, "_lib", "libbed_probe.so")
PHASES, SUBSTEPS = 64, 16
SUB_NAMES = {1: "dot product", 2: "partial exchange + barrier", 3: "reduction p^T v",
             4: "w broadcast (write, read)", 5: "reduction of the pivot column norm",
             6: "reflector scalars", 7: "v broadcast writes", 8: "rank-2 update"}


def phase_names(n):
    """(id, name) in execution order for order n (leaves of at most 8 elements
    for n > 32, else 4: the library's default cutoffs)."""
    leaf = 8 if n > 32 else 4
    D = 0
    while ((n + (1 << D) - 1) >> D) > leaf:
        D += 1
    out = [(1, "load"), (2, "Householder (+ Q_H)"), (3, "tear + leaves")]
    for d in range(D - 1, -1, -1):
        for j, nm in enumerate(["merge setup", "secular roots", "Loewner zhat",
                                "vectors + assembly", "type-2 rotations", "back-multiplication"]):
            out.append((10 + 8 * d + j, f"depth {d}: {nm}"))
    out += [(4, "back-transform"), (5, "store")]
    return out


def run(n, threads, dtype="f32", lib_path=PROBE_LIB, batch=512):
    import torch

    from paper_2604_27325_amd import load_library, workloads
    load_library()  # torch's HIP runtime first
    lib = ctypes.CDLL(lib_path)
    vp = ctypes.c_void_p
    lib.bed_probe_phases.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp]
    A_np, _, _ = workloads.paper_scale(n)
    A_np = A_np[:batch]
    dt = torch.float32 if dtype == "f32" else torch.float64
    A = torch.from_numpy(A_np).to("cuda", dt)
    b = A.shape[0]
    lam = torch.empty(b, n, device="cuda", dtype=dt)
    Q = torch.empty_like(A)
    marks = torch.zeros(b * PHASES, dtype=torch.int64, device="cuda")
    steps = torch.zeros(b * SUBSTEPS, dtype=torch.int64, device="cuda")
    defl = torch.zeros(b * 2, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream()
    for _ in range(3):  # warm-up, then the recorded launch
        st = lib.bed_probe_phases(0 if dtype == "f32" else 1, threads, n, b, vp(A.data_ptr()),
                                  vp(lam.data_ptr()), vp(Q.data_ptr()), vp(marks.data_ptr()),
                                  vp(steps.data_ptr()), vp(defl.data_ptr()), vp(s.cuda_stream))
        if st != 0:
            raise RuntimeError(f"bed_probe_phases returned {st}")
    torch.cuda.synchronize()
    return (marks.view(b, PHASES).cpu().numpy(), steps.view(b, SUBSTEPS).cpu().numpy(),
            defl.view(b, 2).cpu().numpy())


def report(n, threads, hstep, marks, steps, defl=None):
    order = phase_names(n)
    lines = [f"phase timing, batch {marks.shape[0]} n={n} FP32, {threads} threads per matrix "
             "(mean over teams, 100 MHz clock)", "", "| phase | mean us | max us |", "|---|---|---|"]
    prev = marks[:, 0]
    total = np.zeros(marks.shape[0])
    for pid, name in order:
        cur = marks[:, pid]
        d = (cur - prev) * 1e-2  # 100 MHz ticks -> us
        lines.append(f"| {name} | {d.mean():.2f} | {d.max():.2f} |")
        total += d
        prev = cur
    lines.append(f"| **team total** | {total.mean():.2f} | {total.max():.2f} |")
    span = (marks[:, 5].max() - marks[:, 0].min()) * 1e-2
    lines.append("")
    lines.append(f"first team start to last team end: {span:.1f} us")
    st = steps[steps[:, 0] != 0]
    if st.size:
        mark = float(np.mean(st[:, 9] - st[:, 8]))
        lines += ["", f"Householder step k = {hstep}, wave 0: shader-clock cycles between "
                  f"markers, mean over {st.shape[0]} teams, with one marker's own cost "
                  f"({mark:.0f} cycles, which include waiting for outstanding LDS and scalar "
                  "operations) subtracted", "", "| sub-step | cycles |", "|---|---|"]
        prev = 0
        for i in sorted(SUB_NAMES):
            if np.all(st[:, i] != 0):
                c = float(np.mean(st[:, i] - st[:, prev])) - mark
                lines.append(f"| {SUB_NAMES[i]} | {c:.0f} |")
                prev = i
        full = float(np.mean(st[:, 8] - st[:, 0]))
        lines.append(f"| **step (start to end of update, markers included)** | {full:.0f} |")
    if defl is not None:
        lines += ["", f"deflations per matrix (mean over {defl.shape[0]}): type 1 "
                  f"{defl[:, 0].mean():.2f}, type 2 {defl[:, 1].mean():.3f}; matrices with a "
                  f"type-2 rotation: {int((defl[:, 1] > 0).sum())}"]
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--lib", default=PROBE_LIB, help="probe library to load")
    ap.add_argument("--batch", type=int, default=512,
                    help="matrices (at most 512; 256 puts one team on each CU)")
    a = ap.parse_args()
    threads = a.threads or (64 if a.n <= 16 else (256 if a.n <= 32 else 512))
    hstep = 8 if a.n <= 16 else (16 if a.n <= 32 else 32)
    marks, steps, defl = run(a.n, threads, lib_path=a.lib, batch=a.batch)
    print(report(a.n, threads, hstep, marks, steps, defl))


if __name__ == "__main__":
    main()

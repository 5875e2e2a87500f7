"""Summarize rocprofv3 CSV output for one kernel into the markdown kept in
profiles/ (measurement tool; reads profiler output, runs nothing on the GPU).

Inputs: the kernel statistics of a kernel-trace run (--trace, a
*_kernel_stats.csv, or the per-dispatch *_kernel_trace.csv when --grid picks
one launch shape) and a directory of counter runs (--pmc-dir, files
p<i>_counter_collection.csv, one counter set per run).  FETCH_SIZE and
WRITE_SIZE are calibrated against the device copy that `bench.py
--copy-calibration` launches in the same process (--calib-bytes bytes read and
written).  Reported per launch of the kernel: the trace's mean duration, the
mean of every counter, and derived figures: HBM traffic, achieved clock
(GRBM_GUI_ACTIVE over the dispatch's own duration), executed FP32/FP64 vector
and matrix-core flops (instruction counts x 64 lanes, FMA = 2, MFMA ops x 512)
against the algorithmic model, LDS bank-conflict cycles per active LDS cycle,
the share of wave cycles spent waiting, and the mean occupancy.

    python -m paper_2604_27325_amd.profile_summary --kernel 'k_syevd_uniform<float, 64, 512>' \\
        --trace T.csv --pmc-dir D --flops F --bytes B --sources a.hip b.hpp ... \\
        --trace-command '...' --pmc-command '...' > profiles/x.md
"""
import argparse
import csv
import glob
import hashlib
import os
import shlex
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def trace_stats(path, kernel, grid=None):
    """Launch count and mean/min/max duration of `kernel`: from a kernel-stats
    file, or from a per-dispatch kernel-trace file, where `grid` (work-items)
    selects the dispatches of one launch shape."""
    if "kernel_trace" in os.path.basename(path):
        d = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in csv.DictReader(open(path))
             if kernel in r["Kernel_Name"] and (grid is None or int(r["Grid_Size_X"]) == grid)]
        if not d:
            raise SystemExit(f"{kernel} (grid {grid}) not in {path}")
        return {"calls": len(d), "avg_ns": sum(d) / len(d), "min_ns": float(min(d)),
                "max_ns": float(max(d))}
    for r in csv.DictReader(open(path)):
        if kernel in r["Name"]:
            return {"calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                    "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"])}
    raise SystemExit(f"{kernel} not in {path}")


def counters(pmc_dir, kernel, calib_kernel, grid=None):
    """{counter: mean value per dispatch of `kernel`} (only dispatches of `grid`
    work-items when given), per-dispatch durations (ns), and the calibration
    kernel's FETCH/WRITE values (largest dispatch)."""
    vals, durs, calib = defaultdict(list), defaultdict(list), {}
    for f in sorted(glob.glob(os.path.join(pmc_dir, "p*_counter_collection.csv"))):
        for r in csv.DictReader(open(f)):
            name, v = r["Counter_Name"], float(r["Counter_Value"])
            if kernel in r["Kernel_Name"] and (grid is None or int(r["Grid_Size"]) == grid):
                vals[name].append(v)
                durs[name].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
            elif calib_kernel and calib_kernel in r["Kernel_Name"] and name in ("FETCH_SIZE",
                                                                                "WRITE_SIZE"):
                calib[name] = max(calib.get(name, 0.0), v)
    mean = {k: sum(v) / len(v) for k, v in vals.items()}
    return mean, vals, durs, calib


def gpu_agent(pmc_dir):
    """(XCD count, max engine clock in MHz) of the GPU agent of the counter runs."""
    for f in sorted(glob.glob(os.path.join(pmc_dir, "p*_agent_info.csv"))):
        for r in csv.DictReader(open(f)):
            if r.get("Agent_Type") == "GPU":
                return int(r.get("Num_Xcc") or 1), float(r.get("Max_Engine_Clk_Fcompute") or 0)
    return 1, 0.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--title", default=None)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--pmc-dir", required=True)
    ap.add_argument("--calib-kernel", default="__amd_rocclr_copyBuffer")
    ap.add_argument("--calib-dir", default=None,
                    help="counter runs holding the calibration copy (default: --pmc-dir)")
    ap.add_argument("--calib-bytes", type=float, default=256 * 2 ** 20)
    ap.add_argument("--grid", type=int, default=None,
                    help="only dispatches of this many work-items (one launch shape)")
    ap.add_argument("--flops", type=float, required=True, help="algorithmic flops per launch")
    ap.add_argument("--bytes", type=float, required=True, help="algorithmic bytes per launch")
    ap.add_argument("--sources", nargs="+", required=True)
    ap.add_argument("--trace-command", required=True)
    ap.add_argument("--pmc-command", required=True)
    a = ap.parse_args()

    tr = trace_stats(a.trace, a.kernel, a.grid)
    mean, vals, durs, calib = counters(a.pmc_dir, a.kernel, a.calib_kernel, a.grid)
    if a.calib_dir:
        calib = counters(a.calib_dir, "\0no kernel\0", a.calib_kernel)[3]
    xcc, fmax = gpu_agent(a.pmc_dir)
    t = tr["avg_ns"] * 1e-9
    out = [f"# {a.title or a.kernel}", ""]
    out += ["Commands (from /tmp, with TMPDIR=/tmp; REPO is the repository root):", "",
            "    " + a.trace_command, "    " + a.pmc_command, "",
            "Summary written by:", "",
            "    python -m paper_2604_27325_amd.profile_summary " + shlex.join(sys.argv[1:]), ""]
    out += [f"kernel-trace: {tr['calls']} launches, mean {tr['avg_ns'] / 1e3:.2f} us "
            f"(min {tr['min_ns'] / 1e3:.2f}, max {tr['max_ns'] / 1e3:.2f})", ""]
    out += ["| counter | mean per launch |", "|---|---|"]
    for k in sorted(mean):
        out.append(f"| {k} | {mean[k]:.6g} |")
    out.append("")
    der = []
    fetch, write = mean.get("FETCH_SIZE"), mean.get("WRITE_SIZE")
    traffic = None
    if fetch is not None and write is not None and "FETCH_SIZE" in calib and "WRITE_SIZE" in calib:
        ff = a.calib_bytes / (calib["FETCH_SIZE"] * 1024.0)
        fw = a.calib_bytes / (calib["WRITE_SIZE"] * 1024.0)
        traffic = fetch * 1024.0 * ff + write * 1024.0 * fw
        der.append(f"HBM traffic: {traffic / 1e6:.3f} MB per launch (FETCH_SIZE x {ff:.3f}, "
                   f"WRITE_SIZE x {fw:.3f} from the {a.calib_bytes / 2 ** 20:.0f} MiB copy); "
                   f"algorithmic {a.bytes / 1e6:.3f} MB, ratio {traffic / a.bytes:.3f}; "
                   f"{traffic / t / 1e9:.1f} GB/s at the traced duration")
    if "GRBM_GUI_ACTIVE" in vals:
        g, d = vals["GRBM_GUI_ACTIVE"], durs["GRBM_GUI_ACTIVE"]
        clk = sum(gi / di for gi, di in zip(g, d)) / len(g) / xcc
        der.append(f"achieved clock: {clk:.2f} GHz (GRBM_GUI_ACTIVE, summed over the {xcc} XCDs, "
                   f"per XCD over the dispatch's duration; the agent's maximum is "
                   f"{fmax / 1e3:.2f} GHz; short dispatches overstate it)")
    v32 = sum(mean.get(k, 0.0) * w for k, w in (("SQ_INSTS_VALU_FMA_F32", 2),
                                                 ("SQ_INSTS_VALU_ADD_F32", 1),
                                                 ("SQ_INSTS_VALU_MUL_F32", 1),
                                                 ("SQ_INSTS_VALU_TRANS_F32", 1))) * 64
    v64 = sum(mean.get(k, 0.0) * w for k, w in (("SQ_INSTS_VALU_FMA_F64", 2),
                                                 ("SQ_INSTS_VALU_ADD_F64", 1),
                                                 ("SQ_INSTS_VALU_MUL_F64", 1),
                                                 ("SQ_INSTS_VALU_TRANS_F64", 1))) * 64
    m32 = mean.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) * 512
    m64 = mean.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512
    if "SQ_INSTS_VALU_FMA_F32" in mean:
        der.append(f"executed flops per launch (64 lanes per instruction): vector FP32 "
                   f"{v32 / 1e6:.1f} M, vector FP64 {v64 / 1e6:.1f} M, MFMA FP32 {m32 / 1e6:.1f} M, "
                   f"MFMA FP64 {m64 / 1e6:.1f} M; algorithmic model {a.flops / 1e6:.1f} M")
        der.append(f"achieved at the traced duration: vector {(v32 + v64) / t / 1e12:.2f} TFLOP/s, "
                   f"MFMA {(m32 + m64) / t / 1e12:.2f} TFLOP/s, model {a.flops / t / 1e12:.2f} "
                   f"TFLOP/s ({a.flops / t / 1e12 / 157.3:.4f} of 157.3)")
    if "SQ_LDS_BANK_CONFLICT" in mean and mean.get("SQ_LDS_IDX_ACTIVE", 0) > 0:
        der.append(f"LDS bank-conflict cycles per active LDS cycle: "
                   f"{mean['SQ_LDS_BANK_CONFLICT'] / mean['SQ_LDS_IDX_ACTIVE']:.3f}")
    if "SQ_WAIT_INST_ANY" in mean and mean.get("SQ_WAVE_CYCLES", 0) > 0:
        der.append(f"wave cycles waiting for any instruction's operands: "
                   f"{mean['SQ_WAIT_INST_ANY'] / mean['SQ_WAVE_CYCLES']:.3f}")
    if "SQ_WAIT_ANY" in mean and "SQ_WAVE_CYCLES" in mean:
        der.append(f"SQ_WAIT_ANY per wave cycle: {mean['SQ_WAIT_ANY'] / mean['SQ_WAVE_CYCLES']:.3f}")
    if "MeanOccupancyPerCU" in mean:
        der.append(f"mean occupancy: {mean['MeanOccupancyPerCU']:.2f} waves per CU")
    if "SQ_INSTS_VALU" in mean and "SQ_WAVES" in mean and mean["SQ_WAVES"] > 0:
        der.append(f"per wave: {mean['SQ_INSTS_VALU'] / mean['SQ_WAVES']:.0f} VALU, "
                   f"{mean.get('SQ_INSTS_LDS', 0) / mean['SQ_WAVES']:.0f} LDS, "
                   f"{mean.get('SQ_INSTS_MFMA', 0) / mean['SQ_WAVES']:.0f} MFMA, "
                   f"{mean.get('SQ_INSTS_SALU', 0) / mean['SQ_WAVES']:.0f} SALU instructions")
    out += ["Derived:", ""] + [f"- {x}" for x in der] + [""]
    h = hashlib.sha256()
    for src in a.sources:
        with open(os.path.join(HERE, "csrc", src), "rb") as f:
            h.update(f.read())
    out += [f"kernel_sources = {' '.join(a.sources)}",
            f"kernel_sources_sha256 = {h.hexdigest()}",
            f"trace_mean_us = {tr['avg_ns'] / 1e3:.3f}"]
    if traffic is not None:
        out.append(f"traffic_bytes_per_launch = {traffic:.0f}")
    print("\n".join(out))


if __name__ == "__main__":
    main()

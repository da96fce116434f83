"""Summaries of rocprofv3 output for the banded kernels.

  python profsum.py stats KERNEL_STATS_CSV --cmd "..."
      per-kernel call counts and durations (rocprofv3 --kernel-trace --stats)
  python profsum.py mfma COUNTERS_CSV --stats KERNEL_STATS_CSV --cmd "..." --cmd-stats "..."
      MFMA flops, busy cycles and utilisation per kernel (rocprofv3 --pmc
      SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE)
  python profsum.py traffic --fetch CSV --write CSV \\
      --copy-fetch CSV --copy-write CSV --copy-bytes B --rows R --cmd "..."
      HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counters (KiB per
      dispatch), each scaled by what the same counter reads for a plain copy of
      a known size.

Both print short text on stdout.  The traffic summary records a hash of the
kernel sources: bench.py reports the measured traffic only while the kernels
are unchanged since the counters were taken.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "paper_1902_10078_amd", "csrc")

# rocprofv3 kernel name -> the library's profiling slot name
_KERNEL_SLOTS = [
    (r"k_f1_sum<", "f1_summary"),
    (r"k_f1_sum_q<", "f1_summary"),
    (r"k_f1_rep<", "f1_replay"),
    (r"k_pc<", "chunk_product"),
    (r"k_fs<\d+, \w+, false", "fs_summary"),
    (r"k_fs<\d+, \w+, true", "fs_replay"),
    (r"k_f2<\d+, \w+, false", "f2_summary"),
    (r"k_f2<\d+, \w+, true", "f2_replay"),
    (r"k_b1<\d+, \w+, false", "b1_summary"),
    (r"k_b1<\d+, \w+, true", "b1_replay"),
    (r"k_b2<\d+, \w+, false", "b2_summary"),
    (r"k_b2<\d+, \w+, true", "b2_replay"),
    (r"k_f1_gscan", "f1_group_compose"),
    (r"k_f1_gcomp_q", "f1_group_compose"),
    (r"k_f1_pscan", "f1_group_sweep"),
    (r"k_f1_sweep_q<\d+, true>", "f1_group_sweep"),
    (r"k_f1_sweep_q<\d+, false>", "f1_chunk_sweep"),
    (r"k_lin_sweep_q<\d+, true, true>", "desc_group_sweep"),
    (r"k_lin_sweep_q<\d+, true, false>", "desc_chunk_sweep"),
    (r"k_lin_sweep_q<\d+, false, true>", "asc_group_sweep"),
    (r"k_lin_sweep_q<\d+, false, false>", "asc_chunk_sweep"),
    (r"k_f1_capply", "f1_chunk_sweep"),
    (r"k_lin_gscan<\d+, true>", "desc_group_compose"),
    (r"k_lin_gcomp_q<\d+, true>", "desc_group_compose"),
    (r"k_lin_gcomp_q<\d+, false>", "asc_group_compose"),
    (r"k_lin_pscan<\d+, true>", "desc_group_sweep"),
    (r"k_lin_capply<\d+, true>", "desc_chunk_sweep"),
    (r"k_lin_gscan<\d+, false>", "asc_group_compose"),
    (r"k_lin_pscan<\d+, false>", "asc_group_sweep"),
    (r"k_lin_capply<\d+, false>", "asc_chunk_sweep"),
    (r"F1GroupCompose", "f1_group_compose"),
    (r"F1GroupSweep", "f1_group_sweep"),
    (r"F1ChunkSweep", "f1_chunk_sweep"),
    (r"LinGroupCompose<\d+, true>", "desc_group_compose"),
    (r"LinGroupSweep<\d+, true>", "desc_group_sweep"),
    (r"LinChunkSweep<\d+, true>", "desc_chunk_sweep"),
    (r"LinGroupCompose<\d+, false>", "asc_group_compose"),
    (r"LinGroupSweep<\d+, false>", "asc_group_sweep"),
    (r"LinChunkSweep<\d+, false>", "asc_chunk_sweep"),
    (r"k_wf1_sum", "wide_f1_sum"),
    (r"k_wf1_scan", "wide_f1_scan"),
    (r"k_wf1_rep", "wide_f1"),
    (r"k_wfin", "wide_finalize"),
    (r"k_wlin_sum", "wide_lin_sum"),
    (r"k_wlin_scan", "wide_lin_scan"),
    (r"k_wf2_rep", "wide_f2"),
    (r"k_wb1_rep", "wide_b1"),
    (r"k_wb2<false>", "wide_b2_sum"),
    (r"k_wb2<true>", "wide_b2"),
    (r"k_kl_pre", "vi_pre"),
    (r"k_kl_post", "vi_post"),
    (r"k_kl_neg", "vi_neg"),
    (r"k_solve_mat<", "solve_mat"),
    (r"k_solve_mat_g<", "solve_mat_g"),
    (r"k_solve_mat_lbar", "solve_mat_out"),
    (r"k_ml_post<", "ml_post"),
    (r"k_ml_finalize", "ml_finalize"),
    (r"k_kl_finalize|k_finalize", "finalize"),
    (r"k_csr_to_band", "csr_to_band"),
    (r"k_band_to_csr", "band_to_csr"),
    (r"k_ng_pre<", "ng_pre"),
    (r"k_ng_post<", "ng_post"),
    (r"k_ng_neg<", "ng_neg"),
    (r"k_ng_finalize", "ng_finalize"),
    (r"ClearPart", "clear_partials"),
    (r"k_gbmm", "gbmm"),
    (r"k_gbmv", "gbmv"),
    (r"k_outer", "outer_band"),
    (r"k_logdet_bwd", "logdet_bwd"),
]


def slot_of(kernel_name: str) -> str | None:
    for pat, slot in _KERNEL_SLOTS:
        if re.search(pat, kernel_name):
            return slot
    return None


# Sources of the row-streaming kernels, their scans and their schedule (the
# default set a traffic summary is tied to); a summary can name others.
_KERNEL_SOURCES = ("bandops_algo.hpp", "bandops_step.hpp", "bandops_items.hpp", "bandops_tile.hpp",
                   "bandops_driver.hpp", "bandops_steps.hpp", "bandops_kern.hip")


def source_hash(sources=None) -> str:
    """Hash of the sources (file names under csrc/) that decide what the
    measured kernels execute; default: the row-streaming kernels."""
    h = hashlib.sha256()
    names = sorted(sources.split(",") if isinstance(sources, str) else (sources or _KERNEL_SOURCES))
    for f in names:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _counter_means(path: str, counter: str):
    vals = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in vals.items()}


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    print(f"# rocprofv3 kernel trace summary")
    print(f"# command: {args.cmd}")
    print(f"# {'slot':22s} {'calls':>6s} {'avg_ms':>10s} {'total_%':>8s}  kernel")
    for r in rows:
        name = r["Name"]
        slot = slot_of(name) or "-"
        print(f"  {slot:22s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e6:10.4f} "
              f"{float(r['Percentage']):8.2f}  {name[:110]}")


def traffic(args):
    cf = _counter_means(args.copy_fetch, "FETCH_SIZE")
    cw = _counter_means(args.copy_write, "WRITE_SIZE")
    copy_k = [k for k in cf if "copy" in k.lower()]
    if not copy_k:
        sys.exit("no copy kernel in the calibration run")
    kib = args.copy_bytes / 1024.0
    fscale = kib / cf[copy_k[0]][0]
    wscale = kib / cw[copy_k[0]][0]
    fe = _counter_means(args.fetch, "FETCH_SIZE")
    wr = _counter_means(args.write, "WRITE_SIZE")
    print("# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (KiB per dispatch)")
    print(f"# command (fetch): {args.cmd_fetch or args.cmd}")
    print(f"# command (write): {args.cmd_write or args.cmd}")
    print(f"# calibration: a plain copy of {args.copy_bytes} bytes ({copy_k[0]}) reads "
          f"FETCH_SIZE {cf[copy_k[0]][0]:.1f} KiB and WRITE_SIZE {cw[copy_k[0]][0]:.1f} KiB")
    print(f"fetch_scale: {fscale:.4f}")
    print(f"write_scale: {wscale:.4f}")
    print(f"rows_per_launch: {args.rows}")
    srcs = args.sources or ",".join(_KERNEL_SOURCES)
    print(f"hash_sources: {srcs}")
    print(f"source_hash: {source_hash(srcs)}")
    print(f"# {'slot':20s} {'fetch_GB':>10s} {'write_GB':>10s} {'traffic_GB':>11s} {'B/row':>8s}")
    seen = set()
    for k, (fv, n) in fe.items():
        slot = slot_of(k)
        if slot is None or slot in seen or k not in wr:
            continue
        seen.add(slot)
        fb = fv * 1024 * fscale
        wb = wr[k][0] * 1024 * wscale
        print(f"traffic {slot:20s} {fb / 1e9:10.4f} {wb / 1e9:10.4f} {(fb + wb) / 1e9:11.4f} "
              f"{(fb + wb) / args.rows:8.1f}")


def mfma(args):
    """MFMA work and busy cycles per kernel slot from one rocprofv3 --pmc run
    of SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE,
    with the average durations of a kernel-trace summary."""
    mops = _counter_means(args.csv, "SQ_INSTS_VALU_MFMA_MOPS_F32")
    busy = _counter_means(args.csv, "SQ_VALU_MFMA_BUSY_CYCLES")
    gui = _counter_means(args.csv, "GRBM_GUI_ACTIVE")
    dur = {}
    for r in csv.DictReader(open(args.stats)):
        dur[r["Name"]] = float(r["AverageNs"]) / 1e9
    print("# MFMA use per dispatch from rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_VALU_MFMA_BUSY_CYCLES "
          "GRBM_GUI_ACTIVE")
    print(f"# command: {args.cmd}")
    print(f"# durations: {args.cmd_stats}")
    print(f"# FP32 MFMA flops = MOPS_F32 * 512 (executed, zeros of the dense blocks included);")
    print(f"# util = MFMA busy cycles (summed over SIMDs) / (average kernel duration * {args.clock_ghz} GHz * "
          f"{args.simds} SIMDs)")
    print(f"# (GRBM_GUI_ACTIVE, shown for reference, spans the profiler's serialised dispatch, not the kernel alone);")
    print(f"# TFLOP/s = flops / average kernel duration; peak FP32 MFMA {args.peak} TFLOP/s")
    print(f"# {'slot':16s} {'GFLOP':>9s} {'busy_Mcyc':>10s} {'gui_Mcyc':>9s} {'util_%':>7s} {'avg_ms':>8s} {'TFLOP/s':>8s} "
          f"{'of_peak':>7s}")
    seen = set()
    for k, (mv, n) in mops.items():
        slot = slot_of(k)
        if slot is None or (slot, k) in seen or k not in busy or k not in gui:
            continue
        seen.add((slot, k))
        fl = mv * 512
        d = dur.get(k)
        util = 100.0 * busy[k][0] / (d * args.clock_ghz * 1e9 * args.simds) if d else float("nan")
        tf = fl / d / 1e12 if d else float("nan")
        print(f"mfma {slot:16s} {fl / 1e9:9.3f} {busy[k][0] / 1e6:10.2f} {gui[k][0] / 1e6:9.3f} {util:7.2f} "
              f"{(d or float('nan')) * 1e3:8.3f} {tf:8.3f} {tf / args.peak:7.4f}")


def read_traffic(path: str):
    """Parse a traffic summary: {slot: bytes per launch}, plus its source hash."""
    out, meta = {}, {}
    if not os.path.exists(path):
        return out, meta
    for line in open(path):
        if line.startswith("#"):
            continue
        parts = line.split()
        if not parts:
            continue
        if parts[0] == "traffic" and len(parts) >= 5:
            out[parts[1]] = float(parts[4]) * 1e9
        elif parts[0].endswith(":") and len(parts) == 2:
            meta[parts[0][:-1]] = parts[1]
    return out, meta


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    for nm in ("--fetch", "--write", "--copy-fetch", "--copy-write"):
        t.add_argument(nm, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--rows", type=int, required=True)
    t.add_argument("--cmd", default="")
    t.add_argument("--cmd-fetch", default="")
    t.add_argument("--cmd-write", default="")
    t.add_argument("--sources", default="", help="comma-separated csrc/ files the measured kernels come from")
    m = sub.add_parser("mfma")
    m.add_argument("csv")
    m.add_argument("--stats", required=True, help="kernel_stats.csv of a kernel-trace run of the same workload")
    m.add_argument("--cmd", required=True)
    m.add_argument("--cmd-stats", required=True)
    m.add_argument("--simds", type=int, default=1024)
    m.add_argument("--peak", type=float, default=157.3)
    m.add_argument("--clock-ghz", type=float, default=2.4)
    a = ap.parse_args(argv)
    {"stats": stats, "traffic": traffic, "mfma": mfma}[a.cmd_name](a)


if __name__ == "__main__":
    main()

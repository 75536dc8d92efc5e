"""Summaries of rocprofv3 output for the committed profile records.

Two reports, each written as short text (plus JSON for traffic) that names the
command which produced the raw data:

  stats   -- from ``rocprofv3 --kernel-trace --stats --output-format csv``:
             per kernel the number of dispatches and the average / total
             duration.
  traffic -- from two ``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``
             runs of the same program: HBM bytes per dispatch of each kernel,
             scaled by what the same counters read for a device copy of known
             size in that program (the calibration).
  mfma    -- from ``rocprofv3 --pmc MfmaUtil MfmaFlopsF64 MfmaFlopsF32``: per
             kernel the matrix-core FLOPs per dispatch (FP64 and FP32) and the
             fraction of SIMD cycles the matrix cores were busy.

Usage:
  python -m paper_1710_08471_amd.profiling stats DIR --command CMD --out FILE
  python -m paper_1710_08471_amd.profiling traffic --fetch DIR --write DIR \\
      --copy-bytes N --command-fetch CMD --command-write CMD --out-json F --out-txt F
  python -m paper_1710_08471_amd.profiling mfma DIR --command CMD --out FILE
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))

# Source files that define and launch each kernel family (the .hip file and
# the device headers it includes): a counter result stays valid while they are
# unchanged.
KERNEL_SOURCE = {
    "k_gram_partials": ["cqr2_gram.hip", "gram_dev.h"],
    "k_gram_reduce": ["cqr2_gram.hip", "gram_dev.h"],
    "k_cholinv": ["cqr2_cholinv.hip", "cholinv_dev.h"],
    "k_apply_rinv": ["cqr2_apply.hip", "apply_dev.h"],
    "k_gemm": ["cqr2_gemm.hip"],
    "k_gemm_f32": ["cqr2_gemm.hip"],
    "k_gemm_reduce": ["cqr2_gemm.hip"],
    "k_gram_wide": ["cqr2_wide.hip", "wide_dev.h", "sync_dev.h"],
    "k_gram_wide_reduce": ["cqr2_wide.hip", "wide_dev.h", "sync_dev.h"],
    "k_syrk_tile": ["cqr2_wide.hip", "wide_dev.h", "sync_dev.h"],
    "k_syrk_reduce": ["cqr2_wide.hip", "wide_dev.h", "sync_dev.h"],
    "k_tall": ["cqr2_wide.hip", "wide_dev.h", "sync_dev.h"],
    "k_upper_image": ["cqr2_wide.hip", "wide_dev.h", "sync_dev.h"],
    "k_step": ["cqr2_step.hip", "gram_dev.h", "cholinv_dev.h", "apply_dev.h", "stream16_dev.h", "wide_dev.h",
               "sync_dev.h"],
    "k_gram16": ["cqr2_stream16.hip", "stream16_dev.h", "sync_dev.h"],
    "k_apply16": ["cqr2_stream16.hip", "stream16_dev.h", "sync_dev.h"],
    "k_fused16": ["cqr2_stream16.hip", "stream16_dev.h", "sync_dev.h"],
    "k_gram16_reduce": ["cqr2_stream16.hip", "stream16_dev.h", "sync_dev.h"],
    "k_apply256": ["cqr2_stream16.hip", "stream16_dev.h", "sync_dev.h"],
}
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_sources(kernel: str):
    return KERNEL_SOURCE.get(kernel, ["cqr2_driver.hip"])


def source_sha(kernel: str) -> str:
    """Short hash of the source files of `kernel` (cqr2_driver.hip if unlisted)."""
    h = hashlib.sha256()
    for name in kernel_sources(kernel):
        with open(os.path.join(PKG, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """'void cqr2::k_apply_rinv<128, 2>(...)' -> 'k_apply_rinv<128, 2>'."""
    base = name.split("(")[0] if not name.startswith("__") else name
    base = re.sub(r"^void\s+", "", base)
    base = base.replace("cqr2::", "")
    return base.strip()[:90]


def kernel_family(name: str) -> str:
    """Template-free kernel name: 'k_apply_rinv<128, 2>' -> 'k_apply_rinv'."""
    return short_name(name).split("<")[0]


def _find(dirpath: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(dirpath, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {dirpath}")
    return hits[0]


def stats_report(dirpath: str, command: str, library_only: bool = False) -> str:
    path = _find(dirpath, "_kernel_stats.csv")
    rows = list(csv.DictReader(open(path)))
    note = []
    if library_only:
        rows = [r for r in rows if short_name(r["Name"]).startswith("k_")]
        note = ["(this library's kernels only; the input generator's kernels are left out, so pct is of the whole run)"]
    lines = [
        "rocprofv3 kernel statistics",
        f"command: {command}",
        *note,
        "",
        f"{'kernel':<60} {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total_ms':>10} {'pct':>6}",
    ]
    for r in rows:
        calls = int(r["Calls"])
        total = float(r["TotalDurationNs"])
        avg = float(r["AverageNs"])
        lines.append(f"{short_name(r['Name'])[:60]:<60} {calls:>6} {avg / 1e3:>10.2f} "
                     f"{float(r['MinNs']) / 1e3:>10.2f} {float(r['MaxNs']) / 1e3:>10.2f} {total / 1e6:>10.3f} "
                     f"{float(r['Percentage']):>6.2f}")
    return "\n".join(lines) + "\n"


def _counter_means(dirpath: str, counter: str):
    """{kernel: (mean value per dispatch, dispatches)}; the copy kernel's entry
    is the calibration copy alone: the dispatch with the largest count (the
    calibration copy is the largest copy the program makes; its other copies,
    host-to-device staging and the 512 MB matrix copies of the mixed sweep, are
    smaller, and copies of different sizes can share one grid size)."""
    path = _find(dirpath, "_counter_collection.csv")
    vals = collections.defaultdict(list)
    copies = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        name = short_name(r["Kernel_Name"])
        if name == COPY_KERNEL:
            copies.append((int(r["Grid_Size"]), int(r["Dispatch_Id"]), float(r["Counter_Value"])))
        else:
            vals[name].append(float(r["Counter_Value"]))
    out = {k: (sum(v) / len(v), len(v)) for k, v in vals.items()}
    if copies:
        out[COPY_KERNEL] = (max(v for _, _, v in copies), 1)
    return out


def traffic_report(fetch_dir: str, write_dir: str, copy_bytes: int, cmd_fetch: str, cmd_write: str):
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")
    copy_f = fetch.get(COPY_KERNEL)
    copy_w = write.get(COPY_KERNEL)
    if copy_f is None or copy_w is None:
        raise RuntimeError("calibration copy kernel not found in the counter runs")
    # counters are in KiB per dispatch; the copy reads and writes copy_bytes
    f_scale = copy_bytes / (copy_f[0] * 1024.0)
    w_scale = copy_bytes / (copy_w[0] * 1024.0)
    kernels = {}
    for name in sorted(set(fetch) & set(write)):
        if not name.startswith("k_"):
            continue
        fam = kernel_family(name)
        rd = fetch[name][0] * 1024.0 * f_scale
        wr = write[name][0] * 1024.0 * w_scale
        kernels[fam] = {"name": name, "dispatches": fetch[name][1], "read_bytes_per_launch": rd,
                        "write_bytes_per_launch": wr, "bytes_per_launch": rd + wr,
                        "source": "+".join(kernel_sources(fam)), "source_sha": source_sha(fam)}
    data = {
        "calibration": {"copy_bytes": copy_bytes, "fetch_kib": copy_f[0], "write_kib": copy_w[0],
                        "fetch_scale": f_scale, "write_scale": w_scale},
        "commands": {"fetch": cmd_fetch, "write": cmd_write},
        "kernels": kernels,
    }
    lines = [
        "HBM traffic per dispatch from rocprofv3 counters (FETCH_SIZE, WRITE_SIZE in KiB, scaled)",
        f"command (FETCH_SIZE): {cmd_fetch}",
        f"command (WRITE_SIZE): {cmd_write}",
        f"calibration: device copy of {copy_bytes} B reads FETCH_SIZE {copy_f[0]:.1f} KiB, "
        f"WRITE_SIZE {copy_w[0]:.1f} KiB -> scale read x{f_scale:.4f}, write x{w_scale:.4f}",
        "",
        f"{'kernel':<32} {'disp':>5} {'read_MB':>10} {'write_MB':>10} {'total_MB':>10}  source@sha",
    ]
    for fam, k in kernels.items():
        lines.append(f"{k['name']:<32} {k['dispatches']:>5} {k['read_bytes_per_launch'] / 1e6:>10.2f} "
                     f"{k['write_bytes_per_launch'] / 1e6:>10.2f} {k['bytes_per_launch'] / 1e6:>10.2f}  "
                     f"{k['source']}@{k['source_sha']}")
    return data, "\n".join(lines) + "\n"


def mfma_report(dirpath: str, command: str) -> str:
    path = _find(dirpath, "_counter_collection.csv")
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        name = short_name(r["Kernel_Name"])
        if not name.startswith("k_"):
            continue
        vals[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = [
        "Matrix-core work per dispatch from rocprofv3 derived counters",
        f"command: {command}",
        "MfmaFlopsF64/F32 = SQ_INSTS_VALU_MFMA_MOPS_F64/F32 x 512; MfmaUtil = SQ_VALU_MFMA_BUSY_CYCLES /",
        "(GRBM_GUI_ACTIVE x SIMDs), in percent, over the dispatch.",
        "",
        f"{'kernel':<40} {'disp':>5} {'GFLOP_f64':>11} {'GFLOP_f32':>11} {'mfma_busy_%':>12}",
    ]
    for name in sorted(vals):
        v = vals[name]
        def mean(c):
            x = v.get(c, [])
            return sum(x) / len(x) if x else float("nan")
        disp = max(len(x) for x in v.values())
        lines.append(f"{name[:40]:<40} {disp:>5} {mean('MfmaFlopsF64') / 1e9:>11.3f} "
                     f"{mean('MfmaFlopsF32') / 1e9:>11.3f} {mean('MfmaUtil'):>12.1f}")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--library-only", action="store_true")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--out-json", required=True)
    t.add_argument("--out-txt", required=True)
    mf = sub.add_parser("mfma")
    mf.add_argument("dir")
    mf.add_argument("--command", required=True)
    mf.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "mfma":
        text = mfma_report(a.dir, a.command)
        with open(a.out, "w") as f:
            f.write(text)
        print(text)
        return
    if a.cmd == "stats":
        text = stats_report(a.dir, a.command, a.library_only)
        with open(a.out, "w") as f:
            f.write(text)
        print(text)
    else:
        data, text = traffic_report(a.fetch, a.write, a.copy_bytes, a.command_fetch, a.command_write)
        with open(a.out_json, "w") as f:
            json.dump(data, f, indent=1)
        with open(a.out_txt, "w") as f:
            f.write(text)
        print(text)


if __name__ == "__main__":
    main()

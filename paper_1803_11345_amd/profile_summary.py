"""Summaries of rocprofv3 output for the profiles/ folder.

  python -m paper_1803_11345_amd.profile_summary stats  <kernel_stats.csv> --command "..." --out X.md
  python -m paper_1803_11345_amd.profile_summary mfma <kernel_stats.csv> <counter_collection.csv>
         --command "..." --out X.md
  python -m paper_1803_11345_amd.profile_summary traffic <fetch counter_collection.csv>
         <write counter_collection.csv> --kernel k_step --copy-bytes 2147483648 --nodes N
         --bytes-per-lup B --command "..." --out X.json

``traffic`` calibrates the two TCC counters with the plain device copy that bench.py --copy-probe
runs (a copy of --copy-bytes bytes reads and writes exactly that many bytes): each counter of the
step kernel is scaled by (copy bytes / what the same counter reads for the copy).  The record
carries the SHA-256 of the kernel source, so bench.py reports the traffic only while the kernel
is the one that was measured.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "lbcm.hip")


def source_digest() -> str:
    return hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()


def _demangle(name: str) -> str:
    if not name.startswith("_Z"):
        return name
    import subprocess

    try:
        out = subprocess.run(["c++filt", name], capture_output=True, text=True, check=True).stdout.strip()
        if out != name:
            return out
    except (OSError, subprocess.CalledProcessError):
        pass
    # names c++filt does not know (bfloat16 parameters): the kernel's identifier inside the anonymous
    # namespace and its integer template arguments
    import re

    m = re.match(r"_ZN12_GLOBAL__N_1(\d+)", name)
    if not m:
        return name
    n, pos = int(m.group(1)), m.end()
    ident, pos = name[pos:pos + n], pos + n
    args = []
    if name[pos:pos + 1] == "I":
        for a in re.finditer(r"Li(-?\d+)E", name[pos + 1:]):
            if a.start() != sum(len(x) for x in args):
                break
            args.append(a.group(0))
    vals = [re.match(r"Li(-?\d+)E", x).group(1) for x in args]
    return ident + (f"<{', '.join(vals)}>" if vals else "")


def _short(name: str) -> str:
    name = _demangle(name).replace("(anonymous namespace)::", "")
    return name.split("(")[0] if not name.startswith("void ") else name[5:].split("(")[0]


def stats_md(path: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    lines = ["# Kernel time (rocprofv3 --kernel-trace --stats)", "", "Command (from /tmp, TMPDIR=/tmp):", "",
             "```", command, "```", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} % |")
    return "\n".join(lines) + "\n"


def _per_kernel(path: str, counter: str):
    out = defaultdict(list)
    grids = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        grids[r["Kernel_Name"]].append(int(r["Grid_Size"]))
    return out, grids


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, nodes: int, bytes_per_lup: int,
            command: str) -> dict:
    res = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        vals, grids = _per_kernel(path, counter)
        step = [v for k, v in vals.items() if kernel in k]
        if not step:
            raise SystemExit(f"no dispatch of {kernel} in {path}")
        step_vals = step[0]
        # the probe copy: the copy-kernel dispatches with the largest grid
        copies = [(g, v) for k in vals if "copyBuffer" in k for g, v in zip(grids[k], vals[k])]
        gmax = max(g for g, _ in copies)
        copy_vals = [v for g, v in copies if g == gmax]
        kib_copy = statistics.median(copy_vals)
        scale = (copy_bytes / 1024.0) / kib_copy
        kib = statistics.mean(step_vals)
        res[key] = {"counter": counter, "step_kib_mean": kib, "step_dispatches": len(step_vals),
                    "copy_kib_median": kib_copy, "copy_dispatches": len(copy_vals), "scale": scale,
                    "bytes_per_launch": kib * 1024.0 * scale}
    alg = nodes * bytes_per_lup
    total = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    return {"kernel": kernel, "source_sha256": source_digest(), "command": command, "nodes": nodes,
            "bytes_per_lup": bytes_per_lup, "algorithmic_bytes_per_launch": alg,
            "traffic_bytes_per_launch": total, "traffic_over_algorithmic": total / alg,
            "read_over_algorithmic": res["fetch"]["bytes_per_launch"] / (alg / 2),
            "write_over_algorithmic": res["write"]["bytes_per_launch"] / (alg / 2), **res}


# Work of the surrogate's kernels in the kernel-only workload of bench.py --sur-kernels (FLOP per
# launch counted as the MFMA computes it, padded channels and recomputed halo rings included;
# 65,536 pixels for one inference box, 524,288 for the training batch of 8), and the peak of the
# arithmetic each runs on (MI355X dense: BF16 MFMA 2.5 PFLOP/s, FP32 MFMA and vector FP32 157.3).
_PX1, _PX8 = 256 * 256, 8 * 256 * 256
_HALO = 340 / 256  # a fused pair's first layer runs on the tile plus a one-pixel ring (10 x 34 of 8 x 32)
SURROGATE_WORK = {
    "k_first_pair": (2 * _PX1 * 9 * (4 * 64 * 1.0 + 64 * 64) * _HALO, "BF16 MFMA (+ FP32 layer 0)", 2500.0),
    "k_pair<64, 0, 64>": (2 * _PX1 * 9 * 64 * 64 * (_HALO + 1), "BF16 MFMA", 2500.0),
    "k_pair<16, 3, 32>": (2 * _PX1 * 9 * (64 * 64 * _HALO + 64 * 16), "BF16 MFMA", 2500.0),
    "k_first<64, false, true>": (2 * _PX8 * 9 * 4 * 64, "FP32 MFMA", 157.3),
    "k_conv<64, 64, 0>": (2 * _PX8 * 9 * 64 * 64, "BF16 MFMA", 2500.0),
    "k_conv<64, 32, 1>": (2 * _PX8 * 9 * 64 * 32, "BF16 MFMA", 2500.0),
    "k_conv<64, 64, 2>": (2 * _PX8 * 9 * 64 * 64, "BF16 MFMA", 2500.0),
    "k_last_dgrad<64>": (2 * _PX8 * 64 * 64, "BF16 MFMA (K = 36 taps x state channels, padded to 64)", 2500.0),
    "k_conv_dw_strip<64>": (2 * _PX8 * 9 * 64 * 64, "BF16 MFMA", 2500.0),
    "k_last_dw<64>": (2 * _PX8 * 64 * 48, "BF16 MFMA (N = 36 taps x state channels, padded to 48)", 2500.0),
    "k_first_dw<64>": (3 * 2 * _PX8 * 48 * 64, "BF16 MFMA (state split in three parts, 48 columns)", 2500.0),
}


# Algorithmic HBM bytes per launch of the training kernels at batch 8 x 256^2 (each tensor once:
# BF16 activations and gradients of 64 channels 128 B per pixel, ReLU masks 16 B, FP32 states
# 16 B, the 4 state channels of the last layer's output gradient 8 B, FP32 partial sums as
# written; halo re-reads not counted), against the 8 TB/s HBM peak.
_A64, _MASK, _ST, _DZ4 = 128 * _PX8, 16 * _PX8, 16 * _PX8, 8 * _PX8
SURROGATE_BYTES = {
    "k_first<64, false, true>": _ST + _A64 + _MASK,
    "k_conv<64, 64, 0>": _A64 + _A64 + _MASK,
    "k_conv<64, 32, 1>": _A64 + _ST + _ST,
    "k_conv<64, 64, 2>": _A64 + _MASK + _A64,
    "k_last_dgrad<64>": _DZ4 + _MASK + _A64,
    "k_conv_dw_strip<64>": _A64 + _A64 + 256 * 9 * 64 * 64 * 4,
    "k_last_dw<64>": _A64 + _DZ4 + 512 * 9 * 64 * 4 * 4,
    "k_first_dw<64>": _ST + _A64 + 512 * 37 * 64 * 4,
}


def mfma_md(stats_csv: str, counters_csv: str, command: str, xcds: int = 8, simds: int = 1024) -> str:
    """Per-kernel TF/s (kernel time from a --kernel-trace --stats run) and MFMA busy fraction
    (SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / xcds x simds): the counter of GPU-active clocks
    is summed over the XCDs, the busy counter over the SIMDs) of the surrogate's kernels."""
    times = {_short(r["Name"]): (int(r["Calls"]), float(r["AverageNs"]) / 1e3) for r in csv.DictReader(open(stats_csv))}
    busy, active = defaultdict(list), defaultdict(list)
    for r in csv.DictReader(open(counters_csv)):
        k = _short(r["Kernel_Name"])
        (busy if r["Counter_Name"] == "SQ_VALU_MFMA_BUSY_CYCLES" else active)[k].append(float(r["Counter_Value"]))
    lines = ["# Surrogate kernels against their peaks", "", "Commands (from /tmp, TMPDIR=/tmp):", "", "```", command, "```", "",
             "| kernel | calls | average (us) | GFLOP per launch | TFLOP/s | unit | fraction of peak | MFMA busy |",
             "|---|---|---|---|---|---|---|---|"]
    for k, (flop, unit, peak) in SURROGATE_WORK.items():
        if k not in times:
            continue
        calls, us = times[k]
        tf = flop / us / 1e6
        mb = ""
        if busy.get(k) and active.get(k):
            mb = f"{statistics.mean(busy[k]) / (statistics.mean(active[k]) / xcds * simds):.2f}"
        lines.append(f"| `{k}` | {calls} | {us:.2f} | {flop / 1e9:.2f} | {tf:.0f} | {unit} | {tf / peak:.3f} | {mb} |")
    lines += ["", "The training kernels against HBM (algorithmic bytes: each tensor once, halo re-reads not counted):", "",
              "| kernel | MB per launch | GB/s | fraction of 8 TB/s |", "|---|---|---|---|"]
    for k, nbytes in SURROGATE_BYTES.items():
        if k not in times:
            continue
        gbs = nbytes / times[k][1] / 1e3
        lines.append(f"| `{k}` | {nbytes / 1e6:.1f} | {gbs:.0f} | {gbs / 8000:.3f} |")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--command", required=True)
    a.add_argument("--out", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--kernel", default="k_step")
    b.add_argument("--copy-bytes", type=int, default=1 << 31)
    b.add_argument("--nodes", type=int, required=True)
    b.add_argument("--bytes-per-lup", type=int, required=True)
    b.add_argument("--command", required=True)
    b.add_argument("--out", required=True)
    c = sub.add_parser("mfma")
    c.add_argument("stats_csv")
    c.add_argument("counters_csv")
    c.add_argument("--command", required=True)
    c.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.what == "mfma":
        open(args.out, "w").write(mfma_md(args.stats_csv, args.counters_csv, args.command))
        return
    if args.what == "stats":
        open(args.out, "w").write(stats_md(args.csv, args.command))
    else:
        rec = traffic(args.fetch_csv, args.write_csv, args.kernel, args.copy_bytes, args.nodes, args.bytes_per_lup,
                      args.command)
        json.dump(rec, open(args.out, "w"), indent=2)
        print(json.dumps({k: rec[k] for k in ("traffic_bytes_per_launch", "traffic_over_algorithmic",
                                               "read_over_algorithmic", "write_over_algorithmic")}))


if __name__ == "__main__":
    main()

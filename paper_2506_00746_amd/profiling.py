"""Summaries of rocprofv3 output for the library's kernels.

``python -m paper_2506_00746_amd.profiling summary --trace DIR --fetch DIR
--write DIR --kernel element_kernel --copy-bytes N --cmd "..."`` turns the CSV
output of three rocprofv3 runs of one command (``--kernel-trace --stats``,
``--pmc FETCH_SIZE``, ``--pmc WRITE_SIZE``) into a short markdown summary:
kernel statistics, and the kernel's HBM traffic per launch with each counter
scaled by what it reads for a plain device copy of known size in the same
run (the largest ``copyBuffer`` dispatch).

``kernel_source_sha256()`` fingerprints the element-kernel sources; a stored
traffic figure is only valid for the sources it was measured on.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/element_kernel.hpp", "csrc/pointwise.hpp", "csrc/dual.hpp",
                  "csrc/kernel_api.hpp"]


def kernel_source_sha256() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(_HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def kernel_stats(trace_dir: str) -> list[dict]:
    with open(_one(os.path.join(trace_dir, "**", "*kernel_stats.csv"))) as f:
        return list(csv.DictReader(f))


def counter_per_dispatch(pmc_dir: str, counter: str) -> list[tuple[str, int, float]]:
    """(kernel name, grid size, counter summed over its instances) per dispatch."""
    per = {}
    with open(_one(os.path.join(pmc_dir, "**", "*counter_collection.csv"))) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            key = int(r["Dispatch_Id"])
            name, grid, v = per.get(key, (r["Kernel_Name"], int(r["Grid_Size"]), 0.0))
            per[key] = (name, grid, v + float(r["Counter_Value"]))
    return [per[k] for k in sorted(per)]


def traffic(fetch_dir: str, write_dir: str, kernel: str, copy_bytes: int) -> dict:
    """Calibrated HBM bytes per launch of ``kernel`` (counters are in KiB)."""
    out = {}
    for name, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = counter_per_dispatch(d, counter)
        copies = [v for n, g, v in rows if "copyBuffer" in n]
        ref = max(copies)
        factor = copy_bytes / (ref * 1024.0)
        vals = [v for n, g, v in rows if re.search(kernel, n)]
        avg_kib = sum(vals) / len(vals)
        out[name] = {"counter": counter, "copy_kib": ref, "factor": factor, "kernel_kib": avg_kib,
                     "dispatches": len(vals), "bytes": avg_kib * 1024.0 * factor}
    out["bytes"] = out["fetch"]["bytes"] + out["write"]["bytes"]
    return out


def counters(pmc_dir: str, kernel: str) -> dict:
    """Every counter of one --pmc run, averaged over the dispatches of ``kernel``."""
    names = set()
    with open(_one(os.path.join(pmc_dir, "**", "*counter_collection.csv"))) as f:
        for r in csv.DictReader(f):
            names.add(r["Counter_Name"])
    out = {}
    for c in sorted(names):
        vals = [v for n, g, v in counter_per_dispatch(pmc_dir, c) if re.search(kernel, n)]
        if vals:
            out[c] = (sum(vals) / len(vals), len(vals))
    return out


# Executed floating-point operations from the VALU instruction counters: each
# counted instruction is one wavefront instruction over 64 lanes; an FMA
# counts 2, add, multiply and transcendental 1.
FLOP_WEIGHTS = {"FMA": 2, "ADD": 1, "MUL": 1, "TRANS": 1}


def executed_flops(cnt: dict, width: str) -> float | None:
    names = [f"SQ_INSTS_VALU_{k}_{width}" for k in FLOP_WEIGHTS]
    if not all(n in cnt for n in names):
        return None
    return 64.0 * sum(FLOP_WEIGHTS[k] * cnt[f"SQ_INSTS_VALU_{k}_{width}"][0] for k in FLOP_WEIGHTS)


def counter_lines(pmc_dirs: list[str], kernel: str) -> list[str]:
    cnt = {}
    for d in pmc_dirs:
        cnt.update(counters(d, kernel))
    if not cnt:
        return []
    lines = ["", f"## Counters of `{kernel}` per dispatch (--pmc, one run per counter group)", "",
             "| counter | average per dispatch | dispatches |", "|---|---|---|"]
    for c, (v, n) in sorted(cnt.items()):
        lines.append(f"| {c} | {v:.6g} | {n} |")
    derived = []
    for width in ("F64", "F32"):
        fl = executed_flops(cnt, width)
        if fl is not None:
            derived.append(f"executed_flops_{width.lower()}_per_launch: {fl:.6g}")
    if derived:
        lines += ["", "Executed FLOPs = 64 lanes x (2 FMA + ADD + MUL + TRANS) wavefront instructions:", ""]
        lines += derived
    return lines


def summary(args) -> str:
    stats = kernel_stats(args.trace)
    t = traffic(args.fetch, args.write, args.kernel, args.copy_bytes)
    lines = [f"# rocprofv3 summary: {args.title}", "", "Command (run from the repository root):", "",
             "```", *args.cmd_lines, "```", "", "## Kernel statistics (--kernel-trace --stats)", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share |",
             "|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {r['Name']} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {r['Percentage']}% |")
    lines += ["", f"## HBM traffic of `{args.kernel}` per launch (--pmc)", "",
              "| counter | plain copy reads (KiB) | scale factor | kernel (KiB/dispatch) | bytes/launch |",
              "|---|---|---|---|---|"]
    for k in ("fetch", "write"):
        x = t[k]
        lines.append(f"| {x['counter']} | {x['copy_kib']:.0f} for {args.copy_bytes} B | {x['factor']:.3f} | "
                     f"{x['kernel_kib']:.1f} ({x['dispatches']} dispatches) | {x['bytes']:.4g} |")
    lines += counter_lines(args.pmc or [], args.kernel)
    lines += ["", f"traffic_bytes_per_launch: {t['bytes']:.6g}",
              f"kernel_source_sha256: {kernel_source_sha256()}", ""]
    return "\n".join(lines)


def read_traffic(path: str):
    """(bytes per launch, source sha) recorded in a summary, or (None, None)."""
    if not os.path.exists(path):
        return None, None
    txt = open(path).read()
    b = re.search(r"^traffic_bytes_per_launch: ([0-9.eE+-]+)$", txt, re.M)
    h = re.search(r"^kernel_source_sha256: ([0-9a-f]+)$", txt, re.M)
    return (float(b.group(1)) if b else None), (h.group(1) if h else None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["summary", "sha"])
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel", default="element_kernel")
    ap.add_argument("--copy-bytes", type=int, default=256 * 1024 * 1024)
    ap.add_argument("--title", default="")
    ap.add_argument("--cmd", action="append", dest="cmd_lines", default=[])
    ap.add_argument("--pmc", action="append", default=[], help="directory of a further --pmc run (repeatable)")
    args = ap.parse_args()
    if args.what == "sha":
        print(kernel_source_sha256())
    else:
        print(summary(args))


if __name__ == "__main__":
    main()

"""Summaries of rocprofv3 output for the sparse FFT kernels.

    python -m paper_1201_2501_amd.prof trace-summary --trace T_kernel_trace.csv \
        --stats T_kernel_stats.csv --command "..." > summary.md
    python -m paper_1201_2501_amd.prof traffic --fetch F_counter_collection.csv \
        --write W_counter_collection.csv --config KEY --signals 512 --command "..." > traffic.json

trace-summary: per kernel and grid size, the number of launches and their
mean/min/max duration (from the kernel trace), then the profiler's own
per-kernel statistics table.

traffic: HBM bytes of the HashToBins pair launch of a batched step, from one
FETCH_SIZE and one WRITE_SIZE counter run (kilobytes per dispatch).  Each
counter is calibrated on the 1 GiB device-to-device copy that the bench runs
first with --copy-calibration (1 GiB read and 1 GiB written; the runtime's
copyBuffer kernel, the first one above 128 MiB): factor = 2^30 bytes /
counter bytes of that copy.  The pair launch taken is the
largest-grid k_h2b_pair dispatch (the first round group, hashed for every
signal).
"""
import argparse
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(PKG, "csrc", f) for f in ("sfft_kernels.hip", "sfft_common.hpp", "sfft_internal.hpp")]
COPY_BYTES = 1 << 30


def kernel_source_hash():
    """Hash of the sources the HashToBins pair kernel is built from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def short_name(name):
    """Kernel name without return type, anonymous-namespace marker and arguments."""
    name = name.replace("void ", "").replace("(anonymous namespace)::", "")
    return name.split("(")[0]


def trace_summary(trace_csv, stats_csv, command):
    rows = list(csv.DictReader(open(trace_csv)))
    groups = defaultdict(list)
    for r in rows:
        if "sfft" not in r["Kernel_Name"]:
            continue
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        groups[(short_name(r["Kernel_Name"]), int(r["Grid_Size_X"]))].append(dur)
    out = ["# rocprofv3 kernel trace: sparse FFT kernels", "", "Command:", "", "    " + command, "",
           "Per kernel and grid size (threads), from the kernel trace:", "",
           "| kernel | grid | launches | mean us | min us | max us |", "|---|---|---|---|---|---|"]
    for (name, grid), ds in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        out.append("| %s | %d | %d | %.1f | %.1f | %.1f |" % (name, grid, len(ds), sum(ds) / len(ds), min(ds), max(ds)))
    out += ["", "rocprofv3 --stats (all kernels of the run):", "", "```"]
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            out.append("%-70s calls %6s  avg %12.1f ns  total %6.2f%%" % (
                short_name(r["Name"])[:70], r["Calls"], float(r["AverageNs"]), float(r["Percentage"])))
    out.append("```")
    return "\n".join(out) + "\n"


def counter_rows(path, counter):
    rows = []
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") == counter:
            rows.append(r)
    return rows


def kib_of(rows, pred):
    """Counter value (KiB) of the dispatches matching pred, largest grid first."""
    sel = [r for r in rows if pred(r)]
    sel.sort(key=lambda r: -int(r["Grid_Size"]))
    return sel


def traffic(fetch_csv, write_csv, config, signals, command):
    rec = {"source_hash": kernel_source_hash(), "config": config, "signals": signals, "command": command}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = counter_rows(path, counter)
        # the calibration copy: the first runtime copy kernel above 128 MiB
        copy = [r for r in rows if "copyBuffer" in r["Kernel_Name"] and float(r["Counter_Value"]) > 2 ** 17]
        copy.sort(key=lambda r: int(r["Dispatch_Id"]))
        pair = kib_of(rows, lambda r: "k_h2b_pair" in r["Kernel_Name"])
        if not copy or not pair:
            raise SystemExit("%s: no copy or k_h2b_pair dispatch with %s" % (path, counter))
        copy_kib = float(copy[0]["Counter_Value"])
        pair_kib = float(pair[0]["Counter_Value"])
        factor = COPY_BYTES / (copy_kib * 1024.0)
        rec[key] = {"copy_kernel": short_name(copy[0]["Kernel_Name"])[:80], "copy_KiB": copy_kib,
                    "factor": factor, "pair_grid": int(pair[0]["Grid_Size"]), "pair_KiB": pair_kib,
                    "pair_bytes": pair_kib * 1024.0 * factor}
    rec["bytes_per_launch"] = rec["fetch"]["pair_bytes"] + rec["write"]["pair_bytes"]
    rec["bytes_per_signal"] = rec["bytes_per_launch"] / signals
    return json.dumps(rec, indent=1) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace-summary")
    t.add_argument("--trace", required=True)
    t.add_argument("--stats", required=True)
    t.add_argument("--command", required=True)
    c = sub.add_parser("traffic")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--config", required=True)
    c.add_argument("--signals", type=int, required=True)
    c.add_argument("--command", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "trace-summary":
        sys.stdout.write(trace_summary(a.trace, a.stats, a.command))
    else:
        sys.stdout.write(traffic(a.fetch, a.write, a.config, a.signals, a.command))


if __name__ == "__main__":
    main()

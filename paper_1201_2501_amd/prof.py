"""Summaries of rocprofv3 output for the sparse FFT kernels.

    python -m paper_1201_2501_amd.prof trace-summary --trace T_kernel_trace.csv \
        --stats T_kernel_stats.csv --command "..." > summary.md
    python -m paper_1201_2501_amd.prof traffic --counters A_counter_collection.csv \
        B_counter_collection.csv --config KEY --signals 512 --samples S --command "..." > traffic.json

trace-summary: per kernel and grid size, the number of launches and their
mean/min/max duration (from the kernel trace), then the profiler's own
per-kernel statistics table.

traffic: L2-to-fabric traffic of the HashToBins pair launch of a batched
step, from request counts by size: one counter run with TCC_EA0_RDREQ,
TCC_EA0_RDREQ_32B, TCC_BUBBLE and TCC_EA0_RDREQ_DRAM, one with
TCC_EA0_WRREQ, TCC_EA0_WRREQ_64B, TCC_MISS and TCC_REQ (summed over the L2
channels of every XCD, per dispatch).  The same counts of the 1 GiB
device-to-device copy that the bench runs first with --copy-calibration
(the runtime's copyBuffer kernel, the first with more than 2^22 read
requests) show what a counted read request carries there: 2^30 bytes /
requests.  Read requests are counted once whatever their size (32 B
flagged by RDREQ_32B, 128 B by BUBBLE); gfx950 does not flag the copy's
full-line reads as 128 B, so a read request of the pair kernel is taken as
64 B (the low reading) to the copy's bytes per request (the high one).
Write bytes: 64 B per WRREQ_64B, 32 B per other write request.  The pair
launch taken is the largest-grid k_h2b_pair dispatch (the first round
group, hashed for every signal).
"""
import argparse
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(PKG, "csrc", f) for f in ("sfft_kernels.hip", "sfft_pair.hpp", "sfft_common.hpp",
                                                          "sfft_internal.hpp")]
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


def counter_values(paths):
    """{(kernel, dispatch, grid): {counter: value}} over the counter files."""
    out = defaultdict(dict)
    for path in paths:
        for r in csv.DictReader(open(path)):
            key = (r["Kernel_Name"], int(r["Dispatch_Id"]), int(r["Grid_Size"]))
            out[key][r["Counter_Name"]] = out[key].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def _c(vals, name):
    return vals.get(name, vals.get(name + "_sum", 0.0))


def request_summary(vals):
    rd, rd32, rd128 = _c(vals, "TCC_EA0_RDREQ"), _c(vals, "TCC_EA0_RDREQ_32B"), _c(vals, "TCC_BUBBLE")
    wr, wr64 = _c(vals, "TCC_EA0_WRREQ"), _c(vals, "TCC_EA0_WRREQ_64B")
    return {"rd_req": rd, "rd_req_32B": rd32, "rd_req_128B": rd128, "rd_req_dram": _c(vals, "TCC_EA0_RDREQ_DRAM"),
            "wr_req": wr, "wr_req_64B": wr64, "l2_req": _c(vals, "TCC_REQ"), "l2_miss": _c(vals, "TCC_MISS"),
            "wr_bytes": 64.0 * wr64 + 32.0 * (wr - wr64)}


def traffic(paths, config, signals, samples, command):
    vals = counter_values(paths)
    copies = sorted((k for k in vals if "copyBuffer" in k[0] and _c(vals[k], "TCC_EA0_RDREQ") > 2 ** 22),
                    key=lambda k: k[1])
    pairs = sorted((k for k in vals if "k_h2b_pair" in k[0]), key=lambda k: -k[2])
    if not copies or not pairs:
        raise SystemExit("no calibration copy or k_h2b_pair dispatch in the counter files")
    copy, pair = request_summary(vals[copies[0]]), request_summary(vals[pairs[0]])
    copy_bpr = COPY_BYTES / copy["rd_req"]
    rd = pair["rd_req"] - pair["rd_req_32B"] - pair["rd_req_128B"]
    low = 32.0 * pair["rd_req_32B"] + 64.0 * rd + 128.0 * pair["rd_req_128B"]
    high = 32.0 * pair["rd_req_32B"] + copy_bpr * rd + 128.0 * pair["rd_req_128B"]
    rec = {"source_hash": kernel_source_hash(), "config": config, "signals": signals, "command": command,
           "copy": {"kernel": short_name(copies[0][0])[:80], "bytes_read": COPY_BYTES, **copy,
                    "bytes_per_read_req": copy_bpr},
           "pair": {"grid": pairs[0][2], **pair, "gathered_samples": samples,
                    "rd_req_per_sample": pair["rd_req"] / samples if samples else None,
                    "read_bytes_low": low, "read_bytes_high": high},
           "bytes_per_launch": low + pair["wr_bytes"], "bytes_per_launch_high": high + pair["wr_bytes"]}
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
    c.add_argument("--counters", required=True, nargs="+", help="counter_collection.csv of each counter run")
    c.add_argument("--config", required=True)
    c.add_argument("--signals", type=int, required=True)
    c.add_argument("--samples", type=int, required=True, help="gathered samples of the pair launch")
    c.add_argument("--command", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "trace-summary":
        sys.stdout.write(trace_summary(a.trace, a.stats, a.command))
    else:
        sys.stdout.write(traffic(a.counters, a.config, a.signals, a.samples, a.command))


if __name__ == "__main__":
    main()

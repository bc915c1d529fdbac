"""Reduce rocprofv3 output of a benchmark workload to the per-launch counter
profile that bench.py reads (profiles/counters_<workload>.json).

  python -m paper_1402_2773_amd.profile_summary --workload mix4 \\
      --classes CLS.csv --issue ISSUE.csv --fetch FETCH.csv --write WRITE.csv \\
      --trace STATS.csv [--lds LDS.csv]

Inputs are rocprofv3 ``*_counter_collection.csv`` files (one run per counter
set: the vector-ALU instruction classes, the issue counters, FETCH_SIZE,
WRITE_SIZE, optionally the LDS counters) and the ``*_kernel_stats.csv`` of a
kernel-trace run.
Every dispatch of one decode-kernel instance in such a run decodes the same
frames, so the median over its dispatches is its per-launch figure.  HBM
bytes are scaled by what the same counter reads for the plain 1 GiB device
copy that ``bench.py --copy-calibration-mib 1024`` runs first.
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# decode-kernel template arguments (waves per frame, quads per lane) -> code
MIX4_INSTANCES = {(1, 1): "C96", (1, 4): "C1008", (2, 4): "C2048", (4, 4): "C4000"}


def dispatches(path):
    """{dispatch id: {"kernel": name, counter: value summed over dimensions}}."""
    out = collections.OrderedDict()
    with open(path) as f:
        for r in csv.DictReader(f):
            d = out.setdefault(int(r["Dispatch_Id"]), {"kernel": r["Kernel_Name"],
                                                       "workgroup_size": r.get("Workgroup_Size")})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def instance_key(kernel: str):
    m = re.search(r"decode_kernel<(\d+), (\d+), (\d+), (false|true), (false|true), (\d+)>", kernel)
    return (int(m.group(1)), int(m.group(2))) if m else None


def per_instance(path, codes):
    """Median per-launch value of every counter, per decode-kernel instance."""
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in dispatches(path).values():
        key = instance_key(d["kernel"])
        if key is None or key not in codes:
            continue
        for k, v in d.items():
            if k == "workgroup_size":
                if v not in (None, ""):
                    vals[codes[key]][k].append(int(float(v)))
            elif k != "kernel":
                vals[codes[key]][k].append(v)
    return {code: {k: statistics.median(v) for k, v in cs.items()} for code, cs in vals.items()}, vals


def copy_scale(path, counter, copy_bytes):
    """Bytes per counter unit for this counter: the 1 GiB copy's reading."""
    for d in dispatches(path).values():
        if "copyBuffer" in d["kernel"] and counter in d:
            return copy_bytes / d[counter], d[counter]
    return None, None


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--classes", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--trace")
    ap.add_argument("--issue", help="counter CSV of the issue pass (SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_VALU2)")
    ap.add_argument("--lds")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--commands", default="", help="JSON object of the commands that made the inputs")
    args = ap.parse_args(argv)

    import bench

    if args.workload == "mix4":
        codes = MIX4_INSTANCES
    else:
        name = bench.WORKLOADS[args.workload][0]
        codes = {k: name for k in [(w, q) for w in (1, 2, 4, 8, 16) for q in (1, 2, 4)]}
    inst, raw = per_instance(args.classes, codes)
    result = {"workload": args.workload, "kernel_sources_sha256": bench.kernel_sources_digest(),
              "commands": json.loads(args.commands) if args.commands else {},
              "dispatches_per_instance": {c: len(v["SQ_INSTS_VALU"]) for c, v in raw.items()},
              "instances": {}}
    for code, cs in inst.items():
        result["instances"][code] = {k: v for k, v in cs.items() if k.startswith("SQ_") or k.startswith("GRBM")}
        if "workgroup_size" in cs:  # threads per workgroup of the profiled launches
            result["instances"][code]["workgroup_size"] = int(cs["workgroup_size"])
        result["instances"][code]["source"] = ("rocprofv3 SQ counters (VALU instruction classes; issue slots "
                                               "SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_VALU2), median per launch")
    if args.fetch and args.write:
        fs, fraw = copy_scale(args.fetch, "FETCH_SIZE", args.copy_bytes)
        ws, wraw = copy_scale(args.write, "WRITE_SIZE", args.copy_bytes)
        result["copy_calibration"] = {"bytes": args.copy_bytes, "FETCH_SIZE": fraw, "WRITE_SIZE": wraw,
                                      "fetch_bytes_per_unit": fs, "write_bytes_per_unit": ws}
        fi, _ = per_instance(args.fetch, codes)
        wi, _ = per_instance(args.write, codes)
        for code in result["instances"]:
            if code in fi and code in wi and fs and ws:
                fb, wb = fi[code]["FETCH_SIZE"] * fs, wi[code]["WRITE_SIZE"] * ws
                result["instances"][code].update(fetch_bytes=fb, write_bytes=wb, traffic_bytes=fb + wb)
    if args.issue:
        ii, _ = per_instance(args.issue, codes)
        for code in result["instances"]:
            if code in ii:
                for k, v in ii[code].items():
                    if k.startswith("SQ_ACTIVE_INST") or k == "SQ_BUSY_CYCLES":
                        result["instances"][code][k] = v
                result["instances"][code]["GRBM_GUI_ACTIVE_issue_pass"] = ii[code].get("GRBM_GUI_ACTIVE")
    if args.lds:
        li, _ = per_instance(args.lds, codes)
        for code in result["instances"]:
            if code in li:
                result["instances"][code]["lds"] = li[code]
    if args.trace:
        with open(args.trace) as f:
            for r in csv.DictReader(f):
                key = instance_key(r["Name"])
                if key in codes and codes[key] in result["instances"]:
                    result["instances"][codes[key]]["trace_calls"] = int(r["Calls"])
                    result["instances"][codes[key]]["trace_avg_ms"] = float(r["AverageNs"]) / 1e6
    json.dump(result, sys.stdout, indent=1, sort_keys=True)
    print()
    return 0


if __name__ == "__main__":
    sys.exit(main())

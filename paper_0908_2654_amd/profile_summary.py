"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

Three subcommands (no GPU needed; they only read CSV files):

  stats    kernel_stats.csv of a ``rocprofv3 --kernel-trace --stats`` run
           -> markdown table (calls, average and total time, share)
  markers  marker_api_stats.csv of a ``rocprofv3 --marker-trace --stats``
           run -> markdown table of the library's ROCTx ranges (host time
           from a range's start to its end: the enqueues of a phase plus
           the waits for the GPU inside it)
  traffic  counter_collection.csv of two ``--pmc FETCH_SIZE`` /
           ``--pmc WRITE_SIZE`` runs of the benchmark and of the plain
           copy (``bench.py --copy-calibration``) -> JSON record of HBM
           bytes per launch of one kernel, scaled by what the counters read
           for the copy's known 1 GiB read + 1 GiB write.  bench.py reports
           it as roofline.traffic while the kernel source is unchanged
           (the record carries the source's SHA-256).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the sources a traffic record depends on (its hash goes stale when they change)
KERNEL_SRCS = [os.path.join(ROOT, "paper_0908_2654_amd", "csrc", f)
               for f in ("rh_kernels.hip", "rh_advect.hip", "rh_device.h")]


def kernels_sha256() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _short(name: str) -> str:
    name = name.replace("void ", "").replace("rh::", "").replace("(anonymous namespace)::", "")
    return name.split("(")[0]


def stats_table(path: str, top: int = 25) -> str:
    rows = list(csv.DictReader(open(path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | average ms | total ms | % of GPU time |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        tot = float(r["TotalDurationNs"])
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                   f"{tot / 1e6:.1f} | {100 * tot / total:.1f} |")
    return "\n".join(out)


def markers_table(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| range | calls | average ms | total ms |", "|---|---|---|---|"]
    for r in rows:
        out.append(f"| {r['Name']} | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.1f} |")
    return "\n".join(out)


def _counter(path: str, counter: str, kernel_re: str | None):
    vals = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        if kernel_re is not None and not re.search(kernel_re, r["Kernel_Name"]):
            continue
        vals.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return vals


def traffic_record(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, kernel_re, kind,
                   workload, cells, algorithmic_bytes_per_cell, commands):
    f = [v for _, v in _counter(fetch_csv, "FETCH_SIZE", kernel_re)]
    w = [v for _, v in _counter(write_csv, "WRITE_SIZE", kernel_re)]
    if not f or not w:
        raise SystemExit(f"no dispatches of {kernel_re!r} in the counter files")
    names = {n for n, _ in _counter(fetch_csv, "FETCH_SIZE", kernel_re)}
    cf = [v for n, v in _counter(copy_fetch_csv, "FETCH_SIZE", None) if "copyBuffer" in n]
    cw = [v for n, v in _counter(copy_write_csv, "WRITE_SIZE", None) if "copyBuffer" in n]
    copy_bytes = 1 << 30
    fetch_scale = copy_bytes / (1024.0 * sum(cf) / len(cf))
    write_scale = copy_bytes / (1024.0 * sum(cw) / len(cw))
    fk, wk = sum(f) / len(f), sum(w) / len(w)
    per_launch = 1024.0 * (fk * fetch_scale + wk * write_scale)
    sha = kernels_sha256()
    return {
        "kernel": sorted(names)[0] if len(names) == 1 else sorted(names),
        "class": kind,
        "workload": workload,
        "fetch_kib_per_dispatch": round(fk, 1),
        "write_kib_per_dispatch": round(wk, 1),
        "dispatches": len(f),
        "copy_calibration": {"bytes_read": copy_bytes, "bytes_written": copy_bytes,
                             "fetch_kib": round(sum(cf) / len(cf), 1),
                             "write_kib": round(sum(cw) / len(cw), 1),
                             "fetch_scale": round(fetch_scale, 4),
                             "write_scale": round(write_scale, 4)},
        "traffic_bytes_per_launch": int(per_launch),
        "traffic_bytes_per_cell": round(per_launch / cells, 2),
        "algorithmic_bytes_per_cell": algorithmic_bytes_per_cell,
        "kernels_source_sha256": sha,
        "commands": commands,
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=25)
    m = sub.add_parser("markers")
    m.add_argument("csv")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--kernel", required=True, help="regular expression on the kernel name")
    t.add_argument("--class", dest="kind", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--cells", type=int, required=True)
    t.add_argument("--algorithmic", type=float, required=True)
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_table(a.csv, a.top))
        return 0
    if a.cmd == "markers":
        print(markers_table(a.csv))
        return 0
    rec = traffic_record(a.fetch, a.write, a.copy_fetch, a.copy_write, a.kernel, a.kind,
                         a.workload, a.cells, a.algorithmic, a.command)
    with open(a.out, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps({k: rec[k] for k in ("traffic_bytes_per_cell", "dispatches")}))
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_1502_01629_amd.profiling stats   <kernel_stats.csv> <out.md> "<command>"
    python -m paper_1502_01629_amd.profiling traffic <fetch.csv> <write.csv> <copy_fetch.csv> <copy_write.csv>
                                                     <copy_bytes> <kernel substring> <name> "<command>"

`traffic` scales the per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) of the kernel by what the same
counters read for a plain device copy of copy_bytes, and records the result in
profiles/traffic.json together with a hash of the kernel sources (bench.py reports it only while
the sources are unchanged).
"""
from __future__ import annotations

import csv
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def kernel_stats_markdown(path: str, command: str, top: int = 12) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
           "| kernel | calls | total ms | average us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"].split("(")[0].replace("|", "/")
        out.append(f"| `{name[:90]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def counter_means(path: str, counter: str) -> dict:
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def _pick(means: dict, sub: str) -> float:
    keys = [k for k in means if sub in k]
    if not keys:
        raise KeyError(sub)
    return means[keys[0]]


def write_traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes: int, kernel_sub: str, name: str,
                  command: str) -> dict:
    sys.path.insert(0, ROOT)
    import bench  # noqa: E402 (only for the source hash)

    f = _pick(counter_means(fetch_csv, "FETCH_SIZE"), kernel_sub)
    w = _pick(counter_means(write_csv, "WRITE_SIZE"), kernel_sub)
    cf = max(counter_means(copy_fetch_csv, "FETCH_SIZE").values())
    cw = max(counter_means(copy_write_csv, "WRITE_SIZE").values())
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    entry = {"fetch_kib": f, "write_kib": w, "fetch_scale": f_scale, "write_scale": w_scale,
             "bytes_per_launch": f * 1024.0 * f_scale + w * 1024.0 * w_scale,
             "source_hash": bench.kernel_source_hash(), "command": command}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    data = {}
    if os.path.exists(path):
        data = json.load(open(path))
    data[name] = entry
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    return entry


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        open(sys.argv[3], "w").write(kernel_stats_markdown(sys.argv[2], sys.argv[4]))
    elif sys.argv[1] == "traffic":
        print(write_traffic(*sys.argv[2:6], int(sys.argv[6]), sys.argv[7], sys.argv[8], sys.argv[9]))
    else:
        raise SystemExit(__doc__)

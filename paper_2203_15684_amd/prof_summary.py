"""Summaries of rocprofv3 CSV output for the profiles/ folder.

  python -m paper_2203_15684_amd.prof_summary stats DIR [--top N]
      kernel-trace statistics (the *_kernel_stats.csv of --kernel-trace --stats):
      per kernel: calls, total and average duration.
  python -m paper_2203_15684_amd.prof_summary pmc DIR [DIR ...]
      per kernel and counter (the *_counter_collection.csv of --pmc runs): dispatches,
      mean and max of the per-dispatch value.
  python -m paper_2203_15684_amd.prof_summary traffic --kernel NAME --match SUBSTR
      --workload W --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --items N
      HBM bytes of the dispatches of one kernel that process every item (the maximum
      over dispatches), each counter scaled by what it reads for a plain device copy of
      known size (calib_copy.py), as a per-item figure; writes profiles/traffic_NAME_W.json
      with the hash of the kernel's sources, so that the benchmark drops it once they change.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = {"plane_vloc": ["fft.hip", "hp_internal.h"], "plane_vloc32": ["fft.hip", "hp_internal.h"],
           "zproj": ["la.hip", "hp_internal.h"], "zexpand": ["la.hip", "hp_internal.h"],
           "zproj32": ["la.hip", "hp_internal.h"], "zexpand32": ["la.hip", "hp_internal.h"]}


def short(name):
    name = name.replace("void ", "").replace("(anonymous namespace)::", "").replace("hp::", "")
    name = re.sub(r"\(.*$", "", name)
    return name.replace("HIP_vector_type<float, 2u>", "float2").replace("HIP_vector_type<double, 2u>", "double2")


def rows(pattern):
    out = []
    for f in sorted(glob.glob(pattern, recursive=True)):
        with open(f, newline="") as fh:
            out += list(csv.DictReader(fh))
    return out


def stats(d, top):
    rs = rows(os.path.join(d, "**", "*kernel_stats.csv"))
    if not rs:
        raise SystemExit(f"no kernel_stats.csv under {d}")
    rs.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rs)
    print("| kernel | calls | total ms | avg ms | % |\n|---|---:|---:|---:|---:|")
    for r in rs[:top]:
        print(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.1f} | "
              f"{float(r['AverageNs']) / 1e6:.4f} | {100 * float(r['TotalDurationNs']) / tot:.1f} |")


def pmc_table(dirs):
    acc = defaultdict(list)
    for d in dirs:
        for r in rows(os.path.join(d, "**", "*counter_collection.csv")):
            acc[(short(r["Kernel_Name"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
    return acc


def pmc(dirs):
    acc = pmc_table(dirs)
    print("| kernel | counter | dispatches | mean | max |\n|---|---|---:|---:|---:|")
    for (k, c), v in sorted(acc.items()):
        print(f"| `{k}` | {c} | {len(v)} | {sum(v) / len(v):.6g} | {max(v):.6g} |")


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2203_15684_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic(a):
    def max_of(d, counter, match):
        vals = [v for (k, c), vs in pmc_table([d]).items() if c == counter and match in k for v in vs]
        if not vals:
            raise SystemExit(f"no {counter} rows for {match!r} under {d}")
        return max(vals)

    copy_bytes = float(a.copy_bytes)
    fs = copy_bytes / 1024 / max_of(a.copy_fetch, "FETCH_SIZE", "copy")   # a copy reads its size once
    ws = copy_bytes / 1024 / max_of(a.copy_write, "WRITE_SIZE", "copy")       # ... and writes it once
    fetch = max_of(a.fetch, "FETCH_SIZE", a.match)
    write = max_of(a.write, "WRITE_SIZE", a.match)
    per_item = (fetch * round(fs, 2) + write * round(ws, 2)) * 1024 / a.items
    rec = {"kernel": a.kernel, "workload": a.workload, "source_files": SOURCES[a.kernel],
           "source_hash": source_hash(SOURCES[a.kernel]), "fetch_scale": round(fs, 2), "write_scale": round(ws, 2),
           "full_launch_items": a.items, "full_launch_fetch_kib_raw": fetch, "full_launch_write_kib_raw": write,
           "bytes_per_item": per_item}
    path = os.path.join(ROOT, "profiles", f"traffic_{a.kernel}_{a.workload}.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--top", type=int, default=20)
    p = sub.add_parser("pmc")
    p.add_argument("dirs", nargs="+")
    t = sub.add_parser("traffic")
    for k in ("kernel", "match", "workload", "fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--items", type=int, required=True)
    t.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    a = ap.parse_args()
    if a.cmd == "stats":
        stats(a.dir, a.top)
    elif a.cmd == "pmc":
        pmc(a.dirs)
    else:
        traffic(a)


if __name__ == "__main__":
    sys.exit(main())

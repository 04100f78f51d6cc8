"""Summarise rocprofv3 CSV output of bench.py runs (kernel stats and
FETCH_SIZE / WRITE_SIZE counters) into the text tables kept under profiles/.

Usage (from the repository root, on the CSV directories written by the
commands quoted in the generated file):
    python -m paper_1811_11558_amd.profile_summary stats <kernel_stats.csv>
    python -m paper_1811_11558_amd.profile_summary traffic <fetch.csv> <write.csv> <copy_fetch.csv> <copy_write.csv> <copy_bytes>
The traffic mode scales each counter by the bytes a plain device copy of
known size moves per counted KiB, and reports bytes per launch per kernel.
"""
import csv
import re
import sys
from collections import defaultdict


def short(name):
    name = name.replace("void fvim::(anonymous namespace)::", "")
    return re.sub(r"\(.*\)$", "", name)


def stats(path):
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | average (us) | share |", "|---|---|---|---|"]
    for r in rows:
        out.append("| `%s` | %s | %.2f | %.1f %% |" % (short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3,
                                                     float(r["Percentage"])))
    return "\n".join(out)


def per_kernel(path):
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        acc[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return acc


def traffic(fetch, write, cfetch, cwrite, copy_bytes):
    f, w = per_kernel(fetch), per_kernel(write)
    cf, cw = per_kernel(cfetch), per_kernel(cwrite)
    copy_name = max(cf, key=lambda k: max(cf[k]))          # the large copy kernel
    fs = copy_bytes / max(cf[copy_name])                   # bytes per counted unit (reads)
    ws = copy_bytes / max(cw[copy_name])                   # bytes per counted unit (writes)
    out = ["copy reference `%s`: %d bytes read and written; FETCH_SIZE %.1f, WRITE_SIZE %.1f "
           "-> %.1f / %.1f bytes per unit" % (copy_name, copy_bytes, max(cf[copy_name]), max(cw[copy_name]), fs, ws),
           "", "| kernel | launches | fetched MB / launch | written MB / launch |", "|---|---|---|---|"]
    res = {}
    for k in sorted(f, key=lambda k: -max(f[k])):
        if k not in w:
            continue
        fm = sorted(f[k])[len(f[k]) // 2] * fs
        wm = sorted(w[k])[len(w[k]) // 2] * ws
        res[k] = (fm, wm)
        out.append("| `%s` | %d | %.1f | %.1f |" % (k, len(f[k]), fm / 1e6, wm / 1e6))
    return "\n".join(out), res


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
    else:
        text, _ = traffic(*sys.argv[2:6], int(sys.argv[6]))
        print(text)

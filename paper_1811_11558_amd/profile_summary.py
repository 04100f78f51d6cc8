"""Summarise rocprofv3 CSV output of bench.py runs into the text tables kept
under profiles/ and into profiles/traffic.json (read by bench.py).

Usage (from the repository root):
    python -m paper_1811_11558_amd.profile_summary stats <kernel_stats.csv>
    python -m paper_1811_11558_amd.profile_summary kernels --title T --stats S.csv \\
        --trace T.csv --commands commands.txt --out profiles/NAME.md
    python -m paper_1811_11558_amd.profile_summary report --workload 256x256x64/fp64 \\
        --stats S.csv --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \\
        --copy-bytes 400000000 [--raw-read R1.csv --raw-write R2.csv] [--sq SQ.csv] \\
        --commands commands.txt --out profiles/NAME.md --traffic profiles/traffic.json

Byte accounting.  FETCH_SIZE and WRITE_SIZE are scaled by what they read for
a plain device copy of known size (bytes per counted unit).  On gfx950 the
FETCH_SIZE expression counts a 128-byte read request as 64 bytes (its
128-byte term reads TCC_BUBBLE, which stays 0 there), so the copy factor is
2 for reads; that factor is right for a kernel whose reads are 128-byte
requests like the copy's.  When the raw request counters are given, bytes
are also formed directly, 128 TCC_EA0_RDREQ_128B + 64 (the other requests)
+ 32 TCC_EA0_RDREQ_32B for reads and 64 TCC_EA0_WRREQ_64B + 32 (the rest)
for writes, and both figures are listed.
"""
import argparse
import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1811_11558_amd", "csrc")

# kernel source of each stage; the hash also covers the shared headers
FFT_SOURCES = ("fft.hip", "fft_dev.hpp")
DEPTH_SOURCES = ("depth.hip", "depth_dev.hpp")
SOURCE_OF_STAGE = {"x_fwd": FFT_SOURCES, "y_fwd": FFT_SOURCES, "x_fwd_t": FFT_SOURCES, "y_fwd_t": FFT_SOURCES,
                   "depth": DEPTH_SOURCES, "depth_nyq": DEPTH_SOURCES, "y_inv": FFT_SOURCES, "x_inv": FFT_SOURCES}
HEADERS = ("common.hpp", "kernels.hpp")


def source_sha(names):
    """Hash of the files that hold a stage's kernels (the launching
    translation unit and its device bodies) and of the shared headers."""
    h = hashlib.sha256()
    for f in tuple(names) + HEADERS:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name):
    name = name.replace("void ", "", 1) if name.startswith("void ") else name
    name = name.replace("fvim::(anonymous namespace)::", "")
    return re.sub(r"\(.*\)$", "", name).strip()


def stats_rows(path):
    return [(short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["Percentage"]))
            for r in csv.DictReader(open(path))]


def stats(path):
    out = ["| kernel | calls | average (us) | share |", "|---|---|---|---|"]
    for n, c, us, pct in stats_rows(path):
        out.append("| `%s` | %d | %.2f | %.1f %% |" % (n, c, us, pct))
    return "\n".join(out)


def trace_table(path):
    """Average duration per (kernel, grid) from a --kernel-trace CSV, with the
    VGPR count and scratch size of the launch."""
    acc = defaultdict(list)
    meta = {}
    for r in csv.DictReader(open(path)):
        k = (short(r["Kernel_Name"]), int(r["Grid_Size_X"]))
        acc[k].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        meta[k] = (r["VGPR_Count"], r["Scratch_Size"], r["LDS_Block_Size"])
    out = ["VGPRs: the trace's VGPR_Count, which on gfx950 is half the register count of the code object "
           "(the depth pass's 84 is 168 registers, 3 waves per SIMD).", "",
           "| kernel | grid (threads) | launches | average (us) | VGPRs | scratch (B) | LDS (B) |",
           "|---|---|---|---|---|---|---|"]
    for k in sorted(acc, key=lambda k: -sum(acc[k])):
        v = acc[k]
        out.append("| `%s` | %d | %d | %.2f | %s | %s | %s |" % (k[0], k[1], len(v), sum(v) / len(v), *meta[k]))
    return "\n".join(out)


def dispatches(path):
    """{(kernel, grid): {counter: [values per dispatch]}}"""
    acc = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(path)):
        acc[(short(r["Kernel_Name"]), int(r["Grid_Size"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return acc


def median(v):
    v = sorted(v)
    return v[len(v) // 2]


def stage_keys(keys, launches=None):
    """Map (kernel, grid) keys of one operator run to bench stages.  With
    launches ({kernel name: launches} of the timed run's trace) each
    transform stage takes the instance launched most there (the tuners'
    candidates run only a few times), else the largest grid."""
    by = defaultdict(list)
    for k in keys:
        by[k[0].split("<")[0]].append(k)
    st = {}
    for base, name in (("k_x_r2c", "x_fwd"), ("k_y_fwd", "y_fwd"), ("k_y_inv", "y_inv"), ("k_x_c2r", "x_inv")):
        ks = by.get(base, [])
        if not ks:
            continue
        if launches:
            named = [k for k in ks if launches.get(k[0], 0) == max(launches.get(j[0], 0) for j in ks)]
            if named:
                ks = named
        st[name] = sorted(ks, key=lambda k: -k[1])[0]
    return st, by.get("k_depth", [])


def copy_factor(path, counter, copy_bytes):
    d = dispatches(path)
    name = max(d, key=lambda k: max(d[k].get(counter, [0])))
    return copy_bytes / max(d[name][counter]), name[0], max(d[name][counter])


def report(a):
    fetch, write = dispatches(a.fetch), dispatches(a.write)
    fs, copy_name, cf = copy_factor(a.copy_fetch, "FETCH_SIZE", a.copy_bytes)
    ws, _, cw = copy_factor(a.copy_write, "WRITE_SIZE", a.copy_bytes)
    raw_r = dispatches(a.raw_read) if a.raw_read else None
    raw_w = dispatches(a.raw_write) if a.raw_write else None

    keys = list(fetch.keys())
    # the instances with the most launches in the timing run (the trace) are
    # the tuned ones (every candidate also runs during tuning in the counter
    # runs); depth Nyquist launches are the instances whose sixth flag is true
    launches = defaultdict(int)
    if a.trace:
        for r in csv.DictReader(open(a.trace)):
            launches[short(r["Kernel_Name"])] += 1
    st, depth_keys = stage_keys(keys, launches if a.trace else None)
    if not a.trace:
        for k in depth_keys:
            launches[k[0]] += len(fetch[k]["FETCH_SIZE"])
    def nyq_flag(name):
        # k_depth<T, LPM, P, DISP, WANTX, NYQ, streaming, non-uniform>: the sixth argument
        args = [x.strip() for x in name[name.index("<") + 1:name.rindex(">")].split(",")]
        return "true" if len(args) > 5 and args[5] == "true" else "false"

    for stage, flag in (("depth", "false"), ("depth_nyq", "true")):
        names = [n for n in launches if n.startswith("k_depth<") and nyq_flag(n) == flag]
        if names:
            best = max(names, key=lambda n: launches[n])
            ks = [k for k in depth_keys if k[0] == best]
            if ks:
                st[stage] = ks[0]
    # the Nyquist stage of the default launch averages the sign replicas
    avg = [k for k in keys if k[0].startswith("k_nyq_average")]
    if avg:
        st["depth_nyq"] = avg[0]

    lines = ["Copy reference `%s`: %d bytes read and %d written per launch; FETCH_SIZE reads %.1f and "
             "WRITE_SIZE %.1f, so %.1f bytes per FETCH_SIZE unit and %.1f per WRITE_SIZE unit."
             % (copy_name, a.copy_bytes, a.copy_bytes, cf, cw, fs, ws), "",
             "| stage | kernel | grid | fetched MB (copy-scaled) | written MB (copy-scaled) |"
             + (" fetched MB (requests) | written MB (requests) |" if raw_r else ""),
             "|---|---|---|---|---|" + ("---|---|" if raw_r else "")]
    traffic = {}
    for stage in ("x_fwd", "y_fwd", "x_fwd_t", "y_fwd_t", "depth", "depth_nyq", "y_inv", "x_inv"):
        k = st.get(stage)
        if not k or k not in write:
            continue
        fb = median(fetch[k]["FETCH_SIZE"]) * fs
        wb = median(write[k]["WRITE_SIZE"]) * ws
        row = "| %s | `%s` | %d | %.1f | %.1f |" % (stage, k[0], k[1], fb / 1e6, wb / 1e6)
        rec = {"kernel": k[0], "grid": k[1], "fetch": round(fb), "write": round(wb),
               "bytes_per_launch": round(fb + wb), "source_sha": source_sha(SOURCE_OF_STAGE[stage])}
        if raw_r and k in raw_r and raw_w and k in raw_w:
            r = {c: median(v) for c, v in raw_r[k].items()}
            w = {c: median(v) for c, v in raw_w[k].items()}
            rr = (128 * r["TCC_EA0_RDREQ_128B_sum"] + 32 * r["TCC_EA0_RDREQ_32B_sum"]
                  + 64 * (r["TCC_EA0_RDREQ_sum"] - r["TCC_EA0_RDREQ_128B_sum"] - r["TCC_EA0_RDREQ_32B_sum"]))
            rw = 64 * w["TCC_EA0_WRREQ_64B_sum"] + 32 * (w["TCC_EA0_WRREQ_sum"] - w["TCC_EA0_WRREQ_64B_sum"])
            row += " %.1f | %.1f |" % (rr / 1e6, rw / 1e6)
            rec["fetch_requests"] = round(rr)
            rec["write_requests"] = round(rw)
        lines.append(row)
        traffic["%s/%s" % (stage, a.workload)] = rec

    doc = ["# %s" % a.title, ""]
    if a.commands:
        doc += ["Commands (from the repository root on the GPU host; CSV paths as written by them):", "", "```"]
        doc += [l.rstrip("\n") for l in open(a.commands)] + ["```", ""]
    if a.stats:
        doc += ["## Kernel durations (`rocprofv3 --kernel-trace --stats`)", "", stats(a.stats), ""]
    if a.trace:
        doc += ["Per launch shape (same run, from the kernel trace; the tuning launches of the first "
                "call are the layouts with 4 launches):", "", trace_table(a.trace), ""]
    doc += ["## HBM traffic per launch (`--pmc FETCH_SIZE`, `--pmc WRITE_SIZE`)", ""] + lines + [""]
    if a.sq:
        sq = dispatches(a.sq)
        doc += ["## Waiting and occupancy (`--pmc SQ_WAIT_ANY SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAVES`)", "",
                "wait = SQ_WAIT_ANY / SQ_WAVE_CYCLES (share of the waves' resident cycles spent waiting); "
                "waves per SQ-cycle = SQ_WAVE_CYCLES / SQ_BUSY_CYCLES (resident waves per busy cycle, "
                "summed as the counters sum over the shader engines).", "",
                "| stage | kernel | waves | wait | waves per SQ-cycle |", "|---|---|---|---|---|"]
        for stage in ("x_fwd", "y_fwd", "depth", "depth_nyq", "y_inv", "x_inv"):
            k = st.get(stage)
            if not k or k not in sq:
                continue
            c = {n: median(v) for n, v in sq[k].items()}
            wc = c.get("SQ_WAVE_CYCLES", 0.0)
            doc.append("| %s | `%s` | %d | %.3f | %.1f |" % (stage, k[0], c.get("SQ_WAVES", 0),
                                                             c.get("SQ_WAIT_ANY", 0.0) / wc if wc else 0.0,
                                                             wc / c["SQ_BUSY_CYCLES"] if c.get("SQ_BUSY_CYCLES") else 0.0))
        doc += [""]
    if a.note:
        doc += [a.note, ""]
    with open(a.out, "w") as f:
        f.write("\n".join(doc))
    if a.traffic:
        old = {}
        if os.path.exists(a.traffic):
            old = json.load(open(a.traffic))
        old.update(traffic)
        with open(a.traffic, "w") as f:
            json.dump(old, f, indent=1, sort_keys=True)
            f.write("\n")
    print("\n".join(doc))


def kernels(a):
    """Kernel-time summary of one profiled run: the commands, the per-kernel
    statistics and the per-launch-shape table; with counter CSVs (FETCH_SIZE,
    WRITE_SIZE and the copy references) also the HBM bytes per launch of the
    kernels named by --traffic-kernels, scaled by the copy, and the rate they
    give with the trace's average duration."""
    rows = trace_table(a.trace).split("\n")
    doc = ["# %s" % a.title, "", "Commands (from the repository root on the GPU host):", "", "```"]
    doc += [l.rstrip("\n") for l in open(a.commands)] + ["```", ""]
    doc += ["## Kernel durations (`rocprofv3 --kernel-trace --stats`)", "", stats(a.stats), ""]
    doc += ["Per launch shape (same run, from the kernel trace; the %d with the most time):" % a.top, ""]
    doc += rows[:4 + a.top] + [""]
    if a.fetch and a.write and a.copy_fetch and a.copy_write:
        fetch, write = dispatches(a.fetch), dispatches(a.write)
        fs, copy_name, cf = copy_factor(a.copy_fetch, "FETCH_SIZE", a.copy_bytes)
        ws, _, cw = copy_factor(a.copy_write, "WRITE_SIZE", a.copy_bytes)
        dur = defaultdict(list)
        for r in csv.DictReader(open(a.trace)):
            dur[(short(r["Kernel_Name"]), int(r["Grid_Size_X"]))].append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        doc += ["## HBM traffic per launch (`--pmc FETCH_SIZE`, `--pmc WRITE_SIZE`)", "",
                "Copy reference `%s`: %.1f bytes per FETCH_SIZE unit and %.1f per WRITE_SIZE unit; the "
                "mean over the launches of each shape (launches of one shape may move different amounts, "
                "e.g. surface and volume axpy launches share a grid); rate = (fetched + written) / the "
                "trace's average duration of that shape (the counter and trace runs make the same "
                "launches)." % (copy_name, fs, ws), "",
                "| kernel | grid | launches | fetched MB | written MB | average (us) | TB/s | of 8 TB/s |",
                "|---|---|---|---|---|---|---|---|"]
        pats = [re.compile(x) for x in (a.traffic_kernels or [])]
        for k in sorted(fetch, key=lambda k: -sum(dur.get(k, [0]))):
            if not any(p.search(k[0]) for p in pats) or k not in write or k not in dur:
                continue
            fv, wv = fetch[k]["FETCH_SIZE"], write[k]["WRITE_SIZE"]
            fb = sum(fv) / len(fv) * fs
            wb = sum(wv) / len(wv) * ws
            us = sum(dur[k]) / len(dur[k])
            rate = (fb + wb) / (us * 1e-6) / 1e12
            doc.append("| `%s` | %d | %d | %.2f | %.2f | %.2f | %.2f | %.3f |"
                       % (k[0], k[1], len(dur[k]), fb / 1e6, wb / 1e6, us, rate, rate / 8.0))
        doc += [""]
    if a.note:
        doc += [a.note, ""]
    with open(a.out, "w") as f:
        f.write("\n".join(doc))
    print("\n".join(doc))


def main():
    if len(sys.argv) > 2 and sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "kernels":
        ap = argparse.ArgumentParser()
        ap.add_argument("mode", choices=["kernels"])
        ap.add_argument("--title", required=True)
        ap.add_argument("--stats", required=True)
        ap.add_argument("--trace", required=True)
        ap.add_argument("--commands", required=True)
        ap.add_argument("--top", type=int, default=20)
        ap.add_argument("--fetch")
        ap.add_argument("--write")
        ap.add_argument("--copy-fetch")
        ap.add_argument("--copy-write")
        ap.add_argument("--copy-bytes", type=int, default=400000000)
        ap.add_argument("--traffic-kernels", nargs="*", help="regular expressions of kernel names")
        ap.add_argument("--note")
        ap.add_argument("--out", required=True)
        kernels(ap.parse_args())
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["report"])
    ap.add_argument("--workload", required=True, help="e.g. 256x256x64/fp64 (key of traffic.json)")
    ap.add_argument("--title", default="Operator kernels")
    ap.add_argument("--stats")
    ap.add_argument("--trace")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--raw-read")
    ap.add_argument("--raw-write")
    ap.add_argument("--sq", help="counter CSV of SQ_WAIT_ANY, SQ_WAVE_CYCLES, SQ_BUSY_CYCLES, SQ_WAVES")
    ap.add_argument("--commands")
    ap.add_argument("--note")
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic")
    report(ap.parse_args())


if __name__ == "__main__":
    main()

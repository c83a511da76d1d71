"""Summaries of rocprofv3 CSV output (measurement tooling, not the hot path).

  python -m paper_2512_07311_amd.rocprof_summary counters DIR [--scale S]
      per-kernel mean of each counter in DIR/*_counter_collection.csv
      (one line per dispatch and counter), multiplied by S
  python -m paper_2512_07311_amd.rocprof_summary stats DIR
      the kernel statistics table of DIR/*_kernel_stats.csv
  python -m paper_2512_07311_amd.rocprof_summary stage DIR --kernels a,b,c
      totals over the dispatches of the named kernels (short names): the
      sum of every counter in DIR/*_counter_collection.csv if there is one,
      else calls and total duration from DIR/*_kernel_stats.csv

Rows are streamed, so multi-GB counter files are fine.  Output is a
markdown table on stdout.
"""
import argparse
import collections
import csv
import glob
import os
import sys


def _one(directory, suffix):
    files = sorted(glob.glob(os.path.join(directory, "*" + suffix)))
    if not files:
        sys.exit("no *%s under %s" % (suffix, directory))
    return files[0]


def _short(name):
    return name.split("(")[0].replace("void ", "")


def counters(directory, scale=1.0, top=12):
    acc = collections.defaultdict(lambda: [0, 0.0, 0])   # (kernel, counter) -> n, sum, dur_ns
    with open(_one(directory, "_counter_collection.csv"), newline="") as f:
        for r in csv.DictReader(f):
            a = acc[(_short(r["Kernel_Name"]), r["Counter_Name"])]
            a[0] += 1
            a[1] += float(r["Counter_Value"])
            a[2] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    rows = sorted(acc.items(), key=lambda kv: -kv[1][1])[:top]
    print("| kernel | counter | dispatches | mean per dispatch (x%g) | mean duration us |" % scale)
    print("|---|---|---:|---:|---:|")
    for (k, c), (n, s, d) in rows:
        print("| `%s` | %s | %d | %.1f | %.2f |" % (k, c, n, scale * s / n, d / n / 1e3))


def stats(directory, top=12):
    with open(_one(directory, "_kernel_stats.csv"), newline="") as f:
        rows = list(csv.DictReader(f))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    print("Kernel dispatches: %d, total kernel time %.2f s" % (sum(int(r["Calls"]) for r in rows), tot / 1e9))
    print()
    print("| kernel | calls | total s | avg us | min us | max us | share |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        print("| `%s` | %s | %.2f | %.2f | %.2f | %.2f | %.1f%% |" % (
            _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e9, float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))


def _base(name):
    """Short kernel name without namespace and template arguments."""
    return _short(name).split("<")[0].split("::")[-1]


def stage(directory, kernels):
    want = set(kernels)
    cc = sorted(glob.glob(os.path.join(directory, "*_counter_collection.csv")))
    if cc:
        acc = collections.defaultdict(lambda: [0, 0.0])   # counter -> dispatches, sum
        with open(cc[0], newline="") as f:
            for r in csv.DictReader(f):
                if _base(r["Kernel_Name"]) in want:
                    a = acc[r["Counter_Name"]]
                    a[0] += 1
                    a[1] += float(r["Counter_Value"])
        for c, (n, v) in sorted(acc.items()):
            print("stage %s: %d dispatches, sum %.1f" % (c, n, v))
        return
    calls, ns = 0, 0.0
    with open(_one(directory, "_kernel_stats.csv"), newline="") as f:
        for r in csv.DictReader(f):
            if _base(r["Name"]) in want:
                calls += int(r["Calls"])
                ns += float(r["TotalDurationNs"])
    print("stage duration: %d dispatches, total %.4f s" % (calls, ns / 1e9))


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["counters", "stats", "stage"])
    ap.add_argument("directory")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--kernels", default="")
    a = ap.parse_args()
    if a.mode == "counters":
        counters(a.directory, a.scale)
    elif a.mode == "stage":
        stage(a.directory, [k for k in a.kernels.split(",") if k])
    else:
        stats(a.directory)

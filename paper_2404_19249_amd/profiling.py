"""Summaries of rocprofv3 output for the profiles/ directory.

    python -m paper_2404_19249_amd.profiling stats <dir>/run_kernel_trace.csv [--top N]
    python -m paper_2404_19249_amd.profiling pmc <dir>/run_counter_collection.csv [--regex R]
    python -m paper_2404_19249_amd.profiling traffic <fetch.csv> --write <write.csv> --regex R

`traffic` gives the HBM bytes per launch of the kernels matching R as
FETCH_SIZE x 2 + WRITE_SIZE x 1 (KiB x 1024, medians over dispatches): on
this device a plain 1 GiB device copy reads back FETCH_SIZE = half the bytes
it copies and WRITE_SIZE = all of them.

Kernel launches of the block PCG that return at once (issued after the
solver converged, between two host polls) last a few microseconds; the
stats table lists them apart from the launches that did the work (longer
than --active-us, default 20).
"""
import argparse
import collections
import csv
import re
import statistics


def stats(path, top=25, active_us=20.0):
    rows = list(csv.DictReader(open(path)))
    by = collections.defaultdict(list)
    for r in rows:
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3  # us
        by[r["Kernel_Name"]].append(dur)
    total = sum(sum(v) for v in by.values())
    out = []
    for name, v in sorted(by.items(), key=lambda kv: -sum(kv[1]))[:top]:
        act = [d for d in v if d > active_us]
        out.append((sum(v) / total * 100, len(v), len(act), statistics.mean(act) if act else 0.0,
                    statistics.median(act) if act else 0.0, sum(v) * 1e-3, name))
    print(f"{'%time':>6} {'calls':>6} {'active':>6} {'avg_act_us':>10} {'med_act_us':>10} "
          f"{'total_ms':>9}  kernel")
    for o in out:
        print(f"{o[0]:6.2f} {o[1]:6d} {o[2]:6d} {o[3]:10.1f} {o[4]:10.1f} {o[5]:9.2f}  {o[6][:150]}")


def pmc(path, regex=None):
    rows = list(csv.DictReader(open(path)))
    by = collections.defaultdict(list)
    for r in rows:
        if regex and not re.search(regex, r["Kernel_Name"]):
            continue
        by[(r["Kernel_Name"][:120], r["Counter_Name"], r["Grid_Size"])].append(float(r["Counter_Value"]))
    print(f"{'counter':>14} {'grid':>8} {'n':>5} {'median':>12} {'max':>12}  kernel")
    for (k, c, g), v in sorted(by.items()):
        print(f"{c:>14} {g:>8} {len(v):5d} {statistics.median(v):12.4g} {max(v):12.4g}  {k}")


def traffic(fetch_path, write_path, regex):
    def med(path, counter):
        v = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
             if r["Counter_Name"] == counter and re.search(regex, r["Kernel_Name"])]
        return statistics.median(v), len(v)
    (f, nf), (w, nw) = med(fetch_path, "FETCH_SIZE"), med(write_path, "WRITE_SIZE")
    print(f"FETCH_SIZE median {f:.6g} KiB ({nf} dispatches), WRITE_SIZE median {w:.6g} KiB ({nw} dispatches)")
    print(f"traffic per launch: {int(round((2 * f + w) * 1024))} bytes")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "pmc", "traffic"])
    ap.add_argument("path")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--regex", default=None)
    ap.add_argument("--active-us", type=float, default=20.0)
    ap.add_argument("--write", default=None)
    a = ap.parse_args()
    if a.mode == "stats":
        stats(a.path, a.top, a.active_us)
    elif a.mode == "pmc":
        pmc(a.path, a.regex)
    else:
        traffic(a.path, a.write, a.regex)

"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_1901_01047_amd.profsum trace <kernel_trace.csv> [--noop-us X]
    python -m paper_1901_01047_amd.profsum pmc <counter_collection.csv> <kernel regex> <counter>

`trace` prints a Markdown table per kernel: dispatches, the dispatches that
found no work (window kernels of a walker whose window is closed return at
once; they are told apart by a duration below --noop-us, default 3 us), the
average duration over the working dispatches and the total.  `pmc` prints
the median and mean of one counter per dispatch of the kernels matching the
regex (values as rocprofv3 reports them).
"""
import argparse
import csv
import re
import statistics
import sys


def _rows(path):
    with open(path, newline="") as f:
        yield from csv.DictReader(f)


def trace_summary(path, noop_us=3.0):
    per = {}
    for r in _rows(path):
        name = r.get("Kernel_Name", "")
        try:
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3     # ns -> us
        except (KeyError, ValueError):
            continue
        per.setdefault(name, []).append(d)
    total = sum(sum(v) for v in per.values())
    out = []
    for name, ds in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        work = [d for d in ds if d >= noop_us]
        out.append({"kernel": name, "calls": len(ds), "noop_calls": len(ds) - len(work),
                    "avg_active_us": (sum(work) / len(work)) if work else 0.0, "total_ms": sum(ds) * 1e-3,
                    "share": sum(ds) / total if total else 0.0})
    return out


def trace_table(rows, top=25):
    lines = ["| kernel | dispatches | no-work dispatches | average of working dispatches (us) | total (ms) | share |",
             "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        lines.append(f"| `{r['kernel']}` | {r['calls']} | {r['noop_calls']} | {r['avg_active_us']:.2f} | "
                     f"{r['total_ms']:.2f} | {100 * r['share']:.1f}% |")
    return "\n".join(lines)


def pmc_summary(path, kernel_regex, counter):
    rx = re.compile(kernel_regex)
    vals = {}
    for r in _rows(path):
        name = r.get("Kernel_Name", "")
        if not rx.search(name):
            continue
        cname = r.get("Counter_Name", counter)
        if cname != counter:
            continue
        try:
            v = float(r.get("Counter_Value", r.get(counter, "nan")))
        except ValueError:
            continue
        key = (r.get("Dispatch_Id") or r.get("Correlation_Id") or str(len(vals)))
        vals[key] = vals.get(key, 0.0) + v
    v = list(vals.values())
    if not v:
        return None
    return {"dispatches": len(v), "median": statistics.median(v), "mean": sum(v) / len(v)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--noop-us", type=float, default=3.0)
    t.add_argument("--top", type=int, default=25)
    pm = sub.add_parser("pmc")
    pm.add_argument("csv")
    pm.add_argument("kernel_regex")
    pm.add_argument("counter")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace_table(trace_summary(a.csv, a.noop_us), a.top))
    else:
        r = pmc_summary(a.csv, a.kernel_regex, a.counter)
        if r is None:
            print("no matching dispatches", file=sys.stderr)
            return 1
        print(f"{a.counter}: dispatches {r['dispatches']}, median {r['median']:.1f}, mean {r['mean']:.1f}")
    return 0


if __name__ == "__main__":
    sys.exit(main())

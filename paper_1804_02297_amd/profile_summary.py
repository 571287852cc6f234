"""Summaries of rocprofv3 databases (kernel-trace stats and counter runs) as text.

    python -m paper_1804_02297_amd.profile_summary trace DB            # per-kernel calls/avg/total
    python -m paper_1804_02297_amd.profile_summary pmc DB [DB ...]     # per-kernel counter averages

Kernel names are shortened (template arguments kept, parameter lists dropped).
"""
from __future__ import annotations

import collections
import re
import sqlite3
import sys


def short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("ls::", "")
    return re.sub(r"\(.*$", "", name)


def trace(db: str) -> str:
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    out = ["| kernel | calls | avg (us) | total (us) | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows:          # the view reports microseconds
        out.append(f"| `{short(name)[:90]}` | {calls} | {avg:.1f} | {tot:.1f} | {pct:.1f} |")
    return "\n".join(out)


def dispatches(db: str, pattern: str) -> str:
    """Per-dispatch durations (us) of kernels whose name contains `pattern`."""
    c = sqlite3.connect(db)
    out = ["| kernel | grid | duration (us) |", "|---|---|---|"]
    for name, g, d in c.execute("select name, grid_x, duration from kernels where name like ?", (f"%{pattern}%",)):
        out.append(f"| `{short(name)[:90]}` | {g} | {d / 1000:.1f} |")
    return "\n".join(out)


def pmc(dbs) -> str:
    agg = collections.defaultdict(float)
    names = {}
    for db in dbs:
        c = sqlite3.connect(db)
        for did, kn, cn, v in c.execute(
                "select dispatch_id, kernel_name, counter_name, value from counters_collection"):
            agg[(db, did, cn)] += v
            names[(db, did)] = kn
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for (db, did, cn), v in agg.items():
        per[short(names[(db, did)])][cn].append(v)
    cols = sorted({cn for d in per.values() for cn in d})
    out = ["| kernel | dispatches | " + " | ".join(cols) + " |", "|---|---|" + "---|" * len(cols)]
    for k, d in per.items():
        ndisp = max(len(v) for v in d.values())
        vals = " | ".join(f"{sum(d[cn]) / len(d[cn]):.6g}" if cn in d else "" for cn in cols)
        out.append(f"| `{k[:90]}` | {ndisp} | {vals} |")
    return "\n".join(out)


def pmc_dispatch(db: str, pattern: str) -> str:
    """Per-dispatch counter sums for kernels whose name contains `pattern`."""
    c = sqlite3.connect(db)
    agg = collections.defaultdict(float)
    meta = {}
    for did, kn, g, cn, v in c.execute("select dispatch_id, kernel_name, grid_size, counter_name, value "
                                       "from counters_collection where kernel_name like ?", (f"%{pattern}%",)):
        agg[(did, cn)] += v
        meta[did] = (short(kn), g)
    out = ["| dispatch | kernel | grid | counter | value (KiB) |", "|---|---|---|---|---|"]
    for (did, cn), v in sorted(agg.items()):
        out.append(f"| {did} | `{meta[did][0][:60]}` | {meta[did][1]} | {cn} | {v:.6g} |")
    return "\n".join(out)


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "trace":
        print(trace(sys.argv[2]))
    elif mode == "dispatches":
        print(dispatches(sys.argv[2], sys.argv[3]))
    elif mode == "pmc-dispatch":
        print(pmc_dispatch(sys.argv[2], sys.argv[3]))
    else:
        print(pmc(sys.argv[2:]))

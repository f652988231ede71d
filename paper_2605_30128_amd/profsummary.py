"""Summarises a rocprofv3 results database (kernel trace and, if present,
hardware counters) as a short text table: per kernel, the number of
dispatches and the average duration, and the average of every collected
counter per dispatch.

python -m paper_2605_30128_amd.profsummary <results.db> [--top N] [--match SUBSTR]
"""
from __future__ import annotations

import argparse
import sqlite3


def summarize(db: str, top: int = 15, match: str = "") -> str:
    con = sqlite3.connect(db)
    tables = {r[0] for r in con.execute("select name from sqlite_master where type in ('table','view')")}
    lines = []
    if "kernels" in tables:
        rows = con.execute("select name, count(*), avg(end - start), sum(end - start) from kernels "
                           "group by name order by sum(end - start) desc").fetchall()
        grand = sum(r[3] for r in rows) or 1
        lines.append(f"{'kernel':80s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}")
        for name, calls, avg, total in rows:
            if match and match not in name:
                continue
            lines.append(f"{name[:80]:80s} {calls:7d} {avg / 1e3:10.1f} {total / 1e6:10.2f} "
                         f"{100.0 * total / grand:6.1f}")
            if len(lines) > top:
                break
    if "counters_collection" in tables or any(t.startswith("rocpd_pmc_event") for t in tables):
        try:
            rows = con.execute(
                "select kernel_name, counter_name, avg(value), count(value) from counters_collection "
                "group by kernel_name, counter_name order by kernel_name").fetchall()
        except sqlite3.Error:
            rows = []
        if rows:
            lines.append("")
            lines.append(f"{'kernel':80s} {'counter':24s} {'avg per dispatch':>18s} {'dispatches':>10s}")
            for k, cname, v, n in rows:
                if match and match not in k:
                    continue
                lines.append(f"{k[:80]:80s} {cname:24s} {v:18.1f} {n:10d}")
    return "\n".join(lines)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=15)
    ap.add_argument("--match", default="")
    a = ap.parse_args()
    print(summarize(a.db, a.top, a.match))

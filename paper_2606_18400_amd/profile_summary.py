"""Per-kernel summary of a rocprofv3 kernel trace (rocpd SQLite output).

Usage: python -m paper_2606_18400_amd.profile_summary <results.db> [--top N] [--match SUBSTR]

Prints, per kernel name: dispatch count, average / min / max duration in
microseconds and total milliseconds, sorted by total time.  Used to write the
short text summaries kept under profiles/.
"""

import argparse
import sqlite3
import sys


def summarize(db, top=25, match=None):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), avg(duration), min(duration), max(duration), sum(duration) "
                       "from kernels group by name order by sum(duration) desc").fetchall()
    out = []
    for name, n, avg, mn, mx, tot in rows:
        if match and match not in name:
            continue
        out.append((name, n, avg / 1e3, mn / 1e3, mx / 1e3, tot / 1e6))
    return out[:top]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--match", default=None)
    a = ap.parse_args(argv)
    print(f"{'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total_ms':>10}  kernel")
    for name, n, avg, mn, mx, tot in summarize(a.db, a.top, a.match):
        print(f"{n:6d} {avg:10.2f} {mn:10.2f} {mx:10.2f} {tot:10.2f}  {name}")


if __name__ == "__main__":
    sys.exit(main())

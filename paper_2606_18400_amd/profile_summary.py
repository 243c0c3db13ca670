"""Short text summaries of rocprofv3 output, for the files kept under profiles/.

Usage:
  python -m paper_2606_18400_amd.profile_summary stats <kernel_stats.csv | results.db> [--top N]
  python -m paper_2606_18400_amd.profile_summary trace <kernel_trace.csv> [--match moe]
  python -m paper_2606_18400_amd.profile_summary counters <counter_collection.csv> [...] [--match gemm]
  python -m paper_2606_18400_amd.profile_summary pmc <fetch counter_collection.csv> <write counter_collection.csv>
          [--copy-match MulFunctor] [--copy-bytes 1073741824]

`stats` prints, per kernel: dispatch count, average / min / max duration in
microseconds and total milliseconds, sorted by total time (CSV from
`--kernel-trace --stats --output-format csv`, or the rocpd SQLite database).

`trace` prints, per (kernel, grid), dispatch count and average duration from
the per-dispatch CSV of `--kernel-trace` (grid sizes separate the batch sizes
of one run).

`counters` prints, per kernel (and grid), the mean per dispatch of every
counter in one or more `--pmc` passes (counter_collection.csv files), with
the derived figures the SQ counters allow: MFMA busy share
(SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE x SIMDs; GRBM_GUI_ACTIVE is
summed over the XCDs, `--xcds`), LDS active share (SQ_LDS_IDX_ACTIVE over
the cycles of every CU) and the share of wave time spent
waiting (SQ_WAIT_ANY over SQ_WAVE_CYCLES).

`pmc` reads one `--pmc FETCH_SIZE` and one `--pmc WRITE_SIZE` pass (KiB per
dispatch) and scales each counter by what it reads for a plain elementwise
copy of known size (the bench's calibration kernel reads and writes
`copy-bytes` each): factor = counter KiB * 1024 / copy-bytes; HBM bytes of a
dispatch = counter KiB * 1024 / factor.
"""

import argparse
import collections
import csv
import sqlite3
import sys


def short_name(name):
    return name.replace("void cloak::(anonymous namespace)::", "").replace("cloak::(anonymous namespace)::", "")


def stats_rows(path):
    if path.endswith(".db"):
        con = sqlite3.connect(path)
        rows = con.execute("select name, count(*), avg(duration), min(duration), max(duration), sum(duration) "
                           "from kernels group by name").fetchall()
        return [(n, c, a / 1e3, mn / 1e3, mx / 1e3, t / 1e6) for n, c, a, mn, mx, t in rows]
    out = []
    for r in csv.DictReader(open(path)):
        out.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                    float(r["MaxNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6))
    return out


def print_stats(path, top):
    rows = sorted(stats_rows(path), key=lambda r: -r[5])[:top]
    print(f"{'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total_ms':>10}  kernel")
    for name, n, avg, mn, mx, tot in rows:
        print(f"{n:6d} {avg:10.2f} {mn:10.2f} {mx:10.2f} {tot:10.2f}  {short_name(name)[:120]}")


def print_trace(path, match):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if match and match not in r["Kernel_Name"]:
            continue
        key = (short_name(r["Kernel_Name"]).split("(")[0], int(r["Grid_Size_X"]), int(r["Grid_Size_Y"]))
        d[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    print(f"{'calls':>6} {'avg_us':>10}  {'grid (threads)':>16}  kernel")
    for k in sorted(d, key=lambda k: (k[1], k[2], k[0])):
        v = d[k]
        print(f"{len(v):6d} {sum(v) / len(v):10.2f}  {k[1]:>9}x{k[2]:<6}  {k[0][:90]}")


def counter_means(path):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[(r["Kernel_Name"], r["Grid_Size"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in d.items()}, {k: len(v) for k, v in d.items()}


def print_pmc(fetch_csv, write_csv, copy_match, copy_bytes, factors=None):
    fetch, n = counter_means(fetch_csv)
    write, _ = counter_means(write_csv)
    ck = None
    if factors:
        # a run without the calibration copy: factors measured by another run
        f_fac, w_fac = factors
        print("calibration: factors given")
    else:
        copy = [k for k in fetch if copy_match in k[0]]
        if not copy:
            raise SystemExit(f"no dispatch of a kernel matching {copy_match!r}")
        ck = copy[0]
        f_fac = fetch[ck] * 1024 / copy_bytes
        w_fac = write[ck] * 1024 / copy_bytes
        print(f"calibration kernel: {short_name(ck[0])[:90]} grid {ck[1]} (reads and writes {copy_bytes} B)")
    print(f"FETCH_SIZE factor {f_fac:.5f}  WRITE_SIZE factor {w_fac:.5f}")
    print(f"{'calls':>6} {'fetch_KiB':>14} {'write_KiB':>12} {'hbm_read_B':>14} {'hbm_write_B':>12}  kernel (grid)")
    for k in sorted(fetch, key=lambda k: -fetch[k]):
        if k == ck:
            continue
        rb = fetch[k] * 1024 / f_fac
        wb = write.get(k, 0.0) * 1024 / w_fac
        print(f"{n[k]:6d} {fetch[k]:14.1f} {write.get(k, 0.0):12.1f} {rb:14.0f} {wb:12.0f}  "
              f"{short_name(k[0])[:80]} ({k[1]})")


def print_counters(paths, match, cus, simds_per_cu, xcds):
    d = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in paths:
        for r in csv.DictReader(open(path)):
            if match and match not in r["Kernel_Name"]:
                continue
            d[(short_name(r["Kernel_Name"]).split("(")[0], r["Grid_Size"])][r["Counter_Name"]].append(
                float(r["Counter_Value"]))
    for (k, grid), cs in sorted(d.items()):
        m = {c: sum(v) / len(v) for c, v in cs.items()}
        n = max(len(v) for v in cs.values())
        print(f"{k[:100]}  grid {grid}  ({n} dispatches per pass)")
        for c in sorted(m):
            print(f"    {c:36s} {m[c]:16.6g}")
        g = m.get("GRBM_GUI_ACTIVE")
        if g:
            cyc = g / xcds
            if "SQ_VALU_MFMA_BUSY_CYCLES" in m:
                print(f"    -> MFMA busy {100 * m['SQ_VALU_MFMA_BUSY_CYCLES'] / (cyc * cus * simds_per_cu):.1f}% "
                      f"of {cyc:.4g} cycles per XCD")
            if "SQ_LDS_IDX_ACTIVE" in m:
                print(f"    -> LDS active {100 * m['SQ_LDS_IDX_ACTIVE'] / (cyc * cus):.1f}% of CU cycles")
        if "SQ_WAIT_ANY" in m and "SQ_WAVE_CYCLES" in m:
            print(f"    -> waves waiting {100 * m['SQ_WAIT_ANY'] / m['SQ_WAVE_CYCLES']:.1f}% of wave time")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("path")
    s.add_argument("--top", type=int, default=30)
    t = sub.add_parser("trace")
    t.add_argument("path")
    t.add_argument("--match", default="")
    c = sub.add_parser("counters")
    c.add_argument("paths", nargs="+")
    c.add_argument("--match", default="")
    c.add_argument("--cus", type=int, default=256)
    c.add_argument("--simds-per-cu", type=int, default=4)
    c.add_argument("--xcds", type=int, default=8)
    p = sub.add_parser("pmc")
    p.add_argument("fetch_csv")
    p.add_argument("write_csv")
    p.add_argument("--copy-match", default="MulFunctor")
    p.add_argument("--copy-bytes", type=int, default=1 << 30)
    p.add_argument("--factors", nargs=2, type=float, metavar=("FETCH", "WRITE"),
                   help="counter-to-bytes factors from another run's calibration copy")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print_stats(a.path, a.top)
    elif a.cmd == "trace":
        print_trace(a.path, a.match)
    elif a.cmd == "counters":
        print_counters(a.paths, a.match, a.cus, a.simds_per_cu, a.xcds)
    else:
        print_pmc(a.fetch_csv, a.write_csv, a.copy_match, a.copy_bytes, a.factors)


if __name__ == "__main__":
    sys.exit(main())

"""Summaries of rocprofv3 output (the rocpd SQLite database).

    python -m paper_1606_07550_amd.profiling kernels <results.db> [--top N]
    python -m paper_1606_07550_amd.profiling counters <results.db> [--kernel SUBSTR]

``kernels`` prints per-kernel call counts and durations (the same figures as
``rocprofv3 --stats``); ``counters`` prints the per-dispatch mean of every
PMC counter collected with ``--pmc``, per kernel.
"""
import argparse
import sqlite3


def kernel_stats(db, top=40):
    c = sqlite3.connect(db)
    # durations in the kernels view are nanoseconds
    allsum = c.execute("select sum(end - start) from kernels").fetchone()[0] or 1
    rows = c.execute("select name, count(*), sum(end - start), avg(end - start) from kernels "
                     "group by name order by sum(end - start) desc limit ?", (top,)).fetchall()
    out = [f"{'calls':>6} {'total_ms':>12} {'avg_ms':>10} {'pct':>6}  kernel"]
    for name, calls, tot, avg in rows:
        out.append(f"{calls:>6} {tot / 1e6:>12.3f} {avg / 1e6:>10.3f} {100.0 * tot / allsum:>6.2f}  {name}")
    return "\n".join(out)


def counter_stats(db, kernel=None):
    c = sqlite3.connect(db)
    cols = [d[1] for d in c.execute("pragma table_info(counters_collection)")]
    name_col = "kernel_name" if "kernel_name" in cols else "name"
    q = (f"select {name_col}, counter_name, count(*), avg(value), min(value), max(value) "
         f"from counters_collection group by {name_col}, counter_name order by {name_col}, counter_name")
    out = [f"{'dispatches':>10} {'mean':>16} {'min':>16} {'max':>16}  counter  kernel"]
    for kname, cname, n, avg, mn, mx in c.execute(q):
        if kernel and kernel not in kname:
            continue
        out.append(f"{n:>10} {avg:>16.1f} {mn:>16.1f} {mx:>16.1f}  {cname}  {kname}")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["kernels", "counters"])
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=40)
    ap.add_argument("--kernel", default=None)
    a = ap.parse_args()
    print(kernel_stats(a.db, a.top) if a.what == "kernels" else counter_stats(a.db, a.kernel))


if __name__ == "__main__":
    main()

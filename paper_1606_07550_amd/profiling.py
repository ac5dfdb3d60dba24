"""Summaries of rocprofv3 output (the rocpd SQLite database).

    python -m paper_1606_07550_amd.profiling kernels <results.db> [--top N]
    python -m paper_1606_07550_amd.profiling counters <results.db> [--kernel SUBSTR]
    python -m paper_1606_07550_amd.profiling traffic --fetch F.db --write W.db \
        --kernel SUBSTR --variant V --workload NAME --command "..."

``kernels`` prints per-kernel call counts and durations (the same figures as
``rocprofv3 --stats``); ``counters`` prints the per-dispatch mean of every
PMC counter collected with ``--pmc``, per kernel. ``traffic`` turns a
FETCH_SIZE run and a WRITE_SIZE run into bytes per launch of one kernel,
each scaled by what the same counter reads for the library's streaming copy
kernel (k_probe_copy) of a known size, and prints a summary whose
``key: value`` lines the benchmark reads back (it uses them only while the
intersection kernels' source hash still matches).
"""
import argparse
import hashlib
import os
import sqlite3

PKG = os.path.dirname(os.path.abspath(__file__))
COUNT_SOURCE = os.path.join(PKG, "csrc", "count_kernels.hip")
PROBE_BYTES = 2 << 30  # size of the copy the benchmark's bandwidth probe runs


def count_source_sha256():
    with open(COUNT_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _per_kernel(db, counter, every=1, offset=0):
    """{kernel: (dispatches, mean value)}; with every > 1 only the dispatches
    at positions offset, offset + every, ... (in dispatch order) of each
    kernel count, e.g. one bin's launches when several bins of one count run
    the same kernel."""
    c = sqlite3.connect(db)
    vals = {}
    for k, v in c.execute("select kernel_name, value from counters_collection where counter_name=? "
                          "order by dispatch_id", (counter,)):
        vals.setdefault(k, []).append(v)
    out = {}
    for k, vs in vals.items():
        pick = vs[offset::every] if "k_probe_copy" not in k else vs
        if pick:
            out[k] = (len(pick), sum(pick) / len(pick))
    return out


def traffic_summary(fetch_db, write_db, kernel, variant, workload, command, bin=None, every=1, offset=0):
    f = _per_kernel(fetch_db, "FETCH_SIZE", every, offset)
    w = _per_kernel(write_db, "WRITE_SIZE", every, offset)
    probe = [k for k in f if "k_probe_copy" in k][0]
    fscale = PROBE_BYTES / (f[probe][1] * 1024.0)
    wscale = PROBE_BYTES / (w[probe][1] * 1024.0)
    ks = [k for k in f if kernel in k]
    if len(ks) != 1:
        raise SystemExit(f"kernel substring {kernel!r} matches {len(ks)} kernels")
    k = ks[0]
    fb = f[k][1] * 1024.0 * fscale
    wb = w[k][1] * 1024.0 * wscale
    sel = (f"Dispatches {offset}, {offset} + {every}, ... of this kernel (bin {bin}'s launches; "
           f"{every} bins of one count run it).") if every > 1 else ""
    lines = [
        f"# Memory traffic of {k.split('(')[0].replace('void ', '')} — {workload}",
        "",
        "FETCH_SIZE and WRITE_SIZE (KiB per dispatch, L2 to fabric) from two separate rocprofv3 --pmc runs,",
        "each scaled by the ratio of the true bytes of the library's streaming copy kernel (k_probe_copy,",
        f"{PROBE_BYTES} bytes read and written per launch, run inside the same benchmark) to what the same",
        f"counter reads for it: FETCH x{fscale:.3f}, WRITE x{wscale:.3f}.",
        *([sel] if sel else []),
        "",
        "Commands (from /tmp, repository at /root/repo):",
        f"    {command.replace('PMC', 'FETCH_SIZE')}",
        f"    {command.replace('PMC', 'WRITE_SIZE')}",
        "",
        f"kernel: {k.split('(')[0].replace('void ', '')}",
        f"variant: {variant}",
        *([f"bin: {bin}"] if bin is not None else []),
        f"workload: {workload}",
        f"dispatches: {f[k][0]}",
        f"fetch_bytes_per_launch: {fb:.0f}",
        f"write_bytes_per_launch: {wb:.0f}",
        f"traffic_bytes_per_launch: {fb + wb:.0f}",
        f"count_kernels_sha256: {count_source_sha256()}",
    ]
    return "\n".join(lines)


def read_traffic(path):
    """Parses a summary written by traffic_summary; None if missing."""
    if not os.path.exists(path):
        return None
    out = {}
    with open(path) as fh:
        for line in fh:
            if ": " in line and not line.startswith(("#", " ")):
                key, val = line.rstrip("\n").split(": ", 1)
                out[key.strip()] = val.strip()
    return out


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
    ap.add_argument("what", choices=["kernels", "counters", "traffic"])
    ap.add_argument("db", nargs="?")
    ap.add_argument("--top", type=int, default=40)
    ap.add_argument("--kernel", default=None)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--variant", type=int)
    ap.add_argument("--workload")
    ap.add_argument("--command", default="")
    ap.add_argument("--bin", type=int, default=None, help="the bin whose launches are summarised")
    ap.add_argument("--every", type=int, default=1, help="launches of the kernel per count")
    ap.add_argument("--offset", type=int, default=0, help="position of the bin's launch among them")
    a = ap.parse_args()
    if a.what == "kernels":
        print(kernel_stats(a.db, a.top))
    elif a.what == "counters":
        print(counter_stats(a.db, a.kernel))
    else:
        print(traffic_summary(a.fetch, a.write, a.kernel, a.variant, a.workload, a.command, a.bin, a.every,
                              a.offset))


if __name__ == "__main__":
    main()

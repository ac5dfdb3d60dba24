"""Summaries of rocprofv3 output (the rocpd SQLite database).

    python -m paper_1606_07550_amd.profiling kernels <results.db> [--top N]
    python -m paper_1606_07550_amd.profiling counters <results.db> [--kernel SUBSTR]
    python -m paper_1606_07550_amd.profiling traffic --fetch F.db --write W.db \
        --kernel SUBSTR --variant V --workload NAME --command "..."
    python -m paper_1606_07550_amd.profiling summary --fetch F.db --write W.db \
        --hitmiss H.db --dram D.db --kernel SUBSTR --variant V --bin B --workload NAME \
        --command "..."

``kernels`` prints per-kernel call counts and durations (the same figures as
``rocprofv3 --stats``); ``counters`` prints the per-dispatch mean of every
PMC counter collected with ``--pmc``, per kernel. ``traffic`` turns a
FETCH_SIZE run and a WRITE_SIZE run into bytes per launch of one kernel,
each scaled by what the same counter reads for the library's streaming copy
kernel (k_probe_copy) of a known size, and prints a summary whose
``key: value`` lines the benchmark reads back (it uses them only while the
intersection kernels' source hash still matches). ``summary`` adds the L2
hit rate (TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)) and the DRAM-side
requests of L2 (TCC_EA0_RDREQ_DRAM_sum, TCC_EA0_WRREQ_DRAM_sum), turned into
bytes by the same counters' reading for the streaming copy of known size: an
upper bound on what reached HBM (the requests are counted before the
Infinity Cache). Each counter set comes from its own rocprofv3 --pmc run.
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


def _selection(bin, every, offset):
    """The sentence naming which dispatches a summary averages."""
    if every > 1:
        return (f"Dispatches {offset}, {offset} + {every}, ... of this kernel (bin {bin}'s launches; "
                f"{every} bins of one count run it).")
    if bin is not None and "-" in str(bin):
        return f"Every dispatch of this kernel in the command is one launch over bins {bin}."
    return ""


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
    sel = _selection(bin, every, offset)
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


def _calib(db, counter, every, offset, kernel):
    """(mean per launch of the kernel, mean per launch of the copy probe)."""
    vals = _per_kernel(db, counter, every, offset)
    probe = [k for k in vals if "k_probe_copy" in k]
    ks = [k for k in vals if kernel in k]
    if len(ks) != 1 or not probe:
        raise SystemExit(f"{counter}: kernel substring {kernel!r} matches {len(ks)} kernels, probe {len(probe)}")
    return vals[ks[0]][1], vals[probe[0]][1], vals[ks[0]][0], ks[0]


def counters_summary(fetch_db, write_db, hitmiss_db, dram_db, kernel, variant, workload, command, bin=None,
                     every=1, offset=0):
    f_k, f_p, disp, kname = _calib(fetch_db, "FETCH_SIZE", every, offset, kernel)
    w_k, w_p, _, _ = _calib(write_db, "WRITE_SIZE", every, offset, kernel)
    h_k, h_p, _, _ = _calib(hitmiss_db, "TCC_HIT_sum", every, offset, kernel)
    m_k, m_p, _, _ = _calib(hitmiss_db, "TCC_MISS_sum", every, offset, kernel)
    r_k, r_p, _, _ = _calib(dram_db, "TCC_EA0_RDREQ_DRAM_sum", every, offset, kernel)
    wr_k, wr_p, _, _ = _calib(dram_db, "TCC_EA0_WRREQ_DRAM_sum", every, offset, kernel)
    fetch = f_k / f_p * PROBE_BYTES
    write = w_k / w_p * PROBE_BYTES
    dram_rd = r_k / r_p * PROBE_BYTES if r_p else 0.0
    dram_wr = wr_k / wr_p * PROBE_BYTES if wr_p else 0.0
    short = kname.split("(")[0].replace("void ", "")
    sel = _selection(bin, every, offset)
    lines = [
        f"# rocprofv3 counters of {short} — {workload}",
        "",
        "Four rocprofv3 --pmc runs of the same command, one counter set each. Bytes are calibrated per",
        "counter against the library's streaming copy kernel (k_probe_copy, run inside the same command),",
        f"which reads and writes {PROBE_BYTES} bytes per launch: bytes = counter(kernel) / counter(copy) x",
        f"{PROBE_BYTES}. FETCH_SIZE/WRITE_SIZE are L2-to-fabric traffic; TCC_EA0_RDREQ_DRAM/WRREQ_DRAM are",
        "L2 requests addressed to DRAM, counted before the Infinity Cache: an upper bound on HBM bytes,",
        "not HBM bytes. L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS).",
        *([sel] if sel else []),
        "",
        "Commands (from /tmp, repository at /root/repo; PMC is each counter set in turn):",
        f"    {command}",
        "    PMC = FETCH_SIZE | WRITE_SIZE | TCC_HIT_sum TCC_MISS_sum | TCC_EA0_RDREQ_DRAM_sum TCC_EA0_WRREQ_DRAM_sum",
        "",
        "| counter | kernel, per launch | copy probe, per launch |",
        "|---|---|---|",
        f"| FETCH_SIZE (KiB) | {f_k:.0f} | {f_p:.0f} |",
        f"| WRITE_SIZE (KiB) | {w_k:.0f} | {w_p:.0f} |",
        f"| TCC_HIT_sum | {h_k:.0f} | {h_p:.0f} |",
        f"| TCC_MISS_sum | {m_k:.0f} | {m_p:.0f} |",
        f"| TCC_EA0_RDREQ_DRAM_sum | {r_k:.0f} | {r_p:.0f} |",
        f"| TCC_EA0_WRREQ_DRAM_sum | {wr_k:.0f} | {wr_p:.0f} |",
        "",
        f"kernel: {short}",
        f"variant: {variant}",
        *([f"bin: {bin}"] if bin is not None else []),
        f"workload: {workload}",
        f"dispatches: {disp}",
        f"fetch_bytes_per_launch: {fetch:.0f}",
        f"write_bytes_per_launch: {write:.0f}",
        f"traffic_bytes_per_launch: {fetch + write:.0f}",
        f"dram_read_bytes_per_launch: {dram_rd:.0f}",
        f"dram_write_bytes_per_launch: {dram_wr:.0f}",
        f"dram_bytes_per_launch: {dram_rd + dram_wr:.0f}",
        f"l2_hit_rate: {h_k / (h_k + m_k) if h_k + m_k else 0.0:.4f}",
        f"count_kernels_sha256: {count_source_sha256()}",
    ]
    return "\n".join(lines)


def read_summary(path):
    """Parses the ``key: value`` lines of a summary; None if missing."""
    return read_traffic(path)


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
    ap.add_argument("what", choices=["kernels", "counters", "traffic", "summary"])
    ap.add_argument("db", nargs="?")
    ap.add_argument("--top", type=int, default=40)
    ap.add_argument("--kernel", default=None)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--hitmiss")
    ap.add_argument("--dram")
    ap.add_argument("--variant", type=int)
    ap.add_argument("--workload")
    ap.add_argument("--command", default="")
    ap.add_argument("--bin", default=None, help="the bin (or bin range 'a-b' of one launch) summarised")
    ap.add_argument("--every", type=int, default=1, help="launches of the kernel per count")
    ap.add_argument("--offset", type=int, default=0, help="position of the bin's launch among them")
    a = ap.parse_args()
    if a.what == "kernels":
        print(kernel_stats(a.db, a.top))
    elif a.what == "counters":
        print(counter_stats(a.db, a.kernel))
    elif a.what == "summary":
        print(counters_summary(a.fetch, a.write, a.hitmiss, a.dram, a.kernel, a.variant, a.workload, a.command,
                               a.bin, a.every, a.offset))
    else:
        print(traffic_summary(a.fetch, a.write, a.kernel, a.variant, a.workload, a.command, a.bin, a.every,
                              a.offset))


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the single-graph path on one MI355X.

One step is one pass of the whole path over the resident edge list: CSR
build (validate, symmetrise, drop loops, sort, dedup), degree-order
orientation, binning (a1..a5), the intersection kernels and the clustering
epilogue (a6..a7). The edge list is generated on the host, copied to HBM
before the timed region, and stays there.

Prints one JSON line. ``value`` is m / step time, with m the number of
undirected simple edges (edges/s). ``roofline`` describes the dominant
intersection kernel (the bin whose kernel takes longest), timed with HIP
events on the stream it runs on: its achieved rate is the bytes that kernel
moves when nothing is reused between its work items (LDS-table lists, row
bounds, the shorter list streamed per edge, in-list chunks, credits; counted
exactly on the graph by tricc_graph_stats) over its launch time. The bytes a
merge of both lists would read (the classic sorted-list measure) are printed
beside it as a work measure, and the rocprofv3 counters of the same kernel
(DRAM-side bytes, L2 hit rate) are read from the committed summary while the
kernel source is unchanged. The other legs (batched graphs, serving, the
neighbouring methods) each carry their own figures; ``cpu_baseline`` is the
CPU oracle timed on a stated sample of the benchmarked graph on this host.
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

METRIC = "triangle-count edges/s vs HBM roofline; batched graphs/s; p50/p99 query latency"
HBM_PEAK_GBPS = 8000.0

WORKLOADS = {
    # name: (scale, edge_factor, seed)
    "rmat24": (24, 16, 24),
    "rmat22": (22, 16, 22),
    "rmat20": (20, 16, 20),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat24", choices=sorted(WORKLOADS) + ["er"])
    ap.add_argument("--cpu-sample-stride", type=int, default=256,
                    help="CPU oracle: count from the root nodes with id % stride == 0 on all host threads")
    ap.add_argument("--cpu-sample-stride1", type=int, default=8192,
                    help="CPU oracle: the same on one thread from id % stride1 == 0 (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default=None, help="JSON file with bin_limit / bin_variant")
    ap.add_argument("--out", default=None, help="also append the JSON line to this file")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-graphs leg")
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--no-per-graph", action="store_true",
                    help="skip the batched leg's per-graph-launch baseline (for profiling runs)")
    ap.add_argument("--autotune", action="store_true", help="search the batched tuning first (cached per arch)")
    ap.add_argument("--autotune-single", action="store_true",
                    help="search the single-graph bin tuning first (cached per arch/workload)")
    ap.add_argument("--no-edge-queries", action="store_true", help="skip the edge-existence leg")
    ap.add_argument("--no-bin-split", action="store_true",
                    help="skip the untimed per-bin launches that split merged launches by bin (for counter runs)")
    ap.add_argument("--no-core", action="store_true", help="skip the core-number leg")
    ap.add_argument("--no-degeneracy", action="store_true",
                    help="skip the degeneracy-order leg (triangles and 4-cliques under both orders)")
    ap.add_argument("--no-k4", action="store_true", help="skip the 4-clique leg")
    ap.add_argument("--no-gen", action="store_true", help="skip the device generator legs (R-MAT, G(n, m), BA)")
    ap.add_argument("--k4-scale", type=int, default=22, help="4-clique leg: R-MAT scale")
    ap.add_argument("--edge-n", type=int, default=10_000_000, help="edge-existence leg: ER nodes")
    ap.add_argument("--edge-m", type=int, default=100_000_000, help="edge-existence leg: ER edges (= queries)")
    ap.add_argument("--no-serving", action="store_true", help="skip the query-serving leg")
    ap.add_argument("--serve-queries", type=int, default=5000,
                    help="queries of the serving trace (the first ones of the 20,000-query trace's generator)")
    ap.add_argument("--serve-lambdas", default="0.5,0.8,0.95",
                    help="Poisson rates as fractions of the measured saturation rate")
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--serve-gb", type=float, default=24.0, help="server workspace (GB), also the admission budget")
    ap.add_argument("--serve-tune", action="store_true", help="pick the server's batch tuning on a sample first")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_1606_07550_amd import inputs as I
    if name == "er":
        s, d = I.er(10_000, 100_000, 1)
        return {"workload": "er", "n": 10_000, "m_raw": 100_000, "seed": 1}, 10_000, s, d
    scale, ef, seed = WORKLOADS[name]
    n, s, d = I.rmat(scale, ef, seed=seed)
    cfg = {"workload": f"rmat{scale}", "scale": scale, "edge_factor": ef, "n": n, "m_raw": int(s.size),
           "abcd": list(I.RMAT_ABCD), "noise": 0.1, "permuted": True, "seed": seed}
    return cfg, n, s, d


def probe_bandwidth(torch, N, nbytes=2 << 30, reps=5):
    """Achievable HBM bandwidth (read + write) of a streaming copy."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)
    N.check(N.lib().tricc_probe_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()), nbytes, sp),
            "probe")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        N.check(N.lib().tricc_probe_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()), nbytes,
                                         sp), "probe")
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9, ms


def build_line(ms, n, m_raw, m):
    """The build's compulsory bytes: the input pairs read once (8 per pair);
    the symmetric rows (4 per entry, 2m entries), the DAG's out- and
    in-lists (4 per entry each) written once; three offset arrays (8 per
    node) and three degree arrays (4 per node). Everything the sorts and
    the orientation move beyond that is above this floor."""
    b = 8 * m_raw + 4 * 2 * m + 4 * m + 4 * m + 3 * 8 * (n + 1) + 3 * 4 * n
    gbps = b / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"ms": ms, "compulsory_bytes": b, "GBps": gbps, "frac": gbps / HBM_PEAK_GBPS}


def launch_groups(variants):
    """The launches tricc_count issues for a tuning: one (first, last) bin
    range per run of adjacent bins with one kernel variant."""
    groups = []
    b0 = 0
    while b0 < len(variants):
        b1 = b0
        while b1 + 1 < len(variants) and variants[b1 + 1] == variants[b0]:
            b1 += 1
        groups.append((b0, b1))
        b0 = b1 + 1
    return groups


def measured_counters(workload, variant, bin):
    """rocprofv3 counters of the dominant kernel from the committed summary
    (profiles/counters_<workload>.md): DRAM-side bytes, L2 hit rate and the
    calibrated FETCH_SIZE + WRITE_SIZE traffic per launch, if they were taken
    on this workload, variant and bin (or bin range of one launch) with the
    current intersection-kernel source; else None."""
    from paper_1606_07550_amd import profiling
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", f"counters_{workload}.md")
    rec = profiling.read_summary(path)
    if not rec:
        return None
    if rec.get("count_kernels_sha256") != profiling.count_source_sha256() or int(rec.get("variant", -1)) != variant:
        return None
    if "bin" in rec and str(rec["bin"]).strip() != str(bin):
        return None
    out = {"source": f"profiles/counters_{workload}.md"}
    for k in ("traffic_bytes_per_launch", "dram_bytes_per_launch", "l2_hit_rate"):
        if k in rec:
            out[k] = float(rec[k])
    return out


def batched_leg(args, torch, P, N):
    """4096 independent BA / ER graphs (n log-uniform in [64, 65536]): one
    persistent launch captured in a hipGraph, against per-graph launches of
    the single-graph path on the same graphs."""
    from paper_1606_07550_amd import autotune
    from paper_1606_07550_amd import inputs as I
    dev = torch.device("cuda:0")
    G = args.batch_graphs
    t0 = time.perf_counter()
    bt = I.batch(G, 4096)
    log(f"generated batch G={G} nodes={bt['node_off'][-1]} pairs={bt['edge_off'][-1]} "
        f"in {time.perf_counter() - t0:.1f}s")
    src = torch.from_numpy(bt["src"]).to(dev)
    dst = torch.from_numpy(bt["dst"]).to(dev)
    key = f"batched-{G}"
    tuning = autotune.default_or_cached_batch(key)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = P.Batch(bt["node_off"], bt["edge_off"], src, dst, tuning=tuning)
    torch.cuda.synchronize()
    build_ms = 1e3 * (time.perf_counter() - t0)
    if args.autotune:
        tuning, _ = autotune.tune_batch(b, key=key, log=log)
    b.plan()
    stream = torch.cuda.current_stream()
    for _ in range(2):
        b.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.batch_reps):
        b.run()
    e1.record(stream)
    torch.cuda.synchronize()
    launch_ms = e0.elapsed_time(e1) / args.batch_reps
    info = b.info
    # algorithmic bytes of the whole batch, from the union graph
    gptr = N.lib().tricc_batch_graph(b._h)
    N.check(N.lib().tricc_graph_stats(gptr, ctypes.c_void_p(stream.cuda_stream)), "tricc_graph_stats")
    gi = N.GraphInfo()
    N.check(N.lib().tricc_graph_info_get(gptr, ctypes.byref(gi)), "tricc_graph_info_get")
    n_tot = int(bt["node_off"][-1])
    alg = 4 * gi.list_elems + 4 * gi.m + 8 * (n_tot + G) + 12 * n_tot
    tri = int(b.out["graph_tri"].sum().item())
    out = {
        "workload": f"batched-{G}", "graphs": G, "nodes": n_tot, "pairs": int(bt["edge_off"][-1]), "m": int(gi.m),
        "triangles": tri,
        "graphs_per_s": G / (launch_ms * 1e-3), "launch_ms": launch_ms, "edges_per_s": gi.m / (launch_ms * 1e-3),
        "alg_bytes": alg, "achieved_GBps": alg / (launch_ms * 1e-3) / 1e9,
        "frac": alg / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        "build_ms": build_ms, "tuning": tuning, "grid": info["grid"],
        "lists": {"merge": info["merge_nodes"], "wave": info["wave_nodes"], "block": info["block_nodes"],
                  "hub": info["hub_nodes"]},
    }
    if args.no_per_graph:
        return out
    # per-graph launches of the single-graph path on the same graphs
    log("building per-graph handles for the baseline ...")
    graphs = []
    for g in range(G):
        e_a, e_b = bt["edge_off"][g], bt["edge_off"][g + 1]
        graphs.append(P.Graph(int(bt["n"][g]), src[e_a:e_b], dst[e_a:e_b]))
    outs = [{"T": torch.empty(gr.n, dtype=torch.int64, device=dev),
             "cc": torch.empty(gr.n, dtype=torch.float32, device=dev),
             "total": torch.empty(1, dtype=torch.int64, device=dev),
             "avg": torch.empty(1, dtype=torch.float64, device=dev)} for gr in graphs]
    for gr, o in zip(graphs, outs):
        gr.count(out=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for gr, o in zip(graphs, outs):
        gr.count(out=o)
    torch.cuda.synchronize()
    per_graph_ms = 1e3 * (time.perf_counter() - t0)
    tri_pg = sum(int(o["total"].item()) for o in outs)
    del graphs, outs
    out["triangles_match_per_graph"] = tri == tri_pg
    out["per_graph_launches"] = {"graphs_per_s": G / (per_graph_ms * 1e-3), "ms": per_graph_ms}
    out["speedup_vs_per_graph"] = per_graph_ms / launch_ms
    return out


def run_trace(P, N, g, queries, arrivals, slots, max_batch, budget, tuning=None):
    """Replays a query trace against a fresh server. arrivals: offsets in
    seconds from the start (None: all at once). Latency = completion seen on
    the host - scheduled arrival (includes queueing and admission waits)."""
    srv = P.Server(g, budget, slots=slots, max_batch_queries=max_batch)
    if tuning is not None:
        srv.set_tuning(tuning)
    Q = len(queries)
    t0 = srv.now() + 0.01
    results = {}
    i = 0
    while len(results) < Q:
        now = srv.now()
        progressed = False
        while i < Q and (arrivals is None or t0 + arrivals[i] <= now):
            ta = t0 + (arrivals[i] if arrivals is not None else 0.0)
            if srv.submit(i, queries[i], t_arrival=ta) == N.TRICC_EBUSY:
                break
            i += 1
            progressed = True
        for r in srv.poll():
            results[r["qid"]] = r
            progressed = True
        if not progressed:
            time.sleep(0.0002)
    srv.drain()
    srv.close()
    bad = sum(1 for r in results.values() if r["status"] != 0)
    lat = np.array([r["t_done"] - r["t_arrival"] for r in results.values()])
    t_end = max(r["t_done"] for r in results.values())
    t_first = t0 + (arrivals[0] if arrivals is not None else 0.0)
    return {
        "queries": Q, "failed": bad, "qps": Q / (t_end - t_first),
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_batch": float(np.mean([r["batch_size"] for r in results.values()])),
        "triangles": int(sum(r["triangles"] for r in results.values())),
        "edges": int(sum(r["m"] for r in results.values())),
        "edges_per_s": sum(r["m"] for r in results.values()) / (t_end - t_first),
    }


def core_leg(g, torch, m):
    """Core numbers on the benchmark's graph: the 3-core (the paper times its
    extraction, Section 6.3) and the full decomposition, each timed on the
    host around the call (it synchronises: the peeling loop reads frontier
    sizes back). Rate = undirected edges / time."""
    out = {}
    for name, k in (("three_core", 3), ("full", -1)):
        g.core(k)  # warm-up
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            c, mx = g.core(k)
        sec = (time.perf_counter() - t0) / reps
        out[name] = {"k_stop": k, "ms": 1e3 * sec, "edges_per_s": m / sec, "max_core": mx,
                     "nodes_at_max": int((c == mx).sum().item())}
    return out


def gen_leg(args, torch, P, N):
    """Device R-MAT generator on the benchmark's own graph (R-MAT 24, edge
    factor 16, relabelled), timed with HIP events around the kernel on its
    stream, against the host input generator that the other legs use (same
    edges, bit for bit) and the oracle's R-MAT on a 2M-edge sample."""
    from paper_1606_07550_amd import inputs as I
    from paper_1606_07550_amd.generators import rmat
    dev = torch.device("cuda:0")
    sc = 24
    perm_h = I.rmat_perm(sc, sc)
    perm = torch.from_numpy(perm_h).to(dev)
    m = 16 << sc
    out = (torch.empty(m, dtype=torch.int32, device=dev), torch.empty(m, dtype=torch.int32, device=dev))
    stream = torch.cuda.current_stream()
    rmat(sc, seed=sc, perm=perm, out=out, stream=stream)
    reps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        rmat(sc, seed=sc, perm=perm, out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    _, hs, hd = I.rmat(sc, 16, seed=sc, threads=threads)
    host_s = time.perf_counter() - t0
    sample = np.random.default_rng(1).integers(0, m, 4096)
    ti = torch.from_numpy(sample).to(dev)
    same = bool(np.array_equal(out[0][ti].cpu().numpy(), hs[sample])
                and np.array_equal(out[1][ti].cpu().numpy(), hd[sample]))
    line = {"workload": f"rmat{sc}-ef16", "edges": m, "ms": ms, "edges_per_s": m / (ms * 1e-3),
            "write_GBps": 8 * m / (ms * 1e-3) / 1e9, "host_generator": {"s": host_s, "threads": threads,
                                                                        "edges_per_s": m / host_s},
            "sampled_edges_equal_host": same}
    del out, perm
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        import oracle
        k = 2_000_000
        t0 = time.perf_counter()
        oracle.rmat(sc, k, seed=sc, perm=perm_h)
        sec = time.perf_counter() - t0
        line["cpu_oracle"] = {"value": k / sec, "unit": "edges/s", "kind": "oracle", "cores": 1,
                              "sample": f"first {k} edges of R-MAT 24, relabelled, {sec:.2f} s"}
    return line


def gen_er_ba_leg(args, torch, P, N):
    """Device G(n, m) and Barabasi-Albert generators at the sizes the other
    legs use: G(10^7, 10^8) (the edge-existence workload) and BA with n =
    2^22, k = 16 (the batch's largest attachment count), each timed on the
    host around the call (both synchronise), against the host input
    generators and the oracle's generators of the same definitions on a
    prefix (the first edges of a smaller instance of the same seed)."""
    from paper_1606_07550_amd import generators as GEN
    from paper_1606_07550_amd import inputs as I
    import oracle
    dev = torch.device("cuda:0")
    out = {}
    n, m = args.edge_n, args.edge_m
    need = ctypes.c_size_t()
    N.check(N.lib().tricc_gen_er_workspace_size(n, m, ctypes.byref(need)), "ws")
    ws = torch.empty(need.value, dtype=torch.uint8, device=dev)
    buf = (torch.empty(m, dtype=torch.int32, device=dev), torch.empty(m, dtype=torch.int32, device=dev))
    GEN.er(n, m, seed=2016, out=buf, workspace=ws)
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        GEN.er(n, m, seed=2016, out=buf, workspace=ws)
    sec = (time.perf_counter() - t0) / reps
    k = 1_000_000
    t1 = time.perf_counter()
    so, do = oracle.er(n, k, 2016)
    osec = time.perf_counter() - t1
    same = bool(np.array_equal(buf[0][:k].cpu().numpy(), so) and np.array_equal(buf[1][:k].cpu().numpy(), do))
    t1 = time.perf_counter()
    I.er(n, m, 2016)
    hsec = time.perf_counter() - t1
    out["er"] = {"workload": f"er-n{n}-m{m}", "ms": 1e3 * sec, "edges_per_s": m / sec, "workspace_bytes": need.value,
                 "prefix_equal_oracle": same,
                 "cpu_oracle": {"value": k / osec, "unit": "edges/s", "kind": "oracle", "cores": 1,
                                "sample": f"the first {k} edges of the same definition, {osec:.2f} s"},
                 "host_input_generator": {"s": hsec, "edges_per_s": m / hsec,
                                          "note": "the tests' own G(n, m) sampler (Floyd), not this definition"}}
    del ws, buf
    torch.cuda.empty_cache()
    n, kk = 1 << 22, 16
    mb = GEN.ba_edges(n, kk)
    buf = (torch.empty(mb, dtype=torch.int32, device=dev), torch.empty(mb, dtype=torch.int32, device=dev))
    GEN.ba(n, kk, seed=22, out=buf)
    t0 = time.perf_counter()
    for _ in range(reps):
        GEN.ba(n, kk, seed=22, out=buf)
    sec = (time.perf_counter() - t0) / reps
    n1 = 1 << 16
    t1 = time.perf_counter()
    so, do = oracle.ba(n1, kk, 22)
    osec = time.perf_counter() - t1
    same = bool(np.array_equal(buf[0][:so.size].cpu().numpy(), so) and
                np.array_equal(buf[1][:do.size].cpu().numpy(), do))
    out["ba"] = {"workload": f"ba-n{n}-k{kk}", "edges": mb, "ms": 1e3 * sec, "edges_per_s": mb / sec,
                 "prefix_equal_oracle": same,
                 "cpu_oracle": {"value": so.size / osec, "unit": "edges/s", "kind": "oracle", "cores": 1,
                                "sample": f"BA(n={n1}, k={kk}) of the same seed (a prefix), {osec:.2f} s"}}
    del buf
    torch.cuda.empty_cache()
    return out


def k4_leg(args, torch, P, N):
    """4-clique count on R-MAT (same generator parameters as the main
    workload) at --k4-scale, timed with HIP events around the kernel on its
    stream; rate = undirected edges / time. The CPU oracle's rate is taken
    on R-MAT 16."""
    from paper_1606_07550_amd import inputs as I
    dev = torch.device("cuda:0")
    sc = args.k4_scale
    n, s, d = I.rmat(sc, 16, seed=sc)
    g = P.Graph(n, torch.from_numpy(s).to(dev), torch.from_numpy(d).to(dev))
    m = int(g.info["m"])
    out = torch.empty(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    g.count_k4(out=out, stream=stream)
    reps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        g.count_k4(out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    line = {"workload": f"rmat{sc}", "n": n, "m": m, "max_outdeg": int(g.info["max_outdeg"]),
            "cliques4": int(out.cpu().numpy().view(np.uint64)[0]), "ms": ms, "edges_per_s": m / (ms * 1e-3)}
    del g, out
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
        n1, s1, d1 = I.rmat(16, 16, seed=16)
        t0 = time.perf_counter()
        c1 = oracle.k4(n1, s1, d1, order=1, threads=threads)
        sec = time.perf_counter() - t0
        m1 = oracle.count(n1, s1, d1)["m"]
        line["cpu_oracle"] = {"value": m1 / sec, "unit": "edges/s", "kind": "oracle", "cores": threads,
                              "sample": f"R-MAT scale 16 (m={m1}, {c1} 4-cliques), build + count {sec:.2f} s"}
    return line


def edge_query_leg(args, torch, P, N):
    """Edge-existence tests as the paper times them (Section 6.2): an ER graph
    G(n, m) and m tests of random (source, destination) pairs, here the
    paper's largest configuration (10M nodes, 100M edges). Timed with HIP
    events around the query kernel on its stream, inputs resident in HBM.
    Algorithmic bytes per query: the pair (8) and its result (1), both
    degrees (8), the shorter row's start (8), and 4 bytes per step of the
    binary search, ceil(log2(d_min + 1)) steps."""
    from paper_1606_07550_amd import inputs as I
    dev = torch.device("cuda:0")
    n, m = args.edge_n, args.edge_m
    t0 = time.perf_counter()
    s, d = I.er(n, m, 2016)
    log(f"edge-existence leg: G(n={n}, m={m}) generated in {time.perf_counter() - t0:.1f}s")
    g = P.Graph(n, torch.from_numpy(s).to(dev), torch.from_numpy(d).to(dev))
    gen = torch.Generator(device=dev)
    gen.manual_seed(2017)
    qu = torch.randint(0, n, (m,), dtype=torch.int32, device=dev, generator=gen)
    qv = torch.randint(0, n, (m,), dtype=torch.int32, device=dev, generator=gen)
    out = torch.empty(m, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        g.has_edges(qu, qv, out=out, stream=stream)
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        g.has_edges(qu, qv, out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    deg = g.arrays()["deg"]
    dmin = torch.minimum(deg[qu.long()], deg[qv.long()]).double()
    steps = torch.ceil(torch.log2(dmin + 1.0))
    alg = float((8 + 1 + 8 + 8) * m + 4.0 * steps.sum().item())
    positives = int((out == 1).sum().item())
    # every input pair must test positive (a property that holds at any size)
    k = min(m, 1 << 22)
    pos = g.has_edges(torch.from_numpy(s[:k]).to(dev), torch.from_numpy(d[:k]).to(dev))
    line = {
        "workload": f"er-n{n}-m{m}", "n": n, "m": int(g.info["m"]), "queries": m, "ms": ms,
        "queries_per_s": m / (ms * 1e-3), "positives": positives, "input_pairs_all_positive": bool(pos.all().item()),
        "roofline": {"bound": "hbm", "achieved": alg / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, "alg_bytes_per_launch": alg,
                     "kernel": "k_has_edges", "kernel_ms": ms},
    }
    del g, qu, qv, out, deg, dmin, steps, pos
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        import oracle
        n1, m1 = 1_000_000, 10_000_000
        s1, d1 = I.er(n1, m1, 2018)
        rng = np.random.default_rng(2019)
        q1u = rng.integers(0, n1, m1).astype(np.int32)
        q1v = rng.integers(0, n1, m1).astype(np.int32)
        t0 = oracle.wtime()
        oracle.has_edges(n1, s1, d1, q1u, q1v)
        sec = oracle.wtime() - t0
        line["cpu_oracle"] = {"value": m1 / sec, "unit": "queries/s", "kind": "oracle",
                              "cores": int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0)),
                              "sample": f"G(n={n1}, m={m1}), {m1} random queries; edge-key sort + searches "
                                        f"{sec:.2f} s"}
    return line


def serving_leg(args, torch, P, N):
    """Resident R-MAT scale 22 (edge factor 16, same a,b,c,d); BFS-ball
    queries of log-uniform size in [16, 100000] (seed 2022; the first
    --serve-queries of the 20,000-query trace, whose queries are drawn per
    index). The continuous-batching server's saturation throughput (all
    queries submitted at once), then open-loop Poisson traces at the given
    fractions of it; the baseline is a FIFO server with one query per launch,
    measured the same way (saturation, and Poisson at 0.8 x its own
    saturation). Latency = completion seen on the host - scheduled arrival."""
    from paper_1606_07550_amd import inputs as I
    dev = torch.device("cuda:0")
    n, s, d = I.rmat(22, 16, seed=22)
    t0 = time.perf_counter()
    Q = args.serve_queries
    off, nodes, _ = I.bfs_queries(n, s, d, Q, seed=2022)
    log(f"generated {Q} BFS-ball queries ({off[-1]} nodes) in {time.perf_counter() - t0:.1f}s")
    queries = [nodes[off[q]:off[q + 1]] for q in range(Q)]
    g = P.Graph(n, torch.from_numpy(s).to(dev), torch.from_numpy(d).to(dev))
    budget = int(args.serve_gb * 1e9)
    tuning = None
    if args.serve_tune:
        best = None
        from paper_1606_07550_amd.autotune import MERGE_CAP
        for ml in (0, 4, 8, 16, 32):
            for pv in sorted(MERGE_CAP):
                if ml > MERGE_CAP[pv]:
                    continue  # above the variant's short-list path
                t = {"merge_limit": ml, "wave_limit": 64, "persist_variant": pv, "blocks_per_cu": 0}
                r = run_trace(P, N, g, queries[:max(200, Q // 10)], None, args.serve_slots, 256, budget, t)
                log(f"serve tuning {t}: {r['qps']:.1f} q/s")
                if best is None or r["qps"] > best[0]:
                    best = (r["qps"], t)
        tuning = best[1]
    sat = run_trace(P, N, g, queries, None, args.serve_slots, 256, budget, tuning)
    log(f"saturation: {sat}")
    sweep = []
    for frac in [float(x) for x in args.serve_lambdas.split(",") if x]:
        lam = frac * sat["qps"]
        arr = I.poisson_arrivals(Q, lam, 4)
        arr = arr - arr[0]
        r = run_trace(P, N, g, queries, arr, args.serve_slots, 256, budget, tuning)
        r.update(lambda_frac=frac, lambda_qps=lam)
        log(f"poisson at {lam:.1f}/s ({frac} x saturation): {r}")
        sweep.append(r)
    fifo_sat = run_trace(P, N, g, queries, None, 1, 1, budget, tuning)
    log(f"fifo saturation: {fifo_sat}")
    lam_f = 0.8 * fifo_sat["qps"]
    arr = I.poisson_arrivals(Q, lam_f, 4)
    fifo_pois = run_trace(P, N, g, queries, arr - arr[0], 1, 1, budget, tuning)
    fifo_pois.update(lambda_frac=0.8, lambda_qps=lam_f)
    log(f"fifo poisson at {lam_f:.1f}/s: {fifo_pois}")
    main_pt = min(sweep, key=lambda r: abs(r["lambda_frac"] - 0.8)) if sweep else sat
    return {
        "workload": f"serving-rmat22-{Q}", "resident": {"n": n, "m": g.info["m"]},
        "queries": Q, "query_nodes": int(off[-1]), "slots": args.serve_slots, "budget_bytes": budget,
        "tuning": tuning,
        "qps": main_pt["qps"], "p50_ms": main_pt["p50_ms"], "p99_ms": main_pt["p99_ms"],
        "lambda_qps": main_pt.get("lambda_qps"), "lambda_frac": main_pt.get("lambda_frac"),
        "saturation": sat, "poisson_sweep": sweep,
        "fifo_per_query": {"saturation": fifo_sat, "poisson": fifo_pois},
        "speedup_vs_fifo_saturation": sat["qps"] / fifo_sat["qps"],
    }


def cpu_baseline(args, n, s, d, m):
    """The CPU oracle on the benchmarked graph itself: its build (symmetrise,
    dedup, sorted rows) over all input pairs, timed apart, then its node
    iterator from a sample of root nodes (ids = 0 mod stride; ids are a random
    permutation, so this is a uniform sample of the per-root work), on all
    host threads and, on a smaller sample, on one thread (the paper's
    protocol is one core). The count rate is m / (sample time x stride)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    st, st1 = args.cpu_sample_stride, args.cpu_sample_stride1
    r = oracle.count_timed(n, s, d, order=1, threads=threads, stride=st, offset=0, stride1=st1)
    est = r["count_s"] * st
    line = {"value": m / est, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": f"the benchmarked R-MAT graph (m={r['m']}): build over all {len(s)} input pairs "
                      f"{r['build_s']:.1f} s (timed apart); node iterator from the roots with id % {st} == 0 "
                      f"({r['tri']} triangles) {r['count_s']:.2f} s on {threads} threads, scaled x{st}",
            "build_s": r["build_s"], "count_s_sample": r["count_s"], "count_s_full_est": est,
            "build_plus_count_edges_per_s": m / (r["build_s"] + est)}
    if st1 > 0:
        est1 = r["count1_s"] * st1
        line["one_thread"] = {"value": m / est1, "unit": "edges/s", "cores": 1,
                              "sample": f"roots with id % {st1} == 0 ({r['tri1']} triangles) "
                                        f"{r['count1_s']:.2f} s, scaled x{st1}",
                              "count_s_full_est": est1}
    return line


def degeneracy_leg(g, torch, P, N):
    """The benchmark's graph under the degree order and under the degeneracy
    order (tricc_graph_degeneracy + tricc_graph_reorient): largest out-degree,
    count time (a6 + a7, HIP events) and 4-clique time for both; the counts
    must agree. The degeneracy order is left on the graph afterwards."""
    stream = torch.cuda.current_stream()

    def time_count(reps=3):
        g.count()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            o = g.count()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, int(o["total"].cpu().numpy().view(np.uint64)[0])

    def time_k4():
        if g.info["max_outdeg"] > 4096:
            return None, None
        out = g.count_k4()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.count_k4(out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), int(out.cpu().numpy().view(np.uint64)[0])

    res = {}
    c_ms, tri = time_count()
    k_ms, k4 = time_k4()
    res["degree"] = {"max_outdeg": g.info["max_outdeg"], "count_ms": c_ms, "triangles": tri, "k4_ms": k_ms,
                     "cliques4": k4}
    t0 = time.perf_counter()
    order, _, dg = g.degeneracy()
    t1 = time.perf_counter()
    try:
        g.reorient(order)
    except N.TriccError:
        g.retune(P.default_tuning())
        g.reorient(order)
    t2 = time.perf_counter()
    c_ms, tri2 = time_count()
    k_ms, k42 = time_k4()
    res["degeneracy"] = {"degeneracy": dg, "max_outdeg": g.info["max_outdeg"], "order_ms": 1e3 * (t1 - t0),
                         "reorient_ms": 1e3 * (t2 - t1), "count_ms": c_ms, "triangles": tri2, "k4_ms": k_ms,
                         "cliques4": k42}
    res["counts_equal"] = tri == tri2 and k4 == k42
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported (this path runs on a "
              "single device; several GPUs would each take a share of the binned work lists and sum "
              "their per-node counts with one all-reduce)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1606_07550_amd as P
    from paper_1606_07550_amd import _native as N

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    cfg, n, s, d = make_workload(args.workload)
    log(f"generated {cfg['workload']} n={n} m_raw={s.size} in {time.perf_counter() - t0:.1f}s")
    src = torch.from_numpy(s).to(dev)
    dst = torch.from_numpy(d).to(dev)
    host_pairs = (s, d)  # the CPU oracle's input (the same arrays)
    del s, d
    from paper_1606_07550_amd import autotune
    tuning = None
    if args.tuning:
        with open(args.tuning) as f:
            tuning = N.Tuning.from_dict(json.load(f))
    elif args.autotune_single:
        g0 = P.Graph(n, src, dst)
        best, ms = autotune.tune_single(g0, key=cfg["workload"], log=log)
        log(f"autotuned {cfg['workload']}: {best} ({ms:.2f} ms of intersection kernels)")
        tuning = N.Tuning.from_dict(best)
        del g0
    else:
        rec = autotune.lookup(cfg["workload"])
        if rec:
            tuning = N.Tuning.from_dict(rec["tuning"])
    ws = torch.empty(P.workspace_size(n, src.numel()), dtype=torch.uint8, device=dev)
    T = torch.empty(n, dtype=torch.int64, device=dev)
    cc = torch.empty(n, dtype=torch.float32, device=dev)
    total = torch.empty(1, dtype=torch.int64, device=dev)
    avg = torch.empty(1, dtype=torch.float64, device=dev)
    L = N.lib()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    nb = N.NUM_BINS
    tuning_used = (tuning or P.default_tuning()).as_dict()
    variants = tuning_used["bin_variant"]
    groups = launch_groups(variants)
    launch_ms = [0.0] * len(groups)
    launch_n = [0] * len(groups)

    def step(timed):
        tb0 = time.perf_counter()
        g = P.Graph(n, src, dst, tuning=tuning, workspace=ws)
        tb1 = time.perf_counter()
        h = g._h
        N.check(L.tricc_count_begin(h, ptr(T), sp), "begin")
        evs = []
        for gi, (b0, b1) in enumerate(groups):
            if sum(g.info["bin_count"][b0:b1 + 1]) == 0:
                continue
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            N.check(L.tricc_count_bins(h, b0, b1, ptr(T), sp), "bins")
            e1.record(stream)
            evs.append((gi, e0, e1))
        N.check(L.tricc_count_finish(h, ptr(T), ptr(cc), ptr(total), ptr(avg), sp), "finish")
        if timed:
            torch.cuda.synchronize()
            for gi, e0, e1 in evs:
                launch_ms[gi] += e0.elapsed_time(e1)
                launch_n[gi] += 1
        return g, tb1 - tb0

    for i in range(args.warmup):
        g, _ = step(False)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    build_s = 0.0
    for i in range(args.steps):
        g, bs = step(True)
        build_s += bs
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_total / args.steps
    info = g.stats()
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")

    # count-only timing (a6..a7) with events
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(3, args.steps)
    e0.record(stream)
    for _ in range(reps):
        g.count(out={"T": T, "cc": cc, "total": total, "avg": avg})
    e1.record(stream)
    torch.cuda.synchronize()
    count_ms = e0.elapsed_time(e1) / reps

    # untimed: every bin in a launch of its own, to split merged launches by bin
    bin_ms = None
    if not args.no_bin_split:
        bin_ms = [0.0] * nb
        split_reps = 2
        h = g._h
        for _ in range(split_reps):
            N.check(L.tricc_count_begin(h, ptr(T), sp), "begin")
            evs = []
            for b in range(nb):
                if g.info["bin_count"][b] == 0:
                    continue
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                N.check(L.tricc_count_bin(h, b, ptr(T), sp), "bin")
                e1.record(stream)
                evs.append((b, e0, e1))
            N.check(L.tricc_count_finish(h, ptr(T), ptr(cc), ptr(total), ptr(avg), sp), "finish")
            torch.cuda.synchronize()
            for b, e0, e1 in evs:
                bin_ms[b] += e0.elapsed_time(e1) / split_reps

    m = info["m"]
    tri = int(total.cpu().item())
    # dominant intersection launch of the timed steps
    avg_launch_ms = [launch_ms[i] / launch_n[i] if launch_n[i] else 0.0 for i in range(len(groups))]
    dom_g = max(range(len(groups)), key=lambda i: avg_launch_ms[i])
    d0, d1 = groups[dom_g]
    dom_label = f"{d0}-{d1}" if d1 > d0 else f"{d0}"
    dom_s = avg_launch_ms[dom_g] * 1e-3
    dom_kbytes = sum(info["bin_kernel_bytes"][d0:d1 + 1])
    dom_merge = sum(4 * info["bin_list_elems"][b] + 4 * info["bin_edges"][b] for b in range(d0, d1 + 1))
    achieved = dom_kbytes / dom_s / 1e9 if dom_s > 0 else 0.0
    stage_bytes = 4 * info["list_elems"] + 4 * m + 8 * (n + 1) + 12 * n
    stage_kbytes = sum(info["bin_kernel_bytes"]) + 8 * (n + 1) + 12 * n
    a6_ms = sum(avg_launch_ms)
    variant = variants[d0]
    prof = measured_counters(cfg["workload"], variant, dom_label)
    traffic = prof.get("traffic_bytes_per_launch") if prof else None
    bw, _ = probe_bandwidth(torch, N)
    line = {
        "metric": METRIC,
        "value": m / (ms_per_step * 1e-3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": dict(cfg, m=m, triangles=tri, max_deg=info["max_deg"], max_outdeg=info["max_outdeg"],
                       tuning=tuning_used),
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "kernel": f"intersection {'bins' if d1 > d0 else 'bin'} {dom_label} (variant {variant}, one launch)",
            "kernel_ms": avg_launch_ms[dom_g],
            # bytes the min-side kernel moves with no reuse between its work
            # items (exact count on this graph); the merge measure (both lists
            # read per edge) is a work measure, not a bandwidth
            "alg_bytes_per_launch": dom_kbytes,
            "merge_bytes_per_launch": dom_merge,
            "merge_GBps": dom_merge / dom_s / 1e9 if dom_s > 0 else 0.0,
            # rocprofv3 counters of this kernel (committed summary; null once
            # the kernel source has changed since they were taken)
            "traffic_GBps": traffic / dom_s / 1e9 if traffic else None,
            "traffic_frac": traffic / dom_s / 1e9 / HBM_PEAK_GBPS if traffic else None,
            "l2_hit_rate": prof.get("l2_hit_rate") if prof else None,
            "dram_bytes_per_launch": prof.get("dram_bytes_per_launch") if prof else None,
            "counters": prof.get("source") if prof else None,
        },
        "stage_a6": {"ms": a6_ms, "kernel_bytes": stage_kbytes,
                     "kernel_GBps": stage_kbytes / (a6_ms * 1e-3) / 1e9 if a6_ms else 0.0,
                     "kernel_frac": stage_kbytes / (a6_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS if a6_ms else 0.0,
                     "merge_bytes": stage_bytes,
                     "compulsory_bytes": 4 * m + 8 * (n + 1) + 12 * n,
                     "launches": [{"bins": [b0, b1], "variant": variants[b0], "ms": avg_launch_ms[i],
                                   "kernel_bytes": sum(info["bin_kernel_bytes"][b0:b1 + 1]),
                                   "kernel_GBps": sum(info["bin_kernel_bytes"][b0:b1 + 1])
                                   / (avg_launch_ms[i] * 1e-3) / 1e9 if avg_launch_ms[i] > 0 else 0.0}
                                  for i, (b0, b1) in enumerate(groups)],
                     # untimed per-bin launches (one bin each)
                     "bin_ms": bin_ms, "bin_count": info["bin_count"],
                     "bin_kernel_bytes": info["bin_kernel_bytes"],
                     "bin_kernel_GBps": [info["bin_kernel_bytes"][b] / (bin_ms[b] * 1e-3) / 1e9
                                         if bin_ms and bin_ms[b] > 0 else 0.0 for b in range(nb)]},
        "count_only": {"ms": count_ms, "edges_per_s": m / (count_ms * 1e-3)},
        "build_ms": 1e3 * build_s / args.steps,
        "build": build_line(1e3 * build_s / args.steps, n, int(src.numel()), m),
        "probe_copy_GBps": bw,
    }
    if not args.no_core:
        log("core-number leg ...")
        line["core"] = core_leg(g, torch, m)
    if not args.no_degeneracy:
        log("degeneracy-order leg ...")
        line["degeneracy"] = degeneracy_leg(g, torch, P, N)
    del src, dst, ws, T, cc, g
    torch.cuda.empty_cache()
    if not args.no_batched:
        log("batched leg ...")
        line["batched"] = batched_leg(args, torch, P, N)
    if not args.no_gen:
        log("generator leg ...")
        line["generator"] = gen_leg(args, torch, P, N)
        log("G(n, m) and Barabasi-Albert generator leg ...")
        line["generator"].update(gen_er_ba_leg(args, torch, P, N))
    if not args.no_k4:
        log("4-clique leg ...")
        line["k4"] = k4_leg(args, torch, P, N)
    if not args.no_edge_queries:
        log("edge-existence leg ...")
        line["edge_queries"] = edge_query_leg(args, torch, P, N)
    if not args.no_serving:
        log("serving leg ...")
        line["serving"] = serving_leg(args, torch, P, N)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on its sample ...")
        line["cpu_baseline"] = cpu_baseline(args, n, host_pairs[0], host_pairs[1], m)
    else:
        line["cpu_baseline"] = None
    text = json.dumps(line)
    print(text, flush=True)
    if args.out:
        with open(args.out, "a") as f:
            f.write(text + "\n")


if __name__ == "__main__":
    main()

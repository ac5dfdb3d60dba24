"""Autotuner for the intersection kernels.

Single graph: coordinate search over each bin's kernel variant (among those
whose capacity covers the bin) and over a few sets of bin limits, timing
each bin's kernel alone with events on its stream.
Batch: grid search over the persistent kernel's work split (merge_limit,
wave_limit), its variant (block-table capacity, short-list path) and grid
size (blocks_per_cu),
timing whole graph launches.

Results are cached in ``tuning_cache.json`` next to this file, keyed by
"<gcn arch>/<workload class>"; the tuned values are plain ints, so a cache
entry can be passed straight back as a tuning.
"""
import ctypes
import json
import os

import torch

from . import _native as N
from .batch import default_batch_tuning
from .graph import default_tuning, variant_capacity, variant_count

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")

LIMIT_SETS = [
    [64, 256, 1024, 2048, 4096],
    [64, 256, 512, 1024, 4096],
    [32, 128, 512, 1024, 4096],
    [64, 128, 512, 1024, 4096],
    [32, 128, 256, 1024, 4096],
    [64, 256, 512, 768, 4096],
    [64, 256, 640, 1024, 4096],
    [64, 256, 512, 1024, 2048],
    [96, 256, 512, 1024, 4096],
    [64, 192, 512, 1024, 4096],
]


def arch():
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def load_cache():
    if not os.path.exists(CACHE):
        return {}
    with open(CACHE) as f:
        return json.load(f)


def lookup(key):
    return load_cache().get(f"{arch()}/{key}")


def store(key, value):
    c = load_cache()
    c[f"{arch()}/{key}"] = value
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def _time(fn, reps):
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _bin_ms(graph, T, b, reps):
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = N.lib()
    h = graph._h
    tp = ctypes.c_void_p(T.data_ptr())

    def run():
        N.check(L.tricc_count_bin(h, b, tp, sp), "tricc_count_bin")
    return _time(run, reps)


def tune_single(graph, reps=3, key=None, log=None, min_side=(1,)):
    """Tunes a built :class:`Graph` in place; returns (tuning dict, ms).
    With min_side on, bins 0..4 only take min-side variants (min_side=(1, 0)
    also searches the variants that count every edge from its tail)."""
    T = torch.zeros(max(graph.n, 1), dtype=torch.int64, device=graph.device)
    best_total, best = None, None
    max_outdeg = graph.info["max_outdeg"]
    ms_ok = [bool(N.lib().tricc_variant_min_side(v)) for v in range(variant_count())]
    for ms, limits in [(m, lim) for m in min_side for lim in LIMIT_SETS]:
        t = default_tuning().as_dict()
        t["bin_limit"] = list(limits)
        t["min_side"] = ms
        # start from variants that fit, then improve bin by bin
        for b in range(N.NUM_BINS):
            bound = max_outdeg if b == N.NUM_BINS - 1 else min(limits[b], max_outdeg)
            if variant_capacity(t["bin_variant"][b]) < bound:
                fits = [v for v in range(variant_count()) if variant_capacity(v) >= bound
                        and (not ms or b == N.NUM_BINS - 1 or ms_ok[v])]
                t["bin_variant"][b] = min(fits, key=variant_capacity)
        graph.retune(t)
        total = 0.0
        for b in range(N.NUM_BINS):
            if graph.info["bin_count"][b] == 0:
                continue
            bound = max_outdeg if b == N.NUM_BINS - 1 else min(limits[b], max_outdeg)
            cands = [v for v in range(variant_count()) if variant_capacity(v) >= bound
                     and (not ms or b == N.NUM_BINS - 1 or ms_ok[v])]
            best_v, best_ms = None, None
            for v in cands:
                t2 = dict(t, bin_variant=list(t["bin_variant"]))
                t2["bin_variant"][b] = v
                graph.retune(t2)
                bin_ms = _bin_ms(graph, T, b, reps)
                if best_ms is None or bin_ms < best_ms:
                    best_v, best_ms = v, bin_ms
            t["bin_variant"][b] = best_v
            total += best_ms
        if log:
            log(f"min_side {ms} limits {limits}: {total:.2f} ms {t['bin_variant']}")
        if best_total is None or total < best_total:
            best_total, best = total, t
    graph.retune(best)
    if key:
        store(key, {"tuning": best, "ms": best_total})
    return best, best_total


# largest merge_limit of each persistent variant's short-list path
MERGE_CAP = {0: 64, 1: 64, 2: 16, 3: 16, 4: 32, 5: 8, 6: 16, 7: 16}
BATCH_SPACE = [(ml, wl, pv, bpc) for pv in sorted(MERGE_CAP) for wl in (32, 64) for ml in (0, 8, 16, 32, 64)
               for bpc in (0, 4) if ml <= wl and ml <= MERGE_CAP[pv]]


def tune_batch(batch, reps=3, key=None, log=None):
    """Tunes a built :class:`Batch` in place (and re-plans it); returns
    (tuning dict, ms per launch)."""
    best_ms, best = None, None
    for ml, wl, pv, bpc in BATCH_SPACE:
        t = {"merge_limit": ml, "wave_limit": wl, "persist_variant": pv, "blocks_per_cu": bpc}
        try:
            batch.retune(t)
        except N.TriccError:
            continue
        batch.plan()
        ms = _time(batch.run, reps)
        if log:
            log(f"batch tuning {t}: {ms:.3f} ms")
        if best_ms is None or ms < best_ms:
            best_ms, best = ms, t
    batch.retune(best)
    batch.plan()
    if key:
        store(key, {"tuning": best, "ms": best_ms})
    return best, best_ms


def default_or_cached_batch(key):
    rec = lookup(key)
    return rec["tuning"] if rec else default_batch_tuning().as_dict()

"""The autotuner's searches run end to end on small inputs and the tunings
they pick reproduce the oracle: tune_single over the bin-limit sets and
per-bin variants of a built graph, tune_batch over the persistent kernel's
work splits. Nothing is written to the tuning cache (no key)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1606_07550_amd as P
from paper_1606_07550_amd import _native as N
from paper_1606_07550_amd import autotune
from paper_1606_07550_amd import inputs as I

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


def test_tune_single_picks_a_valid_tuning_that_counts_right():
    n, s, d = I.rmat(15, 16, seed=91)
    ref = oracle.count(n, s, d, order=1)
    g = P.Graph(n, dev(s), dev(d))
    best, ms = autotune.tune_single(g, reps=1)
    assert ms > 0
    mo = g.info["max_outdeg"]
    for b in range(N.NUM_BINS):
        bound = mo if b == N.NUM_BINS - 1 else min(best["bin_limit"][b], mo)
        assert P.variant_capacity(best["bin_variant"][b]) >= bound
        if best["min_side"] and b < N.NUM_BINS - 1:
            assert N.lib().tricc_variant_min_side(best["bin_variant"][b])
    # the graph is left retuned to the pick; a fresh graph built with it agrees
    for gr in (g, P.Graph(n, dev(s), dev(d), tuning=best)):
        o = gr.count()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(o["T"].cpu().numpy().view(np.uint64), ref["T"])
        assert int(o["total"].cpu().numpy().view(np.uint64)[0]) == ref["total"]


def test_tune_batch_picks_a_tuning_that_counts_right():
    bt = I.batch(64, 31, nmin=64, nmax=4000)
    b = P.Batch(bt["node_off"], bt["edge_off"], dev(bt["src"]), dev(bt["dst"]))
    best, ms = autotune.tune_batch(b, reps=1)
    assert ms > 0 and best["persist_variant"] in autotune.MERGE_CAP
    assert best["merge_limit"] <= autotune.MERGE_CAP[best["persist_variant"]]
    b.run()
    torch.cuda.synchronize()
    T = b.out["T"].cpu().numpy().view(np.uint64)
    gtri = b.out["graph_tri"].cpu().numpy().view(np.uint64)
    no, eo = bt["node_off"], bt["edge_off"]
    for gi in range(64):
        ref = oracle.count(int(no[gi + 1] - no[gi]), bt["src"][eo[gi]:eo[gi + 1]], bt["dst"][eo[gi]:eo[gi + 1]])
        np.testing.assert_array_equal(T[no[gi]:no[gi + 1]], ref["T"], err_msg=f"graph {gi}")
        assert int(gtri[gi]) == ref["total"]

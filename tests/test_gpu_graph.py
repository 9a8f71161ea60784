"""The join-aggregate and the group-by captured in one HIP graph and replayed.

Both calls are stream-ordered kernels only (no memset, no host copy), so a
caller may capture them.  The graph holds the partitioned join (16 groups) on
the skew layout, the single-pass join on the identity layout, and the
partitioned group-by with un-permuting; every replay, with eager work and a
synchronisation between replays, must give the oracle's answers again.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1910_10063_amd import skew
from paper_1910_10063_amd import workload as W

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_join_and_group_replayed_from_a_graph():
    N, F = 100_003, (1 << 22) + 5
    say(f"graph: join N={N} F={F}, group-by")
    h = W.host_join_inputs(3, N, F, 1.0)
    C, price, cat = to_dev(h["fact"]), to_dev(h["price"]), to_dev(h["category"])
    L = skew.build_skew_layout(C, N, price, cat)
    ej16 = oracle.fk_join_aggregate(h["fact"], h["price"], h["category"], 16, True)
    ej1 = oracle.fk_join_aggregate(h["fact"], h["price"], h["category"], 7, False)
    M = 50_000
    rng = np.random.default_rng(11)
    gk = (rng.zipf(1.1, F) % M).astype(np.int32)
    gv = rng.integers(-3, 5000, F).astype(np.int32)  # both cold streams
    eg = oracle.group_aggregate(gk, gv, M)
    assert eg[2] == 0
    Lg = skew.build_skew_layout(to_dev(gk), M)
    gvd = to_dev(gv)

    wj = skew.workspace(skew.SKEW_OP_JOIN, F, N, DEV)
    wj1 = skew.workspace(skew.SKEW_OP_JOIN_SINGLE_PASS, F, N, DEV)
    wg = skew.workspace(skew.SKEW_OP_GROUP, F, M, DEV)
    oj16 = (torch.empty(16, dtype=torch.int64, device=DEV), torch.empty(16, dtype=torch.int64, device=DEV))
    oj1 = (torch.empty(1, dtype=torch.int64, device=DEV), torch.empty(1, dtype=torch.int64, device=DEV))
    og = (torch.empty(M, dtype=torch.int64, device=DEV), torch.empty(M, dtype=torch.int64, device=DEV))

    def calls():
        skew.fk_join_aggregate(L.fact_recoded, L.price, L.category, 16, True, hot_rows=skew.SKEW_HOT_AUTO, ws=wj,
                               out=oj16)
        skew.fk_join_aggregate(C, price, cat, 7, False, hot_rows=0, ws=wj1, out=oj1)
        skew.group_aggregate(Lg.fact_recoded, gvd, M, hot_groups=skew.SKEW_HOT_AUTO, perm=Lg.perm, ws=wg, out=og)

    def check(tag):
        assert (host(oj16[0]) == ej16[0]).all() and (host(oj16[1]) == ej16[1]).all(), tag
        assert (host(oj1[0]) == ej1[0]).all() and (host(oj1[1]) == ej1[1]).all(), tag
        assert (host(og[0]) == eg[0]).all() and (host(og[1]) == eg[1]).all(), tag

    calls()  # eager: also sets the kernels' LDS limits
    check("eager")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        calls()
    for replay in range(3):
        for o in (*oj16, *oj1, *og):
            o.fill_(-7)
        torch.cuda.synchronize()
        _ = (C[:1000].to(torch.int64) * 3).sum().item()  # eager work between replays
        g.replay()
        check(f"replay {replay}")
    assert skew.query_status(wg) == skew.SKEW_OK
    del g

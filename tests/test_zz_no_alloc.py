"""fk_join_aggregate_noalloc: the join without a workspace, through the C ABI.

Two calls in a row on one stream, the second with a smaller input (fewer
dimension rows, fewer fact keys, other data), each compared element by
element with fk_join_aggregate (the entry point with a workspace) on the same
inputs and with the oracle.  The call captured in a HIP graph gives the
oracle's answer on every replay.  A dimension larger than the library's fixed
scratch is rejected on the host.
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


def inputs(k, N, F, s):
    h = W.host_join_inputs(k, N, F, s)
    return h, {n: torch.from_numpy(h[n]).to(DEV) for n in ("fact", "price", "category")}


@pytest.mark.parametrize("by_cat,cat_lt", [(True, 16), (False, 4)])
def test_noalloc_matches_workspace_entry_point(by_cat, cat_lt):
    g = 16 if by_cat else 1
    cases = ((1, 200_000, 3_000_007, 1.0), (3, 20_000, 500_003, 0.5))  # the second call is smaller
    for k, N, F, s in cases:
        say(f"noalloc join k={k} N={N} F={F} by_cat={by_cat}")
        h, d = inputs(k, N, F, s)
        L = skew.build_skew_layout(d["fact"], N, d["price"], d["category"])
        es, ec = oracle.fk_join_aggregate(h["fact"], h["price"], h["category"], cat_lt, by_cat)
        for keys, pr, ca, t in ((L.fact_recoded, L.price, L.category, skew.SKEW_HOT_AUTO),
                                (d["fact"], d["price"], d["category"], 0)):
            out = (torch.full((g,), -5, dtype=torch.int64, device=DEV), torch.full((g,), -5, dtype=torch.int64,
                                                                                    device=DEV))
            skew.fk_join_aggregate_noalloc(keys, pr, ca, cat_lt, by_cat, out, hot_rows=t)
            ws_s, ws_c = skew.fk_join_aggregate(keys, pr, ca, cat_lt, by_cat, hot_rows=t)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out[0].cpu().numpy(), ws_s.cpu().numpy(), err_msg=f"sum, t={t}")
            np.testing.assert_array_equal(out[1].cpu().numpy(), ws_c.cpu().numpy(), err_msg=f"count, t={t}")
            np.testing.assert_array_equal(out[0].cpu().numpy(), es, err_msg=f"sum vs oracle, t={t}")
            np.testing.assert_array_equal(out[1].cpu().numpy(), ec, err_msg=f"count vs oracle, t={t}")


def test_noalloc_rejects_a_dimension_larger_than_its_scratch():
    say("noalloc join: dimension above the scratch limit")
    keys = torch.zeros(16, dtype=torch.int32, device=DEV)
    price = torch.empty(skew.SKEW_NOALLOC_MAX_ROWS + 1, dtype=torch.int32, device=DEV)
    cat = torch.empty(skew.SKEW_NOALLOC_MAX_ROWS + 1, dtype=torch.int8, device=DEV)
    out = (torch.empty(16, dtype=torch.int64, device=DEV), torch.empty(16, dtype=torch.int64, device=DEV))
    with pytest.raises(skew.SkewError) as e:
        skew.fk_join_aggregate_noalloc(keys, price, cat, 16, True, out)
    assert e.value.code == skew.SKEW_EINVAL


def test_noalloc_replayed_from_a_hip_graph():
    """The entry point captured in a HIP graph (what a caller that cannot allocate does with it): every replay,
    with eager work and synchronisations between them, equals the oracle."""
    N, F = 100_000, 2_000_003
    say(f"noalloc join in a HIP graph N={N} F={F}")
    h, d = inputs(2, N, F, 1.0)
    L = skew.build_skew_layout(d["fact"], N, d["price"], d["category"])
    es, ec = oracle.fk_join_aggregate(h["fact"], h["price"], h["category"], 16, True)
    out = (torch.empty(16, dtype=torch.int64, device=DEV), torch.empty(16, dtype=torch.int64, device=DEV))
    skew.fk_join_aggregate_noalloc(L.fact_recoded, L.price, L.category, 16, True, out)  # eager first call
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        skew.fk_join_aggregate_noalloc(L.fact_recoded, L.price, L.category, 16, True, out)
    for i in range(3):
        out[0].fill_(-1)
        out[1].fill_(-7)
        junk = torch.randn(1 << 20, device=DEV).sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out[0].cpu().numpy(), es, err_msg=f"sum, replay {i}")
        np.testing.assert_array_equal(out[1].cpu().numpy(), ec, err_msg=f"count, replay {i}")
        assert torch.isfinite(junk)

"""Parity at the full sizes the bench times, in the same launch configuration.

The join workload (1e7-row dimension, 1e9 Zipf(1.0) fact keys, 16 groups) and
the group-by workload (1e6 groups, 5e8 Zipf(1.1) rows, values U[0,1000]) are
generated on the device from the same seeds as the bench; the layout is built,
and the query runs with the library's default hot prefix (SKEW_HOT_AUTO) on
the frequency-ordered layout and with no prefix on the identity layout.  The
oracle computes every output from the host copy of the identity-layout
columns; the GPU results must equal it exactly.  The layouts of the join and
group-by columns are compared with the oracle's element by element: key
counts by rank, permutation, rank, the permuted dimension columns and the
whole recoded column (in chunks); the layouts of the other workloads through
properties that hold at any size.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1910_10063_amd import skew
from paper_1910_10063_amd import workload as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DEV = "cuda"


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def check_layout_properties(L, n_keys, n_fact):
    perm, rank, cbr = host(L.perm), host(L.rank), host(L.counts_by_rank).astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n_keys, dtype=np.int32)), "perm is a permutation"
    assert np.array_equal(rank[perm], np.arange(n_keys, dtype=np.int32)), "rank inverts perm"
    assert cbr.sum() == n_fact, "frequencies sum to the column length"
    assert (np.diff(cbr) <= 0).all(), "frequencies do not increase along perm"
    ties = np.flatnonzero(np.diff(cbr) == 0)
    assert (perm[ties] < perm[ties + 1]).all(), "equal frequencies in ascending key order"


def check_layout_vs_oracle(L, keys_h, n_keys, price_h=None, cat_h=None, chunk=1 << 27):
    cnt, inv = oracle.key_counts(keys_h, n_keys)
    assert inv == 0
    perm, rank = oracle.permutation_index(cnt)
    np.testing.assert_array_equal(host(L.perm), perm, err_msg="perm")
    np.testing.assert_array_equal(host(L.rank), rank, err_msg="rank")
    np.testing.assert_array_equal(host(L.counts_by_rank).astype(np.uint32).astype(np.int64), cnt[perm],
                                  err_msg="counts by rank")
    if price_h is not None:
        np.testing.assert_array_equal(host(L.price), oracle.permute_dim(price_h, perm), err_msg="permuted price")
    if cat_h is not None:
        np.testing.assert_array_equal(host(L.category), oracle.permute_dim(cat_h, perm), err_msg="permuted category")
    for a in range(0, keys_h.size, chunk):
        b = min(a + chunk, keys_h.size)
        np.testing.assert_array_equal(host(L.fact_recoded[a:b]), oracle.recode(keys_h[a:b], rank),
                                      err_msg=f"recoded keys [{a}, {b})")


def test_join_full_size():
    N, F, S = 10_000_000, 1_000_000_000, 1.0
    say(f"join full size N={N} F={F} s={S}")
    d = W.device_join_inputs(2, N, F, S, DEV)
    L = skew.build_skew_layout(d["fact"], N, d["price"], d["category"])
    check_layout_properties(L, N, F)
    fact_h, price_h, cat_h = host(d["fact"]), host(d["price"]), host(d["category"])
    say("join full size: layout vs oracle")
    check_layout_vs_oracle(L, fact_h, N, price_h, cat_h)
    es, ec = oracle.fk_join_aggregate(fact_h, price_h, cat_h, 16, True)
    ws = skew.workspace(skew.SKEW_OP_JOIN, F, N, DEV)
    s, c = skew.fk_join_aggregate(L.fact_recoded, L.price, L.category, 16, True, hot_rows=skew.SKEW_HOT_AUTO, ws=ws)
    assert (host(s) == es).all() and (host(c) == ec).all(), "skew layout"
    s, c = skew.fk_join_aggregate(d["fact"], d["price"], d["category"], 16, True, hot_rows=0, ws=ws)
    assert (host(s) == es).all() and (host(c) == ec).all(), "identity layout"
    assert skew.query_status(ws) == skew.SKEW_OK
    del d, L, ws, fact_h
    torch.cuda.empty_cache()


def test_group_by_full_size():
    M, F, S = 1_000_000, 500_000_000, 1.1
    say(f"group-by full size M={M} F={F} s={S}")
    g = W.device_group_inputs(3, M, F, S, device=DEV)
    L = skew.build_skew_layout(g["keys"], M)
    check_layout_properties(L, M, F)
    keys_h = host(g["keys"])
    say("group-by full size: layout vs oracle")
    check_layout_vs_oracle(L, keys_h, M)
    es, ec, inv = oracle.group_aggregate(keys_h, host(g["vals"]), M)
    assert inv == 0
    ws = skew.workspace(skew.SKEW_OP_GROUP, F, M, DEV)
    s, c = skew.group_aggregate(L.fact_recoded, g["vals"], M, hot_groups=skew.SKEW_HOT_AUTO, perm=L.perm, ws=ws)
    assert (host(s) == es).all() and (host(c) == ec).all(), "skew layout"
    s, c = skew.group_aggregate(g["keys"], g["vals"], M, hot_groups=0, ws=ws)
    assert (host(s) == es).all() and (host(c) == ec).all(), "identity layout"
    assert skew.query_status(ws) == skew.SKEW_OK
    del g, L, ws
    torch.cuda.empty_cache()


def test_group_by_two_rounds():
    """2^29 + 2^20 + 3 rows: a full round of the partitioned group-by and a ragged second one, on both layouts,
    with the bench's values and with values up to 7e4 (cold rows as pairs, hot rows over 2^16 partitioned)."""
    M, F, S = 1_000_000, (1 << 29) + (1 << 20) + 3, 1.1
    say(f"group-by two rounds M={M} F={F} s={S}")
    g = W.device_group_inputs(3, M, F, S, device=DEV)
    L = skew.build_skew_layout(g["keys"], M)
    keys_h = host(g["keys"])
    ws = skew.workspace(skew.SKEW_OP_GROUP, F, M, DEV)
    for scale in (1, 70):
        vals = g["vals"] * scale
        es, ec, inv = oracle.group_aggregate(keys_h, host(vals), M)
        assert inv == 0
        s, c = skew.group_aggregate(L.fact_recoded, vals, M, hot_groups=skew.SKEW_HOT_AUTO, perm=L.perm, ws=ws)
        assert (host(s) == es).all() and (host(c) == ec).all(), f"skew layout, values x{scale}"
        s, c = skew.group_aggregate(g["keys"], vals, M, hot_groups=0, ws=ws)
        assert (host(s) == es).all() and (host(c) == ec).all(), f"identity layout, values x{scale}"
        del vals
    assert skew.query_status(ws) == skew.SKEW_OK
    del g, L, ws
    torch.cuda.empty_cache()


@pytest.mark.parametrize("S", [0.0, 0.5, 1.5])
def test_join_zipf_sweep_one_round(S):
    """The other exponents of the sweep on a 1e7-row dimension, 2^28 + 3 keys (a ragged tail)."""
    N, F = 10_000_000, (1 << 28) + 3
    say(f"join sweep N={N} F={F} s={S}")
    d = W.device_join_inputs(2, N, F, S, DEV)
    L = skew.build_skew_layout(d["fact"], N, d["price"], d["category"])
    check_layout_properties(L, N, F)
    es, ec = oracle.fk_join_aggregate(host(d["fact"]), host(d["price"]), host(d["category"]), 16, True)
    ws = skew.workspace(skew.SKEW_OP_JOIN, F, N, DEV)
    for keys, pr, ca, t in ((L.fact_recoded, L.price, L.category, skew.SKEW_HOT_AUTO),
                            (d["fact"], d["price"], d["category"], 0)):
        s, c = skew.fk_join_aggregate(keys, pr, ca, 16, True, hot_rows=t, ws=ws)
        assert (host(s) == es).all() and (host(c) == ec).all(), t
    del d, L, ws
    torch.cuda.empty_cache()


def test_star_batch_full_size():
    """The bench's batch: 64 queries, fact sizes log-uniform in [1e5, 1e8] rows, product dimension 1e7 rows
    (Zipf 1.0), customer dimension 2e6 rows (Zipf 0.8), with the autotuned tuning, replayed from a HIP graph."""
    k, n_prod, n_cust, nq = 4, 10_000_000, 2_000_000, 64
    sizes, lt, start = W.star_batch_spec(k, nq, 1e5, 1e8)
    say(f"star batch full size rows={int(start[-1])}")
    d = W.device_star_inputs(k, n_prod, n_cust, sizes, device=DEV)
    qs, ql = torch.from_numpy(start).to(DEV), torch.from_numpy(lt).to(DEV)
    Lp = skew.build_skew_layout(d["prod"], n_prod, d["price"], d["category"])
    Lc = skew.build_skew_layout(d["cust"], n_cust, None, d["cust_attr"])
    sk = skew.StarBatch(Lp.fact_recoded, Lc.fact_recoded, qs, ql, Lp.price, Lp.category, Lc.category)
    ws = skew.star_workspace(sk)
    out = (torch.empty(nq, 16, dtype=torch.int64, device=DEV), torch.empty(nq, 16, dtype=torch.int64, device=DEV))
    best, _ = skew.star_join_autotune(sk, ws=ws)
    skew.star_join_batch(sk, best, ws=ws, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        skew.star_join_batch(sk, best, ws=ws, out=out)
    prod, cust = host(d["prod"]), host(d["cust"])
    price, cat, attr = host(d["price"]), host(d["category"]), host(d["cust_attr"])
    want = [oracle.star_join(prod[int(start[q]):int(start[q + 1])], cust[int(start[q]):int(start[q + 1])], price, cat,
                             attr, int(lt[q])) for q in range(nq)]
    for replay in range(2):  # eager work and a synchronisation between the replays
        out[0].fill_(-1)
        out[1].fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        s, c = host(out[0]), host(out[1])
        for q in range(nq):
            assert (s[q] == want[q][0]).all() and (c[q] == want[q][1]).all(), (replay, q)
    del d, Lp, Lc, sk, ws, g
    torch.cuda.empty_cache()

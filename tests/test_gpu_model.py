"""The stack-distance cache model of Section 3.3 on the device against the oracle.

Both evaluate the same model in fp64 (the device with sorted line counts and
prefix sums, the oracle with direct sums); the tolerance covers a search that
lands one trial apart at a rounding boundary, which moves line i's term by at
most 0.54 / K_i^2 <= 0.54 / S^2, and fp64 summation order.  The model itself
is not pinned to the paper (it prints no model output); the oracle is pinned
to closed forms and to an LRU simulation in tests/pins.py.
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module", params=[(3000, 1.0), (50_000, 0.5), (100_000, 1.0)], ids=str)
def layout(request):
    N, s = request.param
    F = 1_000_000
    say(f"cache model layout N={N} F={F} s={s}")
    h = W.host_join_inputs(1, N, F, s)
    L = skew.build_skew_layout(torch.from_numpy(h["fact"]).to(DEV), N)
    cbr = host(L.counts_by_rank).astype(np.int64)
    rank = host(L.rank)
    return dict(N=N, L=L, cbr=cbr, rank=rank)


@pytest.mark.parametrize("S", [1, 37, 512, 3000, 100_000])
@pytest.mark.parametrize("which", ["skew", "identity"])
def test_model_matches_oracle(layout, S, which):
    N, L, cbr, rank = layout["N"], layout["L"], layout["cbr"], layout["rank"]
    v = 1 if N <= 3000 else 32
    say(f"cache model N={N} v={v} S={S} {which}")
    if which == "skew":
        got = skew.cache_model_hit_rate(L.counts_by_rank, S, values_per_line=v)
        f = oracle.line_frequencies(cbr, v)
    else:
        got = skew.cache_model_hit_rate(L.counts_by_rank, S, values_per_line=v, rank=L.rank)
        f = oracle.line_frequencies(cbr[rank], v)
    want = oracle.cache_model(f, S)
    assert abs(got - want) < 1e-6, (got, want)


@pytest.mark.parametrize("L_,S", [(1000, 1), (1000, 100), (1000, 999), (1000, 1000), (70_000, 4096)])
def test_model_uniform_closed_form(L_, S):
    say(f"cache model uniform L={L_} S={S}")
    counts = torch.full((L_,), 7, dtype=torch.int32, device=DEV)
    got = skew.cache_model_hit_rate(counts, S, values_per_line=1)
    want = 1.0 if S >= L_ else 1 - (1 - 1 / L_) ** S
    assert abs(got - want) < 1e-9


def test_model_edges():
    say("cache model edges")
    z = torch.zeros(100, dtype=torch.int32, device=DEV)
    assert skew.cache_model_hit_rate(z, 10, values_per_line=4) == 0.0
    one = torch.zeros(100, dtype=torch.int32, device=DEV)
    one[0] = 5
    assert abs(skew.cache_model_hit_rate(one, 1, values_per_line=1) - 1.0) < 1e-12
    # the frequency-ordered layout never does worse than the identity layout on a skewed column
    rng = np.random.default_rng(4)
    c = np.sort((rng.zipf(1.3, 20_000) % 5000))[::-1]
    cnt = np.bincount(c, minlength=5000).astype(np.int64)
    order = np.lexsort((np.arange(5000), -cnt))
    cbr = torch.from_numpy(cnt[order].astype(np.int32)).to(DEV)
    rank = np.empty(5000, np.int32)
    rank[order] = np.arange(5000, dtype=np.int32)
    sk = skew.cache_model_hit_rate(cbr, 50, values_per_line=16)
    idn = skew.cache_model_hit_rate(cbr, 50, values_per_line=16, rank=torch.from_numpy(rank).to(DEV))
    assert sk >= idn


# ---------------------------------------------------------------------------
# Threshold prior: the choice follows from the frequencies by its stated rule
# (checked on the host from the oracle's layout), its L2 hit rate is the
# model's on the ranks past the threshold, and the query run with the choice
# gives the oracle's answer.
# ---------------------------------------------------------------------------
def _check_choice(ch, cbr, F, cap, row_threshold, per_line):
    t = 0
    while t < min(cap, cbr.size) and cbr[t] >= row_threshold:
        t += 1
    assert ch["hot_rows"] == t, (ch, t)
    assert abs(ch["cold_share"] - (F - cbr[:t].sum()) / F) < 1e-12
    if t < cbr.size:
        want = oracle.cache_model(oracle.line_frequencies(cbr[t:], per_line), 32768)
        assert abs(ch["l2_hit"] - want) < 1e-6, (ch["l2_hit"], want)
    assert ch["partitioned"] == (1 if ch["bytes_partitioned"] < ch["bytes_single"] else 0)


@pytest.mark.parametrize("s", [0.0, 1.0, 1.5])
def test_join_choice(s):
    N, F = 1_000_000, 20_000_003
    say(f"join threshold prior N={N} F={F} s={s}")
    h = W.host_join_inputs(2, N, F, s)
    ref = oracle.build_layout(h["fact"], N, h["price"], h["category"])
    d = {n: torch.from_numpy(h[n]).to(DEV) for n in ("fact", "price", "category")}
    L = skew.build_skew_layout(d["fact"], N, d["price"], d["category"])
    ch = skew.join_choose(L.counts_by_rank, F, True)
    # one round of 256 workgroups: a row is kept when its count reaches 4 * 256 / 13 bytes
    _check_choice(ch, ref.counts_by_rank.astype(np.int64), F, skew.max_hot_rows(True), 4.0 * 256 / 13.0, 32)
    if s == 0.0:
        assert ch["hot_rows"] == 0  # about 20 keys per row: no row pays for its copies
    ws = skew.workspace(skew.SKEW_OP_JOIN if ch["partitioned"] else skew.SKEW_OP_JOIN_SINGLE_PASS, F, N, DEV)
    es, ec = oracle.fk_join_aggregate(h["fact"], h["price"], h["category"], 16, True)
    gs, gc = skew.fk_join_aggregate(L.fact_recoded, L.price, L.category, 16, True, hot_rows=ch["hot_rows"], ws=ws)
    assert (host(gs) == es).all() and (host(gc) == ec).all()


def test_group_choice():
    M, F = 100_000, 10_000_001
    say(f"group threshold prior M={M} F={F}")
    h = W.host_group_inputs(3, M, F, 1.1)
    ref = oracle.build_layout(h["keys"], M)
    L = skew.build_skew_layout(torch.from_numpy(h["keys"]).to(DEV), M)
    ch = skew.group_choose(L.counts_by_rank, F)
    # one round of 256 workgroups: a group is kept when its count reaches 32 * 256 / 16
    _check_choice(ch, ref.counts_by_rank.astype(np.int64), F, skew.max_hot_groups(), 32 * 256 / 16.0, 16)
    ws = skew.workspace(skew.SKEW_OP_GROUP if ch["partitioned"] else skew.SKEW_OP_GROUP_SINGLE_PASS, F, M, DEV)
    es, ec, _ = oracle.group_aggregate(h["keys"], h["vals"], M)
    gs, gc = skew.group_aggregate(L.fact_recoded, torch.from_numpy(h["vals"]).to(DEV), M,
                                  hot_groups=ch["hot_rows"] if ch["hot_rows"] > 0 else skew.SKEW_HOT_NONE,
                                  perm=L.perm, ws=ws)
    assert (host(gs) == es).all() and (host(gc) == ec).all()

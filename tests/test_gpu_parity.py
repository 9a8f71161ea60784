"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

Every integer output must equal the oracle's byte for byte: the layout arrays
(perm, rank, frequencies, recoded facts, permuted dimension) and the int64
sums and counts, for every hot-prefix size and both layouts.
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


def check_layout(L, ref, exact_recode=True):
    assert (host(L.perm) == ref.perm).all(), "perm"
    assert (host(L.rank) == ref.rank).all(), "rank"
    assert (host(L.counts_by_rank).astype(np.int64) == ref.counts_by_rank).all(), "counts_by_rank"
    if L.fact_recoded is not None and exact_recode:
        assert (host(L.fact_recoded) == ref.fact_recoded).all(), "fact_recoded"
    if L.price is not None:
        assert (host(L.price) == ref.price).all(), "permuted price"
    if L.category is not None:
        assert (host(L.category) == ref.category).all(), "permuted category"


# ---------------------------------------------------------------------------
# Small plain-method workload: N = 1e5 rows, F = 1e6 facts, Zipf s = 1.0,
# SUM(price), COUNT WHERE category < 4.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small():
    k, N, F, s = 1, 100_000, 1_000_000, 1.0
    say(f"small workload N={N} F={F} s={s}")
    h = W.host_join_inputs(k, N, F, s)
    ref = oracle.build_layout(h["fact"], N, h["price"], h["category"])
    d = {n: to_dev(h[n]) for n in ("fact", "price", "category")}
    return dict(N=N, F=F, h=h, ref=ref, d=d)


def test_small_layout_matches_oracle(small):
    say("build_skew_layout small")
    d, N = small["d"], small["N"]
    L = skew.build_skew_layout(d["fact"], N, d["price"], d["category"])
    check_layout(L, small["ref"])
    small["L"] = L


def test_small_layout_in_place(small):
    say("build_skew_layout small in place")
    d, N = small["d"], small["N"]
    f = d["fact"].clone()
    L = skew.build_skew_layout(f, N, d["price"], d["category"], in_place=True)
    assert L.fact_recoded.data_ptr() == f.data_ptr()
    check_layout(L, small["ref"])


@pytest.mark.parametrize("t", [0, 1, 63, 64, 65, 4096, 8192, 16384, 32768, 99_999, 100_000, 100_005,
                               skew.SKEW_HOT_AUTO])
@pytest.mark.parametrize("by_cat,cat_lt", [(False, 4), (True, 16), (True, 4), (False, 127), (False, -128)])
def test_small_join_every_t(small, t, by_cat, cat_lt):
    say(f"fk_join_aggregate small t={t} by_cat={by_cat} cat_lt={cat_lt}")
    h, d, ref, N = small["h"], small["d"], small["ref"], small["N"]
    es, ec = oracle.fk_join_aggregate(h["fact"], h["price"], h["category"], cat_lt, by_cat)
    if "Ld" not in small:
        small["Ld"] = {n: to_dev(getattr(ref, n)) for n in ("fact_recoded", "price", "category")}
    Ld = small["Ld"]
    # skew layout (recoded keys, permuted dimension) and identity layout (original columns)
    for keys, price, cat in ((Ld["fact_recoded"], Ld["price"], Ld["category"]),
                             (d["fact"], d["price"], d["category"])):
        s, c = skew.fk_join_aggregate(keys, price, cat, cat_lt, by_cat, hot_rows=t)
        assert (host(s) == es).all() and (host(c) == ec).all(), (t, by_cat, cat_lt)


# ---------------------------------------------------------------------------
# Join-aggregate at reduced scale of the 16-group query: several tiles per
# workgroup, ragged tails, each Zipf exponent of the sweep.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("s", [0.0, 0.5, 1.0, 1.5])
def test_join_by_category_reduced(s):
    k, N, F = 2, 1_000_000, 20_000_003
    say(f"join reduced N={N} F={F} s={s}")
    h = W.host_join_inputs(k, N, F, s)
    ref = oracle.build_layout(h["fact"], N, h["price"], h["category"])
    es, ec = oracle.fk_join_aggregate(h["fact"], h["price"], h["category"], 16, True)
    d = {n: to_dev(h[n]) for n in ("fact", "price", "category")}
    L = skew.build_skew_layout(d["fact"], N, d["price"], d["category"])
    check_layout(L, ref)
    for op in (skew.SKEW_OP_JOIN, skew.SKEW_OP_JOIN_SINGLE_PASS):  # partitioned and single-pass forms
        ws = skew.workspace(op, F, N, DEV)
        # past the LDS capacity the partitioned form gathers the warm rows [capacity, t) in pass 1
        for t in (0, 4096, 32768, skew.SKEW_HOT_AUTO, 65_536, 262_144, 999_999, 1_000_000):
            s_, c_ = skew.fk_join_aggregate(L.fact_recoded, L.price, L.category, 16, True, hot_rows=t, ws=ws)
            assert (host(s_) == es).all() and (host(c_) == ec).all(), ("skew", op, t)
        s_, c_ = skew.fk_join_aggregate(d["fact"], d["price"], d["category"], 16, True, hot_rows=0, ws=ws)
        assert (host(s_) == es).all() and (host(c_) == ec).all(), ("identity", op)
        s1, c1 = oracle.fk_join_aggregate(h["fact"], h["price"], h["category"], 4, False)
        s_, c_ = skew.fk_join_aggregate(L.fact_recoded, L.price, L.category, 4, False, hot_rows=1000, ws=ws)
        assert (host(s_) == s1).all() and (host(c_) == c1).all(), ("one group", op)


# ---------------------------------------------------------------------------
# Grouped aggregation at reduced scale: 1e5 groups, Zipf s = 1.1.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def groups():
    k, M, F, s = 3, 100_000, 10_000_001, 1.1
    say(f"group workload M={M} F={F} s={s}")
    h = W.host_group_inputs(k, M, F, s)
    ref = oracle.build_layout(h["keys"], M)
    es, ec, inv = oracle.group_aggregate(h["keys"], h["vals"], M)
    assert inv == 0
    return dict(M=M, F=F, h=h, ref=ref, es=es, ec=ec)


def test_group_layout_matches_oracle(groups):
    say("group layout")
    d = to_dev(groups["h"]["keys"])
    L = skew.build_skew_layout(d, groups["M"])
    check_layout(L, groups["ref"])


GROUP_OPS = [skew.SKEW_OP_GROUP, skew.SKEW_OP_GROUP_SINGLE_PASS]


@pytest.mark.parametrize("op", GROUP_OPS, ids=["partitioned", "single_pass"])
@pytest.mark.parametrize("t", [1, 15, 16, 17, 64, 1024, 8192, 100_000, skew.SKEW_HOT_AUTO])
def test_group_skew_every_t(groups, t, op):
    say(f"group_aggregate skew t={t} op={op}")
    ref, M, F = groups["ref"], groups["M"], groups["F"]
    keys = to_dev(ref.fact_recoded)
    vals = to_dev(groups["h"]["vals"])
    perm = to_dev(ref.perm)
    ws = skew.workspace(op, F, M, DEV)
    s, c = skew.group_aggregate(keys, vals, M, hot_groups=t, perm=perm, ws=ws)
    assert (host(s) == groups["es"]).all() and (host(c) == groups["ec"]).all()


@pytest.mark.parametrize("op", GROUP_OPS, ids=["partitioned", "single_pass"])
@pytest.mark.parametrize("mode", [0, skew.SKEW_HOT_NONE, 4096])
def test_group_identity_modes(groups, mode, op):
    say(f"group_aggregate identity mode={mode} op={op}")
    keys = to_dev(groups["h"]["keys"])
    vals = to_dev(groups["h"]["vals"])
    ws = skew.workspace(op, groups["F"], groups["M"], DEV)
    s, c = skew.group_aggregate(keys, vals, groups["M"], hot_groups=mode, ws=ws)
    assert (host(s) == groups["es"]).all() and (host(c) == groups["ec"]).all()


@pytest.mark.parametrize("offset", [0, 1, 3])
def test_partitioned_edges(offset):
    """Partitioned forms on ragged/unaligned columns with escapes, negatives and bad keys."""
    say(f"partitioned edges offset={offset}")
    rng = np.random.default_rng(40 + offset)
    N, F = 300_001, (1 << 22) + 12_345
    price = rng.integers(1, 10001, N).astype(np.int32)
    price[rng.integers(0, N, 50)] = rng.integers(-2**31, -1, 50)  # escapes, hot and cold
    price[:3] = [-7, 2**30, 5]
    cat = rng.integers(0, 16, N).astype(np.int8)
    cat[rng.integers(0, N, 1000)] = -3
    fact = (rng.zipf(1.2, F + offset) % N).astype(np.int32)
    fd = to_dev(fact)[offset:]
    for by_cat, cat_lt in ((True, 16), (False, 4)):
        es, ec = oracle.fk_join_aggregate(fact[offset:], price, cat, cat_lt, by_cat)
        ws = skew.workspace(skew.SKEW_OP_JOIN, F, N, DEV)
        for t in (0, 7, 32768):
            s, c = skew.fk_join_aggregate(fd, to_dev(price), to_dev(cat), cat_lt, by_cat, hot_rows=t, ws=ws)
            assert (host(s) == es).all() and (host(c) == ec).all(), (by_cat, t)
    # out-of-range keys in the partitioned join: skipped and flagged
    bad = fact.copy()
    bad[offset + 100] = N + 5
    bad[offset + F // 2] = -1
    ws = skew.workspace(skew.SKEW_OP_JOIN, F, N, DEV)
    s, c = skew.fk_join_aggregate(to_dev(bad)[offset:], to_dev(price), to_dev(cat), 16, True, hot_rows=100, ws=ws)
    es, ec = oracle.fk_join_aggregate(bad[offset:], price, cat, 16, True)
    assert (host(s) == es).all() and (host(c) == ec).all()
    with pytest.raises(skew.SkewError):
        skew.query_status(ws)
    # group-by: negative values, bad keys, keys and values misaligned to each other
    M = 50_000
    gk = (rng.zipf(1.1, F + 8) % (M + 3)).astype(np.int32)  # a few keys >= M
    gv = rng.integers(-2**31, 2**31, F + 8, dtype=np.int64).astype(np.int32)
    for voff in (offset, (offset + 2) % 4):
        keys = to_dev(gk)[offset:offset + F]
        vals = to_dev(gv)[voff:voff + F]
        es, ec, inv = oracle.group_aggregate(gk[offset:offset + F], gv[voff:voff + F], M)
        assert inv > 0
        gws = skew.workspace(skew.SKEW_OP_GROUP, F, M, DEV)
        for t in (0, 5, 16, 3000):
            s, c = skew.group_aggregate(keys, vals, M, hot_groups=t, ws=gws)
            assert (host(s) == es).all() and (host(c) == ec).all(), (voff, t)
        with pytest.raises(skew.SkewError):
            skew.query_status(gws)


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------
def test_empty_fact_column():
    say("edge: F = 0")
    price = to_dev(np.array([5, 6, 7], np.int32))
    cat = to_dev(np.array([1, 2, 3], np.int8))
    f = torch.empty(0, dtype=torch.int32, device=DEV)
    L = skew.build_skew_layout(f, 3, price, cat)
    assert host(L.perm).tolist() == [0, 1, 2] and host(L.counts_by_rank).tolist() == [0, 0, 0]
    s, c = skew.fk_join_aggregate(f, price, cat, 16, True, hot_rows=2)
    assert not host(s).any() and not host(c).any()
    s, c = skew.group_aggregate(f, f, 3, hot_groups=2)
    assert not host(s).any() and not host(c).any()


def test_single_dimension_row():
    say("edge: N = 1")
    F = 12345
    f = torch.zeros(F, dtype=torch.int32, device=DEV)
    price = to_dev(np.array([77], np.int32))
    cat = to_dev(np.array([3], np.int8))
    L = skew.build_skew_layout(f, 1, price, cat)
    assert host(L.perm).tolist() == [0] and host(L.counts_by_rank).tolist() == [F]
    for t in (0, 1, skew.SKEW_HOT_AUTO):
        s, c = skew.fk_join_aggregate(f, price, cat, 4, False, hot_rows=t)
        assert host(s).tolist() == [77 * F] and host(c).tolist() == [F]


@pytest.mark.parametrize("offset", [0, 1, 2, 3])
@pytest.mark.parametrize("F", [1, 2, 3, 5, 4097, 65537])
def test_ragged_and_unaligned(offset, F):
    say(f"edge: unaligned offset={offset} F={F}")
    rng = np.random.default_rng(F * 10 + offset)
    N = 1000
    price = rng.integers(1, 10001, N).astype(np.int32)
    cat = rng.integers(0, 16, N).astype(np.int8)
    fact = rng.integers(0, N, F + offset).astype(np.int32)
    vals = rng.integers(-1000, 1000, F + offset).astype(np.int32)
    fd = to_dev(fact)[offset:]
    vd = to_dev(vals)[offset:]
    es, ec = oracle.fk_join_aggregate(fact[offset:], price, cat, 16, True)
    for t in (0, 100, N):
        s, c = skew.fk_join_aggregate(fd, to_dev(price), to_dev(cat), 16, True, hot_rows=t)
        assert (host(s) == es).all() and (host(c) == ec).all()
    gs, gc, _ = oracle.group_aggregate(fact[offset:], vals[offset:], N)
    for t in (0, 100, skew.SKEW_HOT_NONE):
        s, c = skew.group_aggregate(fd, vd, N, hot_groups=t)
        assert (host(s) == gs).all() and (host(c) == gc).all()
    # keys and values misaligned relative to each other take the scalar path
    voff = (offset + 1) % 4
    vals2 = rng.integers(-1000, 1000, F + 4).astype(np.int32)
    vd2 = to_dev(vals2)[voff:voff + F]
    gs2, gc2, _ = oracle.group_aggregate(fact[offset:], vals2[voff:voff + F], N)
    s, c = skew.group_aggregate(fd, vd2, N, hot_groups=100)
    assert (host(s) == gs2).all() and (host(c) == gc2).all()
    ref = oracle.build_layout(fact[offset:], N, price, cat)
    L = skew.build_skew_layout(fd, N, to_dev(price), to_dev(cat))
    check_layout(L, ref)


def test_wide_prices_and_odd_categories():
    """Prices outside [0, 2^26) take the escape path; categories outside [0, 16) join no group."""
    say("edge: wide prices, negative categories")
    rng = np.random.default_rng(5)
    N, F = 5000, 300_000
    price = rng.integers(-2**31, 2**31, N, dtype=np.int64).astype(np.int32)
    price[:100] = rng.integers(0, 2**26, 100)
    cat = rng.integers(-128, 128, N).astype(np.int8)
    cat[:2500] = rng.integers(0, 16, 2500)
    fact = (rng.zipf(1.3, F) % N).astype(np.int32)
    for by_cat, cat_lt in ((True, 16), (True, 4), (False, 4), (False, 127), (True, -5)):
        es, ec = oracle.fk_join_aggregate(fact, price, cat, cat_lt, by_cat)
        for t in (0, 64, N):
            s, c = skew.fk_join_aggregate(to_dev(fact), to_dev(price), to_dev(cat), cat_lt, by_cat, hot_rows=t)
            assert (host(s) == es).all() and (host(c) == ec).all(), (by_cat, cat_lt, t)


def test_out_of_range_keys():
    say("edge: out-of-range keys")
    N = 100
    fact = np.arange(1000, dtype=np.int32) % N
    fact[17] = N
    fact[500] = -3
    price = np.full(N, 2, np.int32)
    cat = np.zeros(N, np.int8)
    fd = to_dev(fact)
    keep = fd.clone()
    with pytest.raises(skew.SkewError) as e:
        skew.build_skew_layout(fd, N, to_dev(price), to_dev(cat), in_place=True)
    assert e.value.code == skew.SKEW_ERANGE
    assert torch.equal(fd, keep), "a failed build must not touch the fact column"
    ws = skew.workspace(skew.SKEW_OP_JOIN, fact.size, N, DEV)
    s, c = skew.fk_join_aggregate(fd, to_dev(price), to_dev(cat), 16, False, hot_rows=10, ws=ws)
    es, ec = oracle.fk_join_aggregate(fact, price, cat, 16, False)
    assert (host(s) == es).all() and (host(c) == ec).all()
    with pytest.raises(skew.SkewError) as e:
        skew.query_status(ws)
    assert e.value.code == skew.SKEW_ERANGE
    ok = to_dev(np.arange(1000, dtype=np.int32) % N)
    skew.fk_join_aggregate(ok, to_dev(price), to_dev(cat), 16, False, hot_rows=10, ws=ws)
    assert skew.query_status(ws) == skew.SKEW_OK
    gws = skew.workspace(skew.SKEW_OP_GROUP, fact.size, N, DEV)
    s, c = skew.group_aggregate(fd, fd, N, hot_groups=10, ws=gws)
    gs, gc, inv = oracle.group_aggregate(fact, fact, N)
    assert inv == 2 and (host(s) == gs).all() and (host(c) == gc).all()
    with pytest.raises(skew.SkewError):
        skew.query_status(gws)


def test_negative_values_and_large_counts():
    say("edge: negative int32 values, one very hot group")
    F = 3_000_000
    keys = np.zeros(F, np.int32)
    keys[::7] = 5
    vals = np.full(F, -2**31, np.int32)
    vals[1::3] = 2**31 - 1
    es, ec, _ = oracle.group_aggregate(keys, vals, 10)
    for t in (0, 1, 6, 10, skew.SKEW_HOT_NONE):
        s, c = skew.group_aggregate(to_dev(keys), to_dev(vals), 10, hot_groups=t)
        assert (host(s) == es).all() and (host(c) == ec).all(), t


@pytest.mark.parametrize("offset", [0, 2])
def test_partitioned_group_value_boundaries(offset):
    """Pass 1 of the partitioned group-by packs count and sum of a hot group into one word for values in
    [0, 2^16); values at and around that boundary, on hot and cold groups, with one very hot group."""
    say(f"group value boundaries offset={offset}")
    rng = np.random.default_rng(70 + offset)
    M, F = 40_000, (1 << 22) + 77
    keys = (rng.zipf(1.1, F + offset) % M).astype(np.int32)
    keys[rng.random(F + offset) < 0.3] = 0  # one group takes a third of the rows
    edge = np.array([0, 1, 65534, 65535, 65536, 65537, -1, -65536, 2**31 - 1, -2**31], np.int64)
    vals = edge[rng.integers(0, edge.size, F + offset)].astype(np.int32)
    vals[rng.random(F + offset) < 0.5] = 65535
    es, ec, inv = oracle.group_aggregate(keys[offset:], vals[offset:], M)
    assert inv == 0
    kd, vd = to_dev(keys)[offset:], to_dev(vals)[offset:]
    ws = skew.workspace(skew.SKEW_OP_GROUP, F, M, DEV)
    for t in (1, 16, 17, 3000, M, skew.SKEW_HOT_AUTO):
        s, c = skew.group_aggregate(kd, vd, M, hot_groups=t, ws=ws)
        assert (host(s) == es).all() and (host(c) == ec).all(), t
    assert skew.query_status(ws) == skew.SKEW_OK


@pytest.mark.parametrize("M", [40_000, 1 << 20, (1 << 20) + 1])
@pytest.mark.parametrize("mix", ["edges", "narrow_only", "wide_only"])
def test_partitioned_group_narrow_records(M, mix):
    """Cold rows of the partitioned group-by travel as one word (group << 12 | value) when there are at most 2^20
    groups and the value lies in [0, 2^12), else as a (group, value) pair; values at and around both limits, with
    either stream empty, and group counts on both sides of 2^20."""
    say(f"group narrow records M={M} mix={mix}")
    rng = np.random.default_rng(M % 1000 + len(mix))
    F = (1 << 22) + 77
    keys = (rng.zipf(1.05, F) % M).astype(np.int32)
    keys[rng.random(F) < 0.01] = M - 1  # the last group, in the last slice
    if mix == "edges":
        edge = np.array([0, 1, 4094, 4095, 4096, 4097, 65535, 65536, -1, 2**31 - 1, -2**31], np.int64)
        vals = edge[rng.integers(0, edge.size, F)].astype(np.int32)
        narrow = rng.random(F) < 0.5
        vals[narrow] = rng.integers(0, 4096, int(narrow.sum()))
    elif mix == "narrow_only":
        vals = rng.integers(0, 4096, F).astype(np.int32)
    else:
        vals = rng.integers(4096, 1 << 20, F).astype(np.int32)
    es, ec, inv = oracle.group_aggregate(keys, vals, M)
    assert inv == 0
    kd, vd = to_dev(keys), to_dev(vals)
    ws = skew.workspace(skew.SKEW_OP_GROUP, F, M, DEV)
    for t in (0, 16, skew.SKEW_HOT_AUTO):
        s, c = skew.group_aggregate(kd, vd, M, hot_groups=t, ws=ws)
        assert (host(s) == es).all() and (host(c) == ec).all(), t
    assert skew.query_status(ws) == skew.SKEW_OK


def test_generator_device_matches_host():
    say("generator: device vs host")
    for n_ranks, s in ((100_000, 1.0), (1_000_000, 1.1), (1000, 0.0)):
        cdf = W.zipf_cdf(n_ranks, s)
        pi = W.permutation(W.perm_seed(9), n_ranks)
        out = W.device_fact_keys(77, to_dev(cdf), to_dev(pi), 300_001)
        assert (host(out) == W.fact_keys(77, cdf, pi, 300_001)).all()
        part = W.device_fact_keys(77, to_dev(cdf), to_dev(pi), 1000, start=123_456)
        assert (host(part) == W.fact_keys(77, cdf, pi, 1000, start=123_456)).all()
    v = W.device_uniform_i32(5, 0, 1000, 100_003, DEV)
    assert (host(v) == W.uniform_int(5, 0, 1000, 100_003)).all()


def test_partitioned_join_with_gathered_tail():
    """A dimension larger than the slices can cover (1024 slices of 32768 rows past the hot prefix): keys past the
    last slice are gathered in pass 1, the rest partitioned; escapes and odd categories in both parts.  Thresholds
    past the LDS capacity add a warm range gathered in pass 1 before the slices."""
    say("partitioned join with a gathered tail")
    rng = np.random.default_rng(77)
    N, F = 40_000_000, (1 << 22) + 12_345
    h = W.host_join_inputs(14, N, F, 0.7)
    price, cat = h["price"].copy(), h["category"].copy()
    tail_rows = rng.integers(34_000_000, N, 2000)
    price[tail_rows[:1000]] = rng.integers(1 << 25, 2**31 - 1, 1000)  # escapes in the tail
    cat[tail_rows[1000:]] = -5
    price[rng.integers(0, 1_000_000, 500)] = -3                          # escapes in the slices
    fact = h["fact"]
    assert (fact >= 34_000_000).sum() > 10_000, "the column must reach the tail"
    ws = skew.workspace(skew.SKEW_OP_JOIN, F, N, DEV)
    fd, pd, cd = to_dev(fact), to_dev(price), to_dev(cat)
    for by_cat, cat_lt in ((True, 16), (False, 9)):
        es, ec = oracle.fk_join_aggregate(fact, price, cat, cat_lt, by_cat)
        for t in (0, 7, skew.SKEW_HOT_AUTO, 300_000, 6_000_000):
            s, c = skew.fk_join_aggregate(fd, pd, cd, cat_lt, by_cat, hot_rows=t, ws=ws)
            assert (host(s) == es).all() and (host(c) == ec).all(), (by_cat, t)
    assert skew.query_status(ws) == skew.SKEW_OK


@pytest.mark.parametrize("F", [70_001, (1 << 22) + 3])
@pytest.mark.parametrize("poff,coff", [(0, 0), (1, 0), (0, 3), (3, 1)])
def test_join_dimension_columns_at_any_alignment(F, poff, coff):
    """The dimension is packed four rows at a time when the price column is 16-byte aligned and the categories
    4-byte aligned, one row at a time otherwise; a ragged dimension (N % 4 = 1) and both forms of the query."""
    say(f"join dimension alignment F={F} poff={poff} coff={coff}")
    N = 50_001
    h = W.host_join_inputs(12, N, F, 1.0)
    price = torch.zeros(N + 4, dtype=torch.int32, device=DEV)
    cat = torch.zeros(N + 4, dtype=torch.int8, device=DEV)
    price[poff:poff + N] = to_dev(h["price"])
    cat[coff:coff + N] = to_dev(h["category"])
    pv, cv = price[poff:poff + N], cat[coff:coff + N]
    keys = to_dev(h["fact"])
    for cat_lt, by_cat in ((16, True), (4, False)):
        es, ec = oracle.fk_join_aggregate(h["fact"], h["price"], h["category"], cat_lt, by_cat)
        for t in (0, 1000, skew.SKEW_HOT_AUTO):
            s, c = skew.fk_join_aggregate(keys, pv, cv, cat_lt, by_cat, hot_rows=t)
            assert (host(s) == es).all() and (host(c) == ec).all(), (cat_lt, t)


# ---------------------------------------------------------------------------
# The partitioned join under key orders far from a shuffled Zipf column:
# keys sorted (each workgroup's cold keys fall into a few slices), every key
# in one slice, and runs of hot keys between runs of keys spread over all
# slices.  With prefixes below 2048 rows the slice-0 counts of pass 1 and the
# scatter's slice-0 ranks are combined per slot where slice 0 is dense, which
# these orders switch on for some workgroups and off for others.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", ["sorted", "one_slice", "runs"])
def test_join_adversarial_key_orders(shape):
    rng = np.random.default_rng({"sorted": 61, "one_slice": 62, "runs": 63}[shape])
    N, F = 1_000_000, (1 << 22) + 777
    say(f"join key order {shape} N={N} F={F}")
    price = rng.integers(1, 10001, N).astype(np.int32)
    cat = rng.integers(0, 16, N).astype(np.int8)
    if shape == "sorted":
        fact = np.sort(rng.integers(0, N, F)).astype(np.int32)
    elif shape == "one_slice":
        fact = rng.integers(200_000, 200_000 + 32768, F).astype(np.int32)
    else:
        fact = rng.integers(0, N, F).astype(np.int32)
        run = np.arange(F) // 50_000 % 2 == 0
        fact[run] = rng.integers(0, 1000, int(run.sum()))
    ws = skew.workspace(skew.SKEW_OP_JOIN, F, N, DEV)
    fd, pd, cd = to_dev(fact), to_dev(price), to_dev(cat)
    for by_cat, cat_lt in ((True, 16), (False, 4)):
        es, ec = oracle.fk_join_aggregate(fact, price, cat, cat_lt, by_cat)
        for t in (0, 1000, skew.SKEW_HOT_AUTO):
            s, c = skew.fk_join_aggregate(fd, pd, cd, cat_lt, by_cat, hot_rows=t, ws=ws)
            assert (host(s) == es).all() and (host(c) == ec).all(), (by_cat, t)
    assert skew.query_status(ws) == skew.SKEW_OK

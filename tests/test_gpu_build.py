"""GPU parity of the index build at sizes that take the partitioned key histogram.

Fact columns of at least 2^22 keys are counted by partitioning the keys into
slices of 32768 key ids and counting each slice in LDS; the layout (perm,
rank, frequencies, recoded facts, permuted dimension) must equal the oracle's
byte for byte: several rounds of 2^28 keys, key domains that are not a
multiple of the slice, unaligned columns, out-of-range keys, and a domain too
large for the slice table (the hash-privatised count).
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


def check(L, ref):
    assert (host(L.perm) == ref.perm).all(), "perm"
    assert (host(L.rank) == ref.rank).all(), "rank"
    assert (host(L.counts_by_rank).astype(np.int64) == ref.counts_by_rank).all(), "counts_by_rank"
    if L.fact_recoded is not None:
        assert (host(L.fact_recoded) == ref.fact_recoded).all(), "fact_recoded"
    if L.price is not None:
        assert (host(L.price) == ref.price).all(), "price"


@pytest.mark.parametrize("N,s", [(1_000_003, 1.0), (32768, 0.5), (65537, 1.5), (5_000_000, 0.0), (1, 0.0)])
def test_partitioned_build(N, s):
    F = (1 << 22) + 12_345
    say(f"build N={N} F={F} s={s}")
    h = W.host_join_inputs(5, N, F, s)
    ref = oracle.build_layout(h["fact"], N, h["price"], h["category"])
    L = skew.build_skew_layout(to_dev(h["fact"]), N, to_dev(h["price"]), to_dev(h["category"]))
    check(L, ref)


@pytest.mark.parametrize("offset", [1, 2, 3])
def test_partitioned_build_unaligned(offset):
    N, F = 200_000, (1 << 22) + 3
    say(f"build unaligned offset={offset}")
    h = W.host_join_inputs(6, N, F + offset, 1.0)
    fact = h["fact"][offset:]
    ref = oracle.build_layout(fact, N, h["price"], h["category"])
    buf = to_dev(h["fact"])
    L = skew.build_skew_layout(buf[offset:], N, to_dev(h["price"]), to_dev(h["category"]))
    check(L, ref)


def test_partitioned_build_out_of_range():
    N, F = 100_000, 1 << 22
    say("build partitioned out-of-range keys")
    rng = np.random.default_rng(9)
    fact = rng.integers(0, N, F).astype(np.int32)
    for bad in (N, -1, 2**31 - 1):
        f = fact.copy()
        f[F // 2] = bad
        with pytest.raises(skew.SkewError) as e:
            skew.build_skew_layout(to_dev(f), N)
        assert e.value.code == skew.SKEW_ERANGE


def test_large_domain_uses_hash_count():
    """More than 1024 slices of 32768 keys: the hash-privatised count takes over."""
    N, F = 40_000_000, (1 << 22) + 1
    say(f"build large domain N={N} F={F}")
    rng = np.random.default_rng(10)
    fact = rng.integers(0, N, F).astype(np.int32)
    ref = oracle.build_layout(fact, N)
    L = skew.build_skew_layout(to_dev(fact), N)
    check(L, ref)


@pytest.mark.slow
def test_partitioned_build_three_rounds():
    """2^29 + 7 Zipf(1.0) keys over 1e7 rows: three rounds of the partitioned count."""
    N, F = 10_000_000, (1 << 29) + 7
    say(f"build three rounds N={N} F={F}")
    d = W.device_join_inputs(7, N, F, 1.0, DEV)
    L = skew.build_skew_layout(d["fact"], N, d["price"], d["category"])
    fact = host(d["fact"])
    ref = oracle.build_layout(fact, N, host(d["price"]), host(d["category"]))
    check(L, ref)
    del d, L
    torch.cuda.empty_cache()


@pytest.mark.parametrize("N,s,offset", [(1_000_000, 1.0, 0), (10_000_000, 1.0, 1), (3_000_000, 0.0, 0),
                                        (5_000, 1.5, 3), (40_000_000, 1.0, 2)])
def test_build_with_hot_table(N, s, offset):
    """Columns of at least 2^26 keys count a sample first, then the rest with an LDS table of the keys most frequent
    in the sample; the counts (and the layout) must not depend on the table: skewed keys (table used), uniform keys
    (table skipped), a domain smaller than the table, and a domain too large for the slice table."""
    F = (1 << 26) + 12_345
    say(f"build with hot table N={N} s={s} offset={offset}")
    h = W.host_join_inputs(11, N, F + offset, s)
    fact = h["fact"][offset:]
    ref = oracle.build_layout(fact, N, h["price"], h["category"])
    buf = to_dev(h["fact"])
    L = skew.build_skew_layout(buf[offset:], N, to_dev(h["price"]), to_dev(h["category"]))
    check(L, ref)


def test_build_with_hot_table_out_of_range():
    """An out-of-range key after the sample, where the table is in use, is still reported."""
    N, F = 100_000, (1 << 26) + 5
    say("build with hot table, out-of-range keys")
    h = W.host_join_inputs(12, N, F, 1.0)
    for pos, bad in ((F - 3, N), ((1 << 25), -7)):
        f = h["fact"].copy()
        f[pos] = bad
        with pytest.raises(skew.SkewError) as e:
            skew.build_skew_layout(to_dev(f), N)
        assert e.value.code == skew.SKEW_ERANGE


@pytest.mark.parametrize("N,s,in_place,offset", [(100, 1.0, False, 0), (2_000_000, 1.0, True, 0),
                                                 (10_000_000, 0.0, False, 1), (50_000, 1.5, True, 3)])
def test_recode_hot_keys(N, s, in_place, offset):
    """Columns of at least 2^24 keys recode through an LDS table of the hottest keys."""
    F = (1 << 24) + 4099
    say(f"recode hot keys N={N} s={s} in_place={in_place} offset={offset}")
    h = W.host_join_inputs(8, N, F + offset, s)
    fact = h["fact"][offset:]
    ref = oracle.build_layout(fact, N)
    buf = to_dev(h["fact"])
    L = skew.build_skew_layout(buf[offset:], N, in_place=in_place)
    check(L, ref)


def test_recode_hot_keys_colliding_buckets():
    """Hot keys that all share their low 13 bits fill one bucket of the LDS table; the rest of them are
    gathered from the rank array, and the recode stays exact."""
    N, F = 1 << 20, (1 << 24) + 99
    say("recode hot keys, colliding buckets")
    rng = np.random.default_rng(13)
    fact = rng.integers(0, N, F).astype(np.int32)
    hot = rng.random(F) < 0.5
    fact[hot] = (rng.integers(0, 64, int(hot.sum())) * 8192).astype(np.int32)
    ref = oracle.build_layout(fact, N)
    L = skew.build_skew_layout(to_dev(fact), N)
    check(L, ref)


@pytest.mark.parametrize("in_place", [False, True])
def test_recode_crowded_low_keys(in_place):
    """A column of more than 2^24 keys with most keys in the first eighth of the domain, a ragged end (length
    3 mod 4), in place and into a separate column."""
    N, F = 3_000_000, (1 << 24) + (1 << 22) + 3
    say(f"recode, crowded low keys, in_place={in_place}")
    rng = np.random.default_rng(21)
    fact = rng.integers(0, N, F).astype(np.int32)
    low = rng.random(F) < 0.8
    fact[low] = rng.integers(0, N // 8, int(low.sum())).astype(np.int32)
    ref = oracle.build_layout(fact, N)
    L = skew.build_skew_layout(to_dev(fact), N, in_place=in_place)
    check(L, ref)


# ---------------------------------------------------------------------------
# Index maintenance without a rebuild (Section 3.1): dimension rows appended
# after the build become the least frequent items and new fact rows are
# recoded through the extended index.  Every array equals the oracle's; the
# join over the old and new recoded facts equals the join over the original
# rows.  A batch of 2^24 + 5 new keys takes the recode with the LDS table.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_add_rows,n_add_facts", [(0, 1000), (5000, 2_000_003), (1, 1 << 24 | 5)])
def test_append_layout(n_add_rows, n_add_facts):
    k, N_old, F_old = 1, 100_000, 2_000_000
    say(f"append layout +{n_add_rows} rows +{n_add_facts} facts")
    N_new = N_old + n_add_rows
    h = W.host_join_inputs(k, N_new, F_old, 1.0)
    rng = np.random.default_rng(77 + n_add_rows)
    old = h["fact"] % N_old  # the column the layout was built on references the old rows only
    add = np.where(rng.random(n_add_facts) < 0.5, rng.integers(0, N_new, n_add_facts),
                   h["fact"][rng.integers(0, F_old, n_add_facts)] % N_new).astype(np.int32)
    ref = oracle.build_layout(old, N_old, h["price"][:N_old], h["category"][:N_old])
    perm, rank, pn, cn, add_n, inv = oracle.append_layout(ref, N_new, h["price"], h["category"], add)
    assert inv == 0
    d_old = to_dev(old)
    L = skew.build_skew_layout(d_old, N_old, to_dev(h["price"][:N_old]), to_dev(h["category"][:N_old]))
    L2, add_d = skew.append_skew_layout(L, N_new, to_dev(h["price"]), to_dev(h["category"]), to_dev(add))
    assert (host(L2.perm) == perm).all() and (host(L2.rank) == rank).all()
    assert (host(L2.price) == pn).all() and (host(L2.category) == cn).all()
    assert (host(L2.counts_by_rank)[N_old:] == 0).all()
    assert (host(add_d) == add_n).all()
    facts = np.concatenate([old, add])
    es, ec = oracle.fk_join_aggregate(facts, h["price"], h["category"], 16, True)
    keys = torch.cat([L.fact_recoded, add_d])
    gs, gc = skew.fk_join_aggregate(keys, L2.price, L2.category, 16, True, hot_rows=skew.SKEW_HOT_AUTO)
    assert (host(gs) == es).all() and (host(gc) == ec).all()

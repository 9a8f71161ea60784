"""Pins of the oracle against what the paper and the mathematics fix.

Each function raises AssertionError when the oracle module it is given
disagrees with an independent statement of the result: brute force on tiny
tables, the paper's worked example, closed forms, invariants.  The same
functions run against the real oracle (tests/test_oracle_pins.py) and against
copies of it with planted mistakes (tests/test_oracle_mutants.py), which must
each fail at least one pin.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------------------
# Brute force definitions (Python loops, tiny inputs only)
# ---------------------------------------------------------------------------
def nested_loop_join_aggregate(fact, dim_rows, cat_lt, by_category):
    """SUM(price), COUNT(*) over Sales JOIN Dim ON key, WHERE category < cat_lt.

    dim_rows is a list of (key, price, category) tuples in arbitrary storage
    order: the join matches key values, it never uses a key as an offset.
    """
    g = 16 if by_category else 1
    s = [0] * g
    c = [0] * g
    for fk in fact:
        for key, price, cat in dim_rows:
            if key != fk:
                continue
            if not (cat < cat_lt):
                continue
            grp = 0
            if by_category:
                if not (0 <= cat < 16):
                    continue
                grp = cat
            s[grp] += int(price)
            c[grp] += 1
    return s, c


def dict_group_aggregate(G, V, n_groups):
    s = {}
    c = {}
    for g, v in zip(G, V):
        g = int(g)
        if 0 <= g < n_groups:
            s[g] = s.get(g, 0) + int(v)
            c[g] = c.get(g, 0) + 1
    return [s.get(g, 0) for g in range(n_groups)], [c.get(g, 0) for g in range(n_groups)]


def brute_force_order(fact, n_keys):
    """Among all n_keys! orders, the one whose (-frequency, key) sequence is sorted."""
    freq = [0] * n_keys
    for k in fact:
        freq[int(k)] += 1
    best = None
    for order in itertools.permutations(range(n_keys)):
        seq = [(-freq[k], k) for k in order]
        if all(seq[i] <= seq[i + 1] for i in range(n_keys - 1)):
            assert best is None, "two sorted orders cannot exist for distinct keys"
            best = list(order)
    return best


# ---------------------------------------------------------------------------
# Pins
# ---------------------------------------------------------------------------
def pin_fk_bruteforce(orc, seeds=range(12)):
    for seed in seeds:
        rng = np.random.default_rng(seed)
        n = int(rng.integers(1, 9))
        f = int(rng.integers(0, 17))
        price = rng.integers(-50, 10000, n).astype(np.int32)
        cat = rng.integers(-3, 19, n).astype(np.int8)
        fact = rng.integers(-1, n + 1, f).astype(np.int32)  # includes out-of-range keys
        order = rng.permutation(n)
        rows = [(int(k), int(price[k]), int(cat[k])) for k in order]
        for cat_lt in (-128, 0, 4, 16, 127):
            for by in (False, True):
                s, c = orc.fk_join_aggregate(fact, price, cat, cat_lt, by)
                bs, bc = nested_loop_join_aggregate(fact.tolist(), rows, cat_lt, by)
                assert s.tolist() == bs and c.tolist() == bc, (seed, cat_lt, by)


def pin_fk_special_cases(orc):
    rng = np.random.default_rng(7)
    # N = 1: every fact joins the single row, sum = F * price[0]
    for F in (0, 1, 5, 1000):
        fact = np.zeros(F, dtype=np.int32)
        s, c = orc.fk_join_aggregate(fact, np.array([37], np.int32), np.array([2], np.int8), 4, False)
        assert s[0] == 37 * F and c[0] == F
        s, c = orc.fk_join_aggregate(fact, np.array([37], np.int32), np.array([9], np.int8), 4, False)
        assert s[0] == 0 and c[0] == 0
    # F = 0: all zeros
    s, c = orc.fk_join_aggregate(np.zeros(0, np.int32), np.arange(5, dtype=np.int32),
                                 np.arange(5, dtype=np.int8), 16, True)
    assert not s.any() and not c.any()
    # no filter and categories in [0, 16): group counts sum to F; cat_lt = 16 equals no filter
    n, F = 50, 3000
    price = rng.integers(1, 10001, n).astype(np.int32)
    cat = rng.integers(0, 16, n).astype(np.int8)
    fact = rng.integers(0, n, F).astype(np.int32)
    s16, c16 = orc.fk_join_aggregate(fact, price, cat, 16, True)
    s127, c127 = orc.fk_join_aggregate(fact, price, cat, 127, True)
    assert c16.sum() == F and (s16 == s127).all() and (c16 == c127).all()
    assert s16.sum() == int(price[fact].astype(np.int64).sum())
    # filter cat < 4 without grouping equals the sum of groups 0..3
    s4, c4 = orc.fk_join_aggregate(fact, price, cat, 4, False)
    assert s4[0] == s16[:4].sum() and c4[0] == c16[:4].sum()


def pin_group_bruteforce(orc, seeds=range(10)):
    for seed in seeds:
        rng = np.random.default_rng(100 + seed)
        m = int(rng.integers(1, 12))
        f = int(rng.integers(0, 40))
        G = rng.integers(-1, m + 1, f).astype(np.int32)
        V = rng.integers(-2**31, 2**31, f, dtype=np.int64).astype(np.int32)
        s, c, inv = orc.group_aggregate(G, V, m)
        bs, bc = dict_group_aggregate(G.tolist(), V.tolist(), m)
        assert s.tolist() == bs and c.tolist() == bc, seed
        assert inv == int(((G < 0) | (G >= m)).sum())


def pin_layout_bruteforce(orc):
    # every fact column over N = 3 keys with F = 4 rows (81 columns)
    for fact in itertools.product(range(3), repeat=4):
        fact = np.array(fact, dtype=np.int32)
        L = orc.build_layout(fact, 3)
        assert L.perm.tolist() == brute_force_order(fact.tolist(), 3), fact
    # random columns for N up to 6, including keys that never occur
    for seed in range(40):
        rng = np.random.default_rng(200 + seed)
        n = int(rng.integers(1, 7))
        f = int(rng.integers(0, 12))
        fact = rng.integers(0, n, f).astype(np.int32)
        L = orc.build_layout(fact, n)
        assert L.perm.tolist() == brute_force_order(fact.tolist(), n), (seed, fact)


def pin_fig2(orc):
    d = json.load(open(os.path.join(GOLDEN, "fig2_permutation_index.json")))
    fact = np.array(d["fact_column_1based"], dtype=np.int32) - 1
    letters = d["dimension_rows_1based"]
    n = len(letters)
    # the dimension's first column holds the letters; use their code points as int32 values
    col = np.array([ord(x) for x in letters], dtype=np.int32)
    L = orc.build_layout(fact, n, price=col)
    assert [int(k) + 1 for k in L.perm[:4]] == d["paper_first_four_keys_1based"]
    assert [chr(v) for v in L.price] == d["paper_permuted_dimension"]
    assert L.perm.tolist() == d["expected_perm_0based"]
    assert L.rank.tolist() == d["expected_rank_0based"]
    # the most frequent key is recoded to 0 and so on (Fig. 2c -> 2d)
    assert (L.fact_recoded == np.array(d["expected_rank_0based"])[fact]).all()


def check_layout_invariants(L, fact, n_keys, price=None, category=None):
    perm, rank = L.perm, L.rank
    assert sorted(perm.tolist()) == list(range(n_keys)), "perm is a bijection"
    assert (rank[perm] == np.arange(n_keys)).all(), "rank is the inverse of perm"
    cnt = np.bincount(fact, minlength=n_keys) if fact.size else np.zeros(n_keys, np.int64)
    assert (L.counts_by_rank == cnt[perm]).all()
    assert (np.diff(L.counts_by_rank) <= 0).all(), "frequencies non-increasing along perm"
    ties = np.diff(L.counts_by_rank) == 0
    assert (np.diff(perm)[ties] > 0).all(), "equal frequencies in ascending key order"
    assert L.counts_by_rank.sum() == fact.size
    assert (L.fact_recoded == rank[fact]).all()
    if price is not None:
        assert (L.price[L.fact_recoded] == price[fact]).all(), "materialisation through the new layout"
    if category is not None:
        assert (L.category[L.fact_recoded] == category[fact]).all()


def pin_layout_invariants(orc):
    for seed in range(6):
        rng = np.random.default_rng(300 + seed)
        n = int(rng.integers(1, 2000))
        f = int(rng.integers(0, 20000))
        w = rng.zipf(1.5, f) % n if f else np.zeros(0, np.int64)
        fact = w.astype(np.int32)
        price = rng.integers(1, 10001, n).astype(np.int32)
        cat = rng.integers(0, 16, n).astype(np.int8)
        L = orc.build_layout(fact, n, price, cat)
        check_layout_invariants(L, fact, n, price, cat)


def pin_invariance_all_layouts(orc):
    """Any bijection used as a layout leaves every answer unchanged (Section 3.2)."""
    rng = np.random.default_rng(11)
    n, F = 6, 60
    fact = rng.integers(0, n, F).astype(np.int32)
    price = rng.integers(1, 100, n).astype(np.int32)
    cat = rng.integers(0, 16, n).astype(np.int8)
    vals = rng.integers(-1000, 1000, F).astype(np.int32)
    ref = {(lt, by): orc.fk_join_aggregate(fact, price, cat, lt, by) for lt in (4, 16) for by in (False, True)}
    gs, gc, _ = orc.group_aggregate(fact, vals, n)
    for p in itertools.permutations(range(n)):
        perm = np.array(p, dtype=np.int32)
        rank = np.empty(n, np.int32)
        rank[perm] = np.arange(n, dtype=np.int32)
        fr = orc.recode(fact, rank)
        pp = orc.permute_dim(price, perm)
        cp = orc.permute_dim(cat, perm)
        for (lt, by), (s, c) in ref.items():
            s2, c2 = orc.fk_join_aggregate(fr, pp, cp, lt, by)
            assert (s == s2).all() and (c == c2).all()
        s2, c2, _ = orc.group_aggregate(fr, vals, n)
        # un-permute: group of rank r is key perm[r]
        us = np.empty_like(s2)
        uc = np.empty_like(c2)
        us[perm] = s2
        uc[perm] = c2
        assert (us == gs).all() and (uc == gc).all()


def pin_stale_layout(orc):
    """A layout built on one fact column still gives exact answers on another (Section 3.1)."""
    rng = np.random.default_rng(21)
    n = 500
    a = (rng.zipf(1.2, 5000) % n).astype(np.int32)
    b = rng.integers(0, n, 7000).astype(np.int32)
    price = rng.integers(1, 10001, n).astype(np.int32)
    cat = rng.integers(0, 16, n).astype(np.int8)
    L = orc.build_layout(a, n, price, cat)
    bn = orc.recode(b, L.rank)
    for lt, by in ((4, False), (16, True)):
        s, c = orc.fk_join_aggregate(b, price, cat, lt, by)
        s2, c2 = orc.fk_join_aggregate(bn, L.price, L.category, lt, by)
        assert (s == s2).all() and (c == c2).all()


def pin_append_layout(orc, seeds=range(10)):
    """Index maintenance (Section 3.1): dimension rows appended after the build become the least frequent items
    and fact rows inserted afterwards are recoded through the extended index.  The extended layout must still be a
    bijection whose inverse is the rank form, and the join over the recoded facts and the permuted, extended
    dimension must equal a nested-loop join on key values over the original rows."""
    for seed in seeds:
        rng = np.random.default_rng(500 + seed)
        n_old = int(rng.integers(1, 7))
        n_new = n_old + int(rng.integers(0, 4))
        price = rng.integers(-50, 10000, n_new).astype(np.int32)
        cat = rng.integers(-3, 19, n_new).astype(np.int8)
        old = rng.integers(0, n_old, int(rng.integers(0, 15))).astype(np.int32)
        add = rng.integers(0, n_new, int(rng.integers(0, 15))).astype(np.int32)
        L = orc.build_layout(old, n_old, price[:n_old], cat[:n_old])
        perm, rank, pn, cn, add_n, inv = orc.append_layout(L, n_new, price, cat, add)
        assert inv == 0
        assert sorted(perm.tolist()) == list(range(n_new)), seed
        assert all(rank[perm[r]] == r for r in range(n_new)), seed
        assert all(rank[k] >= n_old for k in range(n_old, n_new)), seed  # appended ids rank after every old one
        assert (perm[:n_old] == L.perm).all() and (rank[:n_old] == L.rank).all(), seed  # no reorganisation
        rows = [(int(k), int(price[k]), int(cat[k])) for k in rng.permutation(n_new)]
        facts = np.concatenate([old, add])
        recoded = np.concatenate([L.fact_recoded, add_n])
        for cat_lt in (4, 16):
            for by in (False, True):
                s, c = orc.fk_join_aggregate(recoded, pn, cn, cat_lt, by)
                bs, bc = nested_loop_join_aggregate(facts.tolist(), rows, cat_lt, by)
                assert s.tolist() == bs and c.tolist() == bc, (seed, cat_lt, by)


# ---------------------------------------------------------------------------
# Operator variants (Section 4.1): materialization, selection, heavy hitters
# ---------------------------------------------------------------------------
def nested_loop_materialize(fact, dim_rows):
    """For every fact key the value of the dimension row whose key matches (0 if none)."""
    out = []
    for fk in fact:
        v = 0
        for key, val in dim_rows:
            if key == fk:
                v = val
        out.append(v)
    return out


def pin_materialize(orc, seeds=range(12)):
    for seed in seeds:
        rng = np.random.default_rng(300 + seed)
        n = int(rng.integers(1, 9))
        f = int(rng.integers(0, 20))
        col = rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32)
        fact = rng.integers(-2, n + 2, f).astype(np.int32)
        rows = [(int(k), int(col[k])) for k in rng.permutation(n)]
        out, inv = orc.materialize(fact, col)
        assert out.tolist() == nested_loop_materialize(fact.tolist(), rows), seed
        assert inv == int(((fact < 0) | (fact >= n)).sum())
    # the materialized price column sums to the join's unfiltered SUM(price)
    rng = np.random.default_rng(31)
    n, F = 200, 5000
    price = rng.integers(1, 10001, n).astype(np.int32)
    cat = rng.integers(0, 16, n).astype(np.int8)
    fact = rng.integers(0, n, F).astype(np.int32)
    out, _ = orc.materialize(fact, price)
    s, _ = orc.fk_join_aggregate(fact, price, cat, 127, False)
    assert int(out.astype(np.int64).sum()) == int(s[0])
    # layout invariance: D'[C'[j]] = D[C[j]] for every row (Section 3.2)
    L = orc.build_layout(fact, n, price, cat)
    out2, _ = orc.materialize(L.fact_recoded, L.price)
    assert (out2 == out).all()


def pin_select(orc, seeds=range(12)):
    for seed in seeds:
        rng = np.random.default_rng(400 + seed)
        n = int(rng.integers(1, 9))
        f = int(rng.integers(0, 25))
        col = rng.integers(-20, 20, n).astype(np.int32)
        fact = rng.integers(-2, n + 2, f).astype(np.int32)
        rows = [(int(k), int(col[k])) for k in rng.permutation(n)]
        for lt in (-100, -3, 0, 7, 100):
            want = []
            for j, fk in enumerate(fact.tolist()):
                for key, val in rows:
                    if key == fk and val < lt:
                        want.append(j)
            assert orc.select(fact, col, lt).tolist() == want, (seed, lt)
    # the number of selected rows is the join's COUNT(*) under the same filter on category
    rng = np.random.default_rng(41)
    n, F = 300, 6000
    price = rng.integers(1, 10001, n).astype(np.int32)
    cat = rng.integers(-5, 20, n).astype(np.int8)
    fact = rng.integers(0, n, F).astype(np.int32)
    for lt in (-1, 4, 16):
        _, c = orc.fk_join_aggregate(fact, price, cat, lt, False)
        assert orc.select(fact, cat.astype(np.int32), lt).size == int(c[0])
    # layout invariance: the same fact offsets qualify on the skew layout
    L = orc.build_layout(fact, n, price, cat)
    assert (orc.select(L.fact_recoded, L.price, 5000) == orc.select(fact, price, 5000)).all()


def pin_heavy_hitters(orc, seeds=range(10)):
    for seed in seeds:
        rng = np.random.default_rng(500 + seed)
        n = int(rng.integers(1, 12))
        f = int(rng.integers(0, 60))
        G = rng.integers(-1, n + 1, f).astype(np.int32)
        cnt = {}
        for g in G.tolist():
            if 0 <= g < n:
                cnt[g] = cnt.get(g, 0) + 1
        order = sorted(range(n), key=lambda g: (-cnt.get(g, 0), g))
        for k in (0, 1, n // 2, n, n + 3):
            keys, counts = orc.heavy_hitters(G, n, k)
            kk = min(k, n)
            assert keys.tolist() == order[:kk], (seed, k)
            assert counts.tolist() == [cnt.get(g, 0) for g in order[:kk]], (seed, k)
    # the top-k are the first k ranks of the permutation index with their frequencies (Section 4.2.2)
    rng = np.random.default_rng(51)
    n = 400
    G = (rng.zipf(1.3, 20000) % n).astype(np.int32)
    L = orc.build_layout(G, n)
    keys, counts = orc.heavy_hitters(G, n, 50)
    assert (keys == L.perm[:50]).all() and (counts == L.counts_by_rank[:50]).all()


# ---------------------------------------------------------------------------
# Stack-distance cache model (Section 3.3)
# ---------------------------------------------------------------------------
def lru_hit_rate(f, S, n, seed):
    """Exact LRU cache of S lines fed n i.i.d. accesses drawn from f (hits after a warm-up fifth)."""
    import collections

    rng = np.random.default_rng(seed)
    acc = rng.choice(f.size, size=n, p=f)
    cache = collections.OrderedDict()
    hits = 0
    warm = n // 5
    for t, a in enumerate(acc.tolist()):
        if a in cache:
            cache.move_to_end(a)
            hits += t >= warm
        else:
            cache[a] = None
            if len(cache) > S:
                cache.popitem(last=False)
    return hits / (n - warm)


def pin_cache_model(orc):
    # uniform lines: no line repeats before S trials, so K = S and the rate is 1 - (1 - 1/L)^S
    for L, S in ((50, 1), (50, 7), (1000, 100), (1000, 999)):
        f = np.full(L, 1.0 / L)
        assert abs(orc.cache_model(f, S) - (1 - (1 - 1 / L) ** S)) < 1e-12, (L, S)
    # one hot line h and L - 1 equal cold lines c: for the hot line no other line repeats before
    # L - 1 trials, so K = S; for a cold line the hot line repeats from k > (1 - c) / h on, so
    # d(k) = k (1 - a) + 1 with a = h / (1 - c) and K = ceil((S - 1) / (1 - a))
    for L, h, S in ((1000, 0.3, 100), (500, 0.05, 40), (2000, 0.6, 300)):
        c = (1 - h) / (L - 1)
        a = h / (1 - c)
        K = max(S, int(np.ceil((S - 1) / (1 - a))))
        assert (1 - c) / h < K < L - 1
        want = h * (1 - (1 - h) ** S) + (1 - h) * (1 - (1 - c) ** K)
        f = np.concatenate([[h], np.full(L - 1, c)])
        assert abs(orc.cache_model(f, S) - want) < 1e-9, (L, h, S)
    # two hot lines h1, h2 and L - 2 equal cold lines c: seen from line 1 the other hot line repeats
    # once k h2 / (1 - h1) > 1, so d(k) = k (1 - h2 / (1 - h1)) + 1; from line 2 likewise; from a
    # cold line both hot lines repeat, d(k) = k (1 - (h1 + h2) / (1 - c)) + 2
    L, h1, h2, S = 1000, 0.5, 0.3, 50
    c = (1 - h1 - h2) / (L - 2)
    K1 = int(np.ceil((S - 1) / (1 - h2 / (1 - h1))))
    K2 = int(np.ceil((S - 1) / (1 - h1 / (1 - h2))))
    Kc = int(np.ceil((S - 2) / (1 - (h1 + h2) / (1 - c))))
    assert max(K1, K2, Kc) < (1 - c) / c / 2
    want = h1 * (1 - (1 - h1) ** K1) + h2 * (1 - (1 - h2) ** K2) + (L - 2) * c * (1 - (1 - c) ** Kc)
    f = np.concatenate([[h1, h2], np.full(L - 2, c)])
    assert abs(orc.cache_model(f, S) - want) < 1e-9
    # a cache that holds every line, or a single line, always hits
    f = np.array([0.5, 0.25, 0.125, 0.125])
    assert abs(orc.cache_model(f, 4) - 1.0) < 1e-12
    assert abs(orc.cache_model(np.array([1.0]), 1) - 1.0) < 1e-12
    # zero-frequency lines change nothing
    g = np.concatenate([f, np.zeros(5)])
    assert abs(orc.cache_model(g, 2) - orc.cache_model(f, 2)) < 1e-12
    # the hit rate grows with the cache
    rng = np.random.default_rng(3)
    r = np.arange(1, 401, dtype=np.float64) ** -1.0
    z = (r / r.sum())[rng.permutation(400)]
    rates = [orc.cache_model(z, S) for S in (1, 5, 20, 80, 200)]
    assert all(a < b for a, b in zip(rates, rates[1:]))
    # within the paper's 5 % of an exact LRU simulation for caches up to a tenth of the lines
    for s in (0.0, 0.5, 1.0, 1.5):
        L = 1500
        r = np.arange(1, L + 1, dtype=np.float64) ** -s
        f = (r / r.sum())[np.random.default_rng(7).permutation(L)]
        for S in (15, 150):
            m = orc.cache_model(f, S)
            sim = lru_hit_rate(f, S, 60_000, 11)
            assert abs(m - sim) < 0.05, (s, S, m, sim)


# ---------------------------------------------------------------------------
# Star join (two dimensions, batched star-join workload)
# ---------------------------------------------------------------------------
def pin_star_join(orc, seeds=range(10)):
    for seed in seeds:
        rng = np.random.default_rng(600 + seed)
        n_p, n_c = int(rng.integers(1, 7)), int(rng.integers(1, 6))
        f = int(rng.integers(0, 25))
        price = rng.integers(-100, 10000, n_p).astype(np.int32)
        cat = rng.integers(-2, 18, n_p).astype(np.int8)
        attr = rng.integers(-5, 100, n_c).astype(np.int8)
        P = rng.integers(-1, n_p + 1, f).astype(np.int32)
        U = rng.integers(-1, n_c + 1, f).astype(np.int32)
        prod = [(int(k), int(price[k]), int(cat[k])) for k in rng.permutation(n_p)]
        cust = [(int(k), int(attr[k])) for k in rng.permutation(n_c)]
        for lt in (-128, 0, 30, 127):
            s = [0] * 16
            c = [0] * 16
            for pk, uk in zip(P.tolist(), U.tolist()):
                for ck, a in cust:
                    if ck != uk or not (a < lt):
                        continue
                    for key, pr, g in prod:
                        if key == pk and 0 <= g < 16:
                            s[g] += pr
                            c[g] += 1
            gs, gc = orc.star_join(P, U, price, cat, attr, lt)
            assert gs.tolist() == s and gc.tolist() == c, (seed, lt)
    # a customer filter that every row passes reduces to the one-dimension join grouped by category
    rng = np.random.default_rng(61)
    n_p, n_c, F = 300, 50, 4000
    price = rng.integers(1, 10001, n_p).astype(np.int32)
    cat = rng.integers(0, 16, n_p).astype(np.int8)
    attr = rng.integers(0, 100, n_c).astype(np.int8)
    P = rng.integers(0, n_p, F).astype(np.int32)
    U = rng.integers(0, n_c, F).astype(np.int32)
    s1, c1 = orc.star_join(P, U, price, cat, attr, 100)
    s2, c2 = orc.fk_join_aggregate(P, price, cat, 16, True)
    assert (s1 == s2).all() and (c1 == c2).all()
    # recoding both key columns through their layouts (union histograms) changes no answer (Section 3.2)
    Lp = orc.build_layout(P, n_p, price, cat)
    Lc = orc.build_layout(U, n_c)
    attr_n = orc.permute_dim(attr, Lc.perm)
    for lt in (10, 50):
        a = orc.star_join(P, U, price, cat, attr, lt)
        b = orc.star_join(Lp.fact_recoded, Lc.fact_recoded, Lp.price, Lp.category, attr_n, lt)
        assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


ALL_PINS = [pin_fk_bruteforce, pin_fk_special_cases, pin_group_bruteforce, pin_layout_bruteforce, pin_fig2,
            pin_layout_invariants, pin_invariance_all_layouts, pin_stale_layout, pin_append_layout, pin_materialize,
            pin_select,
            pin_heavy_hitters, pin_cache_model, pin_star_join]

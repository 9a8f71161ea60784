"""Seeded generator against the Zipf closed form (Section 2.1) and basic properties."""
import math

import numpy as np
import pytest

import oracle
from paper_1910_10063_amd import workload as W


@pytest.mark.parametrize("n,s", [(100_000, 1.0), (10_000, 0.0), (10_000, 0.5), (1_000_000, 1.1), (10_000, 1.5)])
def test_zipf_cumulative_share_matches_closed_form(n, s):
    """Share of rows with rank < r is H_{r,s} / H_{n,s}: binomial, checked within 6 sigma."""
    F = 400_000
    cdf = W.zipf_cdf(n, s)
    ranks = W.zipf_ranks(W.fact_seed(1), cdf, F)
    assert ranks.min() >= 0 and ranks.max() < n
    Hn = W.harmonic(n, s)
    for r in (1, 2, 10, 100, n // 100, n // 10, n // 2):
        if r < 1:
            continue
        p = W.harmonic(r, s) / Hn
        share = np.count_nonzero(ranks < r) / F
        sigma = math.sqrt(max(p * (1 - p), 1e-12) / F)
        assert abs(share - p) <= 6 * sigma + 1e-12, (r, share, p)


def test_zipf_s0_is_uniform():
    cdf = W.zipf_cdf(1000, 0.0)
    assert np.allclose(cdf, np.arange(1, 1001) / 1000.0, rtol=0, atol=1e-12)


def test_cdf_table_properties():
    for s in (0.0, 0.5, 1.0, 1.5):
        cdf = W.zipf_cdf(100_000, s)
        assert cdf[-1] == 1.0 and (np.diff(cdf) >= 0).all() and cdf[0] > 0


def test_permutation_is_bijection_and_seeded():
    p = W.permutation(W.perm_seed(1), 100_000)
    assert sorted(p.tolist()) == list(range(100_000))
    assert (p == W.permutation(W.perm_seed(1), 100_000)).all()
    assert not (p == W.permutation(W.perm_seed(2), 100_000)).all()


def test_head_of_permutation_recovered_by_layout():
    """At s=1.0 the first ranks' expected counts are separated by > 8 sigma, so the
    oracle's frequency order must return the generator's permutation head."""
    n, F, s = 100_000, 1_000_000, 1.0
    cdf = W.zipf_cdf(n, s)
    pi = W.permutation(W.perm_seed(1), n)
    fact = W.fact_keys(W.fact_seed(1), cdf, pi, F)
    cnt, inv = oracle.key_counts(fact, n)
    assert inv == 0
    perm, _ = oracle.permutation_index(cnt)
    H = W.harmonic(n, s)
    r = 0
    while True:  # ranks whose neighbours are > 8 sigma apart
        mu, mu2 = F / H / (r + 1), F / H / (r + 2)
        if mu - mu2 <= 8 * math.sqrt(mu):
            break
        r += 1
    assert r >= 5
    assert (perm[:r] == pi[:r]).all()


def test_uniform_bounds_and_coverage():
    v = W.uniform_int(W.price_seed(1), 1, 10000, 200_000)
    assert v.min() >= 1 and v.max() <= 10000 and len(np.unique(v)) > 9900
    c = W.uniform_int(W.category_seed(1), 0, 15, 100_000)
    counts = np.bincount(c, minlength=16)
    assert counts.size == 16 and counts.min() > 5500
    assert (W.uniform_int(7, -5, 5, 1000) >= -5).all()


def test_streams_are_counter_based():
    """Row j depends only on (seed, j): a slice equals the matching part of a longer run."""
    cdf = W.zipf_cdf(1000, 1.0)
    a = W.zipf_ranks(5, cdf, 1000)
    b = W.zipf_ranks(5, cdf, 100, start=450)
    assert (a[450:550] == b).all()
    x = W.uniform_int(9, 0, 99, 500)
    assert (x[123:200] == W.uniform_int(9, 0, 99, 77, start=123)).all()


def test_splitmix_reference_values():
    """SplitMix64 from seed 0: first outputs of the published generator (state += golden, then mix)."""
    # next() of the published generator with state 0 returns mix(0x9E3779B97F4A7C15)
    x = W.stream(0, 0, 3)
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [int(v) for v in x] == expect

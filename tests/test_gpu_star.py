"""GPU parity of the batched star join against the CPU oracle, bit-exact.

A batch of fact tables of uneven sizes (empty, ragged, several tiles) with a
product key and a customer key per row; every query's SUM(price) and
COUNT(*) by category over rows whose customer segment passes its threshold
must equal the oracle's, on the identity layouts and on the frequency-ordered
layouts of both dimensions (built from all queries' keys), for many tunings,
and from a HIP graph replayed several times.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1910_10063_amd import skew
from paper_1910_10063_amd import workload as W

pytestmark = pytest.mark.gpu

DEV = "cuda"
SIZES = np.array([0, 1, 3, 5, 1000, 4097, 65537, 0, 300_000, 1_000_003, 2], dtype=np.int64)


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def batch():
    k, n_prod, n_cust = 4, 20_000, 5_000
    say(f"star batch n_prod={n_prod} n_cust={n_cust} sizes={SIZES.tolist()}")
    h = W.host_star_inputs(k, n_prod, n_cust, SIZES)
    lt = np.array([1, 50, 25, 7, 33, 50, 12, 40, 2, 49, 30], dtype=np.int32)
    start = np.concatenate([[0], np.cumsum(SIZES)]).astype(np.int64)
    want = []
    for q in range(SIZES.size):
        a, b = start[q], start[q + 1]
        want.append(oracle.star_join(h["prod"][a:b], h["cust"][a:b], h["price"], h["category"], h["cust_attr"], lt[q]))
    ident = skew.StarBatch(to_dev(h["prod"]), to_dev(h["cust"]), to_dev(start), to_dev(lt), to_dev(h["price"]),
                           to_dev(h["category"]), to_dev(h["cust_attr"]))
    Lp = skew.build_skew_layout(ident.prod_keys, n_prod, ident.price, ident.category)
    Lc = skew.build_skew_layout(ident.cust_keys, n_cust, None, ident.segment)
    sk = skew.StarBatch(Lp.fact_recoded, Lc.fact_recoded, ident.query_start, ident.query_cust_lt, Lp.price,
                        Lp.category, Lc.category)
    return dict(identity=ident, skew=sk, want=want)


def check(out, want):
    s, c = host(out[0]), host(out[1])
    for q, (ws, wc) in enumerate(want):
        assert (s[q] == ws).all() and (c[q] == wc).all(), q


@pytest.mark.parametrize("tun", [None, (0, 0, 1024, 0), (0, 0, 65536, 1), (37, 100, 4096, 7),
                                 (-1, 5000, 1 << 20, 0), (-1, 0, 3000, 3), (20_000, 4999, 262_144, 0)],
                         ids=str)
@pytest.mark.parametrize("layout", ["skew", "identity"])
def test_star_batch(batch, tun, layout):
    say(f"star batch {layout} tuning={tun}")
    t = None if tun is None else skew.StarTuning(*tun)
    check(skew.star_join_batch(batch[layout], t), batch["want"])


@pytest.fixture(scope="module")
def wide():
    """A customer dimension larger than the default LDS customer prefix (262144 rows)."""
    k, n_prod, n_cust = 5, 200_000, 300_000
    sizes = np.array([70_001, 1_000_003, 5], dtype=np.int64)
    say(f"star wide batch n_prod={n_prod} n_cust={n_cust}")
    h = W.host_star_inputs(k, n_prod, n_cust, sizes)
    lt = np.array([50, 17, 3], dtype=np.int32)
    start = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    want = [oracle.star_join(h["prod"][a:b], h["cust"][a:b], h["price"], h["category"], h["cust_attr"], lt[q])
            for q, (a, b) in enumerate(zip(start[:-1], start[1:]))]
    ident = skew.StarBatch(to_dev(h["prod"]), to_dev(h["cust"]), to_dev(start), to_dev(lt), to_dev(h["price"]),
                           to_dev(h["category"]), to_dev(h["cust_attr"]))
    Lp = skew.build_skew_layout(ident.prod_keys, n_prod, ident.price, ident.category)
    Lc = skew.build_skew_layout(ident.cust_keys, n_cust, None, ident.segment)
    sk = skew.StarBatch(Lp.fact_recoded, Lc.fact_recoded, ident.query_start, ident.query_cust_lt, Lp.price,
                        Lp.category, Lc.category)
    return dict(identity=ident, skew=sk, want=want)


@pytest.mark.parametrize("tun", [(-1, 65536, 262_144, 0), (-1, 98_304, 65_536, 0), (-1, 131_072, 262_144, 0),
                                 (-1, 250_000, 1 << 20, 0), (3, 131_072, 4096, 5)], ids=str)
@pytest.mark.parametrize("layout", ["skew", "identity"])
def test_star_wide_customer_prefix(wide, tun, layout):
    say(f"star wide {layout} tuning={tun}")
    check(skew.star_join_batch(wide[layout], skew.StarTuning(*tun)), wide["want"])


def test_star_autotune_wide(wide):
    say("star autotune wide")
    best, ms = skew.star_join_autotune(wide["skew"])
    assert ms > 0 and best.cust_hot_rows <= 300_000
    check(skew.star_join_batch(wide["skew"], best), wide["want"])


@pytest.fixture(scope="module")
def signed():
    """1.2M customers (more than the largest LDS bitmap, 2^20 rows) with segments in [-100, 98] and thresholds
    at and around the ends of the int8 range; six queries, so workgroups move between queries' bitmaps."""
    k, n_prod, n_cust = 6, 150_000, 1_200_000
    sizes = np.array([70_001, 900_007, 5, 0, 200_000, 31], dtype=np.int64)
    say(f"star signed batch n_prod={n_prod} n_cust={n_cust}")
    h = W.host_star_inputs(k, n_prod, n_cust, sizes)
    seg = (h["cust_attr"].astype(np.int16) * 2 - 100).astype(np.int8)
    lt = np.array([-50, 17, 127, 0, -128, 128], dtype=np.int32)
    start = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    want = [oracle.star_join(h["prod"][a:b], h["cust"][a:b], h["price"], h["category"], seg, lt[q])
            for q, (a, b) in enumerate(zip(start[:-1], start[1:]))]
    ident = skew.StarBatch(to_dev(h["prod"]), to_dev(h["cust"]), to_dev(start), to_dev(lt), to_dev(h["price"]),
                           to_dev(h["category"]), to_dev(seg))
    Lp = skew.build_skew_layout(ident.prod_keys, n_prod, ident.price, ident.category)
    Lc = skew.build_skew_layout(ident.cust_keys, n_cust, None, ident.segment)
    sk = skew.StarBatch(Lp.fact_recoded, Lc.fact_recoded, ident.query_start, ident.query_cust_lt, Lp.price,
                        Lp.category, Lc.category)
    return dict(identity=ident, skew=sk, want=want)


@pytest.mark.parametrize("tun", [None, (-1, 1 << 20, 262_144, 0), (-1, 1_000_001, 4096, 0), (7, 524_295, 65_536, 9),
                                 (-1, 31, 1024, 0), (0, 0, 262_144, 0)], ids=str)
@pytest.mark.parametrize("layout", ["skew", "identity"])
def test_star_signed_segments_large_prefix(signed, tun, layout):
    say(f"star signed {layout} tuning={tun}")
    check(skew.star_join_batch(signed[layout], None if tun is None else skew.StarTuning(*tun)), signed["want"])


def test_star_autotune_signed(signed):
    say("star autotune signed")
    best, ms = skew.star_join_autotune(signed["skew"])
    assert ms > 0 and 0 <= best.cust_hot_rows <= 1 << 20
    check(skew.star_join_batch(signed["skew"], best), signed["want"])


@pytest.fixture(scope="module")
def many_cust():
    """4096 queries (the most a batch takes) of 0-299 rows over 2.5e6 customers: bitmaps of every customer row
    for every query would take 1.28 GB, over the library's 1 GiB budget, so cold customer rows gather their
    segments instead of a bit."""
    k, n_prod, n_cust, nq = 7, 50_000, 2_500_000, 4096
    rng = np.random.default_rng(77)
    sizes = rng.integers(0, 300, nq).astype(np.int64)
    lt = rng.integers(-5, 106, nq).astype(np.int32)
    say(f"star many-query batch nq={nq} n_cust={n_cust} rows={int(sizes.sum())}")
    h = W.host_star_inputs(k, n_prod, n_cust, sizes)
    start = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    want = [oracle.star_join(h["prod"][a:b], h["cust"][a:b], h["price"], h["category"], h["cust_attr"], lt[q])
            for q, (a, b) in enumerate(zip(start[:-1], start[1:]))]
    ident = skew.StarBatch(to_dev(h["prod"]), to_dev(h["cust"]), to_dev(start), to_dev(lt), to_dev(h["price"]),
                           to_dev(h["category"]), to_dev(h["cust_attr"]))
    Lp = skew.build_skew_layout(ident.prod_keys, n_prod, ident.price, ident.category)
    Lc = skew.build_skew_layout(ident.cust_keys, n_cust, None, ident.segment)
    sk = skew.StarBatch(Lp.fact_recoded, Lc.fact_recoded, ident.query_start, ident.query_cust_lt, Lp.price,
                        Lp.category, Lc.category)
    return dict(identity=ident, skew=sk, want=want, nq=nq, n_cust=n_cust)


@pytest.mark.parametrize("tun", [None, (-1, 1 << 20, 1024, 0), (100, 0, 4096, 3)], ids=str)
@pytest.mark.parametrize("layout", ["skew", "identity"])
def test_star_many_queries_segment_gathers(many_cust, tun, layout):
    say(f"star many queries, 2.5e6 customers, {layout} tuning={tun}")
    b = many_cust
    ws = skew.star_workspace(b[layout])
    assert ws.numel() < b["nq"] * b["n_cust"] // 8  # no room for bitmaps of every row
    check(skew.star_join_batch(b[layout], None if tun is None else skew.StarTuning(*tun), ws=ws), b["want"])


def test_star_autotune(batch):
    say("star autotune")
    best, ms = skew.star_join_autotune(batch["skew"])
    assert ms > 0 and best.tile_rows >= 1024
    check(skew.star_join_batch(batch["skew"], best), batch["want"])


def test_star_graph_replay(batch):
    """The call captured in a HIP graph: every replay equals the eager result."""
    say("star graph capture and replay")
    b = batch["skew"]
    ws = skew.star_workspace(b)
    nq = b.query_cust_lt.numel()
    out = (torch.empty(nq, 16, dtype=torch.int64, device=DEV), torch.empty(nq, 16, dtype=torch.int64, device=DEV))
    tun = skew.StarTuning(-1, 4096, 65536, 0)
    skew.star_join_batch(b, tun, ws=ws, out=out)  # eager run (also sets the kernel's LDS limit)
    torch.cuda.synchronize()
    check(out, batch["want"])
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        skew.star_join_batch(b, tun, ws=ws, out=out)
    for i in range(4):
        out[0].fill_(-1)
        out[1].fill_(-7)
        junk = torch.randn(1 << 20, device=DEV).sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check(out, batch["want"])
        assert torch.isfinite(junk)


def test_star_out_of_range_keys(batch):
    say("star out-of-range keys")
    b = batch["identity"]
    p = b.prod_keys.clone()
    u = b.cust_keys.clone()
    p[10] = 20_000
    u[1500] = -1
    bad = skew.StarBatch(p, u, b.query_start, b.query_cust_lt, b.price, b.category, b.segment)
    ws = skew.star_workspace(bad)
    skew.star_join_batch(bad, ws=ws)
    with pytest.raises(skew.SkewError):
        skew.query_status(ws)


def test_star_rejects_unaligned_keys(batch):
    b = batch["identity"]
    lib = skew.load_library()
    ws = skew.star_workspace(b)
    out = torch.empty(2, b.query_cust_lt.numel(), 16, dtype=torch.int64, device=DEV)
    rc = lib.star_join_batch(ctypes.c_void_p(b.prod_keys.data_ptr() + 4), ctypes.c_void_p(b.cust_keys.data_ptr()),
                             ctypes.c_void_p(b.query_start.data_ptr()), ctypes.c_void_p(b.query_cust_lt.data_ptr()),
                             b.query_cust_lt.numel(), ctypes.c_void_p(b.price.data_ptr()),
                             ctypes.c_void_p(b.category.data_ptr()), b.price.numel(),
                             ctypes.c_void_p(b.segment.data_ptr()), b.segment.numel(), None,
                             ctypes.c_void_p(out[0].data_ptr()), ctypes.c_void_p(out[1].data_ptr()),
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert rc == skew.SKEW_EINVAL


@pytest.fixture(scope="module")
def many():
    """The largest batch, 4096 queries of 0-3000 rows, with thresholds below, inside and above the segment range:
    the tile table fills 16 KB of LDS, and workgroups stage a new query's bitmap on almost every tile."""
    k, n_prod, n_cust, nq = 7, 50_000, 70_000, 4096
    rng = np.random.default_rng(7)
    sizes = rng.integers(0, 3001, nq).astype(np.int64)
    sizes[::97] = 0
    say(f"star batch of {nq} queries, {int(sizes.sum())} rows")
    h = W.host_star_inputs(k, n_prod, n_cust, sizes)
    lt = rng.integers(-5, 106, nq).astype(np.int32)
    start = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    want = [oracle.star_join(h["prod"][a:b], h["cust"][a:b], h["price"], h["category"], h["cust_attr"], lt[q])
            for q, (a, b) in enumerate(zip(start[:-1], start[1:]))]
    ident = skew.StarBatch(to_dev(h["prod"]), to_dev(h["cust"]), to_dev(start), to_dev(lt), to_dev(h["price"]),
                           to_dev(h["category"]), to_dev(h["cust_attr"]))
    Lp = skew.build_skew_layout(ident.prod_keys, n_prod, ident.price, ident.category)
    Lc = skew.build_skew_layout(ident.cust_keys, n_cust, None, ident.segment)
    sk = skew.StarBatch(Lp.fact_recoded, Lc.fact_recoded, ident.query_start, ident.query_cust_lt, Lp.price,
                        Lp.category, Lc.category)
    return dict(identity=ident, skew=sk, want=want)


@pytest.mark.parametrize("tun", [None, (-1, 70_000, 1024, 0), (0, 0, 4096, 2), (-1, 33, 2048, 0)], ids=str)
@pytest.mark.parametrize("layout", ["skew", "identity"])
def test_star_max_queries(many, tun, layout):
    say(f"star 4096 queries {layout} tuning={tun}")
    check(skew.star_join_batch(many[layout], None if tun is None else skew.StarTuning(*tun)), many["want"])

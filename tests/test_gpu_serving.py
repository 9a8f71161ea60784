"""The serving loop on the GPU: continuous batching gives every request the same answer as alone.

Requests arrive at their times and up to six run concurrently on their
slots' streams.  Every request brings its own device output buffers, so its
int64 SUM and COUNT arrays over all 1e5 groups are kept whole: each one is
compared element by element with the same request served alone (one slot)
and with the oracle.  A new table version with re-permuted popularity is
served on the identity layout at once, detected as drift, rebuilt on a side
stream, and served on its own layout afterwards; every answer, before and
after the switch, is compared with the oracle element by element.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1910_10063_amd import serving
from paper_1910_10063_amd import workload as W

pytestmark = pytest.mark.gpu
DEV = "cuda"
M, F = 100_000, 20_000_000


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def version(v, k):
    h = W.host_group_inputs(k, M, F, 1.1)
    return h, serving.TableVersion(v, torch.from_numpy(h["keys"]).to(DEV), torch.from_numpy(h["vals"]).to(DEV), M)


@pytest.fixture(scope="module")
def tables():
    say(f"serving tables M={M} F={F}")
    h1, t1 = version(1, 3)
    h2, t2 = version(2, 13)  # other permutation and rows: popularity re-permuted
    return dict(h1=h1, t1=t1, h2=h2, t2=t2)


def requests(seed):
    arr = serving.poisson_arrivals(200.0, 0.4, seed)
    reqs = serving.make_requests(arr, F, 10_000, 4_000_000, seed)
    for r in reqs[:6]:  # a burst: the first six arrive together, so six slots run them side by side
        r.arrival = reqs[5].arrival
    for r in reqs:  # the request's own outputs, filled with a value no aggregate takes
        r.out = (torch.full((M,), -7, dtype=torch.int64, device=DEV), torch.full((M,), -7, dtype=torch.int64,
                                                                                   device=DEV))
    torch.cuda.synchronize()  # the fills are done before any slot stream writes
    return reqs


def run(tables, slots, versions=None, seed=5):
    t1 = tables["t1"]
    srv = serving.Server(t1, slots, 4_000_000)
    serving.start_layout(srv, t1)
    done = srv.run(requests(seed), versions)
    torch.cuda.synchronize()
    return srv, {r.rid: r for r in done}


def arrays(r):
    return r.out[0].cpu().numpy(), r.out[1].cpu().numpy()


def expected(h, r):
    s, c, inv = oracle.group_aggregate(h["keys"][r.start:r.start + r.rows], h["vals"][r.start:r.start + r.rows], M)
    assert inv == 0
    return s, c


def test_alone_equals_mix_and_oracle(tables):
    say("serving: one slot vs six slots, every request element-wise")
    _, alone = run(tables, 1)
    _, mix = run(tables, 6)
    assert alone.keys() == mix.keys() and len(alone) > 20
    h = tables["h1"]
    for rid in sorted(mix):
        r, a = mix[rid], alone[rid]
        assert r.layout == "skew" and a.layout == "skew"
        ms, mc = arrays(r)
        as_, ac = arrays(a)
        np.testing.assert_array_equal(ms, as_, err_msg=f"request {rid}: SUM alone vs in the mix")
        np.testing.assert_array_equal(mc, ac, err_msg=f"request {rid}: COUNT alone vs in the mix")
        es, ec = expected(h, r)
        np.testing.assert_array_equal(ms, es, err_msg=f"request {rid}: SUM vs oracle")
        np.testing.assert_array_equal(mc, ec, err_msg=f"request {rid}: COUNT vs oracle")
    # overlap: the burst is admitted in one pass of the loop, before any of it is harvested
    rs = sorted(mix.values(), key=lambda r: r.admitted)
    assert any(b.admitted < a.done for a, b in zip(rs, rs[1:]))
    assert all(mix[i].admitted < min(mix[j].done for j in range(6)) for i in range(6))


def test_drift_rebuild_keeps_answers(tables):
    say("serving: new version at 0.2 s, drift detection, rebuild; every request vs the oracle")
    srv, done = run(tables, 4, versions=[(0.2, tables["t2"])], seed=7)
    ev = [e["event"] for e in srv.events]
    assert "version" in ev and "layout_ready" in ev
    chk = [e for e in srv.events if e["event"] == "drift_check"][0]
    assert chk["drift"] and chk["new_share"] < 0.8 * chk["old_share"]
    assert {r.version for r in done.values()} == {1, 2}
    for rid in sorted(done):
        r = done[rid]
        h = tables["h1"] if r.version == 1 else tables["h2"]
        gs, gc = arrays(r)
        es, ec = expected(h, r)
        np.testing.assert_array_equal(gs, es, err_msg=f"request {rid} (version {r.version}, {r.layout}): SUM")
        np.testing.assert_array_equal(gc, ec, err_msg=f"request {rid} (version {r.version}, {r.layout}): COUNT")
    v2 = [r for r in done.values() if r.version == 2]
    assert any(r.layout == "skew" for r in v2)


def test_insert_served_on_the_layout(tables):
    say("serving: rows inserted at 0.2 s, recoded through the current layout; every request vs the oracle")
    n_ins = 3_000_000
    rng = np.random.default_rng(31)
    h1 = tables["h1"]
    pick = rng.integers(0, F, n_ins)
    ins_keys, ins_vals = h1["keys"][pick], rng.integers(0, 1001, n_ins).astype(np.int32)
    batch = serving.InsertBatch(torch.from_numpy(ins_keys).to(DEV), torch.from_numpy(ins_vals).to(DEV))
    t1 = tables["t1"]
    srv = serving.Server(t1, 4, 4_000_000)
    serving.start_layout(srv, t1)
    arr = serving.poisson_arrivals(200.0, 0.4, 9)
    reqs = serving.make_requests(arr, F + n_ins, 10_000, 4_000_000, 9)
    for r in reqs:
        r.out = (torch.full((M,), -7, dtype=torch.int64, device=DEV), torch.full((M,), -7, dtype=torch.int64,
                                                                                   device=DEV))
    torch.cuda.synchronize()
    done = {r.rid: r for r in srv.run(reqs, [(0.2, batch)])}
    torch.cuda.synchronize()
    ev = [e for e in srv.events if e["event"] == "insert"]
    assert len(ev) == 1 and ev[0]["served_on"] == "skew"
    assert not any(e["event"] == "layout_ready" for e in srv.events)  # no rebuild
    keys2 = np.concatenate([h1["keys"], ins_keys])
    vals2 = np.concatenate([h1["vals"], ins_vals])
    assert {r.version for r in done.values()} == {1, 2}
    for rid in sorted(done):
        r = done[rid]
        assert r.layout == "skew"
        kk, vv = (h1["keys"], h1["vals"]) if r.version == 1 else (keys2, vals2)
        es, ec, _ = oracle.group_aggregate(kk[r.start:r.start + r.rows], vv[r.start:r.start + r.rows], M)
        gs, gc = arrays(r)
        np.testing.assert_array_equal(gs, es, err_msg=f"request {rid} (version {r.version}): SUM")
        np.testing.assert_array_equal(gc, ec, err_msg=f"request {rid} (version {r.version}): COUNT")
    assert any(r.version == 2 and r.start + r.rows > F for r in done.values())  # some answer reads inserted rows

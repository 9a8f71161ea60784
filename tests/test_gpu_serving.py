"""The serving loop on the GPU: continuous batching gives every request the same answer as alone.

Requests arrive at their times, up to six run concurrently on their slots'
streams; each result (a digest of the int64 SUM and COUNT of 1e5 groups)
equals the result of the same request served alone, and the oracle's for
sampled requests.  A new table version with re-permuted popularity is served
on the identity layout at once, detected as drift, rebuilt on a side stream,
and served on its own layout afterwards, with unchanged answers.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1910_10063_amd import serving, skew
from paper_1910_10063_amd import workload as W

pytestmark = pytest.mark.gpu
DEV = "cuda"
M, F = 100_000, 20_000_000


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def digest(s, c):
    w0 = np.arange(M, dtype=object) * 2 + 1
    w1 = np.arange(M, dtype=object) + 1

    def wrap(v):
        return ((int(v) + 2**63) % 2**64) - 2**63

    return wrap(sum(s.astype(object) * w0)), wrap(sum(c.astype(object) * w1))


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
    return serving.make_requests(arr, F, 10_000, 4_000_000, seed)


def run(tables, slots, versions=None, seed=5):
    t1 = tables["t1"]
    srv = serving.Server(t1, slots, 4_000_000)
    serving.start_layout(srv, t1)
    done = srv.run(requests(seed), versions)
    return srv, {r.rid: r for r in done}


def test_alone_equals_mix_and_oracle(tables):
    say("serving: one slot vs six slots")
    _, alone = run(tables, 1)
    _, mix = run(tables, 6)
    assert alone.keys() == mix.keys() and len(alone) > 20
    for rid, r in mix.items():
        assert r.digest == alone[rid].digest, rid
        assert r.layout == "skew"
    h = tables["h1"]
    for rid in sorted(alone)[:: max(1, len(alone) // 6)]:
        r = alone[rid]
        s, c, inv = oracle.group_aggregate(h["keys"][r.start:r.start + r.rows], h["vals"][r.start:r.start + r.rows], M)
        assert inv == 0 and digest(s, c) == r.digest, rid
    # overlap: some request was admitted before an earlier one finished
    rs = sorted(mix.values(), key=lambda r: r.admitted)
    assert any(b.admitted < a.done for a, b in zip(rs, rs[1:]))


def test_drift_rebuild_keeps_answers(tables):
    say("serving: new version at 0.2 s, drift detection, rebuild")
    srv, done = run(tables, 4, versions=[(0.2, tables["t2"])], seed=7)
    ev = [e["event"] for e in srv.events]
    assert "version" in ev and "layout_ready" in ev
    chk = [e for e in srv.events if e["event"] == "drift_check"][0]
    assert chk["drift"] and chk["new_share"] < 0.8 * chk["old_share"]
    assert {r.version for r in done.values()} == {1, 2}
    for rid in sorted(done)[::3]:
        r = done[rid]
        h = tables["h1"] if r.version == 1 else tables["h2"]
        s, c, _ = oracle.group_aggregate(h["keys"][r.start:r.start + r.rows], h["vals"][r.start:r.start + r.rows], M)
        assert digest(s, c) == r.digest, (rid, r.version, r.layout)
    v2 = [r for r in done.values() if r.version == 2]
    assert any(r.layout == "skew" for r in v2)

"""Host logic of the serving loop (no GPU): arrivals, request ranges, slot planning."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1910_10063_amd import serving  # noqa: E402


def test_poisson_rate_and_order():
    t = serving.poisson_arrivals(200.0, 50.0, 3)
    assert (np.diff(t) > 0).all() and t[0] >= 0 and t[-1] < 50.0
    # count in 50 s is Poisson(10000): within 5 standard deviations
    assert abs(t.size - 10000) < 5 * 100
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 200) < 5 * (1 / 200) / np.sqrt(gaps.size)


def test_requests_in_range_and_log_uniform():
    arr = np.linspace(0, 1, 4000, endpoint=False)
    reqs = serving.make_requests(arr, 10_000_000, 1000, 1_000_000, 9)
    n = np.array([r.rows for r in reqs])
    s = np.array([r.start for r in reqs])
    assert (n >= 1000).all() and (n <= 1_000_000).all()
    assert (s >= 0).all() and (s + n <= 10_000_000).all()
    # log-uniform: log10 of the sizes is uniform on [3, 6]
    l = np.log10(n)
    assert abs(l.mean() - 4.5) < 0.05 and abs(np.median(l) - 4.5) < 0.08
    assert [r.rid for r in reqs] == list(range(4000))


def test_plan_slots_respects_budget():
    per = serving.slot_bytes(1 << 22, 100_000)
    assert serving.plan_slots(per * 5 + 7, 1 << 22, 100_000) == 5
    assert serving.plan_slots(0, 1 << 22, 100_000) == 1
    assert serving.plan_slots(per * 1000, 1 << 22, 100_000, max_slots=16) == 16


def test_latency_report():
    reqs = [serving.Request(i, 0.001 * i, 0, 100 + i) for i in range(100)]
    for r in reqs:
        r.admitted = r.arrival
        r.done = r.arrival + 0.002 + (0.01 if r.rid == 99 else 0.0)
        r.layout = "skew" if r.rid % 2 else "identity"
    rep = serving.latency_report(reqs)
    assert abs(rep["p50_ms"] - 2.0) < 1e-9 and rep["p99_ms"] >= 2.0
    assert rep["served_on_skew"] == 50 and rep["rows"] == sum(100 + i for i in range(100))


def test_latency_report_counts_requests_in_flight():
    # A runs over [0, 4), B over [1, 2) inside it, C from 4, when A ends (eighths of a second: exact floats)
    reqs = [serving.Request(i, a / 8, 0, 10) for i, a in enumerate((0, 1, 4))]
    for r, (a, d) in zip(reqs, ((0, 4), (1, 2), (4, 5))):
        r.admitted, r.done, r.layout = a / 8, d / 8, "skew"
    rep = serving.latency_report(reqs)
    assert rep["max_in_flight"] == 2 and rep["admitted_while_another_ran"] == 1

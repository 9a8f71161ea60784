"""Serving loop for grouped aggregation on device-resident tables, with continuous batching.

Requests arrive over time.  Each asks for SUM(value) and COUNT(*) per group over a range of rows of the
resident fact table (the grouped aggregation Q3 of Section 1).  The server works as follows:

* It keeps the tables on the device.
* It owns execution slots, as many as a memory budget allows.  Each slot has its own HIP stream, its own
  workspace and its own output buffers.
* It admits a waiting request as soon as a slot is free.  Admitted requests run concurrently on their
  slots' streams, so work from requests that arrived at different times overlaps on the GPU: continuous
  batching, not a queue in front of one stream.
* It maintains the frequency-ordered layout (built as in Section 3.1, rebuilt after a batch of updates, as
  the maintenance discussion there suggests).  A new version of the table, with re-permuted key
  popularity, is served at once on the identity layout with the library's layout-oblivious method, which
  gives the same answers.
* Rows inserted into the table are recoded through the current layout and served on it at once (the
  maintenance rule of Section 3.1); their frequencies are not counted.
* It watches the share of rows that the current layout sends to its hot prefix.  When that share drops
  (drift), it rebuilds the layout on a side stream and switches to the rebuilt layout when it is ready.

Every step of every request runs in the library's HIP kernels (paper_1910_10063_amd.skew).  This module
schedules, and it measures latency with wall-clock times at arrival and at completion.  A request may bring
its own device output buffers; the aggregation then writes its result there and nothing is copied.
"""
from __future__ import annotations

import math
import threading
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import skew


@dataclass
class Request:
    rid: int
    arrival: float  # seconds since the start of the run
    start: int      # first row of the range
    rows: int       # rows in the range
    version: int = -1       # table version it was answered on
    layout: str = ""        # "skew" or "identity"
    admitted: float = math.nan
    done: float = math.nan
    # int64 SUM and COUNT outputs [n_groups] on the device, written by the request's aggregation; None: the
    # slot's own buffers, overwritten by the slot's next request
    out: tuple[torch.Tensor, torch.Tensor] | None = None


@dataclass
class TableVersion:
    """One version of the resident fact table and, once built, its frequency-ordered layout."""

    version: int
    keys: torch.Tensor      # int32 group ids (identity layout)
    vals: torch.Tensor      # int32 values
    n_groups: int
    layout: skew.Layout | None = None
    hot_share: float = math.nan  # share of rows below the hot threshold on its own layout


@dataclass
class InsertBatch:
    """Fact rows inserted into the current table version (appended at its end)."""

    keys: torch.Tensor  # int32 group ids (identity layout)
    vals: torch.Tensor  # int32 values


@dataclass
class Slot:
    stream: torch.cuda.Stream
    ws: torch.Tensor
    out: tuple[torch.Tensor, torch.Tensor]
    done: torch.cuda.Event
    req: Request | None = None


def slot_bytes(max_rows: int, n_groups: int) -> int:
    """Device bytes one execution slot holds: workspace of the partitioned aggregate plus outputs."""
    return skew.workspace_bytes(skew.SKEW_OP_GROUP, max_rows, n_groups) + 16 * n_groups + 16


def plan_slots(memory_budget: int, max_rows: int, n_groups: int, max_slots: int = 16) -> int:
    """Number of slots a memory budget admits (at least one)."""
    return max(1, min(max_slots, memory_budget // slot_bytes(max_rows, n_groups)))


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process of `rate` per second over [0, duration)."""
    rng = np.random.default_rng(seed)
    n = int(rate * duration * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    return t[t < duration]


def make_requests(arrivals: np.ndarray, table_rows: int, min_rows: int, max_rows: int, seed: int) -> list[Request]:
    """Row ranges of log-uniform length in [min_rows, max_rows] at uniform positions."""
    rng = np.random.default_rng(seed + 1)
    out = []
    for i, a in enumerate(arrivals):
        n = int(min_rows * (max_rows / min_rows) ** rng.random())
        n = min(n, table_rows)
        s = int(rng.integers(0, table_rows - n + 1))
        out.append(Request(i, float(a), s, n))
    return out


def start_layout(server: "Server", table: TableVersion) -> None:
    """Build the first layout synchronously and serve it (before a run)."""
    server.build_layout(table, torch.cuda.current_stream(server.device))
    torch.cuda.synchronize(server.device)
    server.measure_hot_share(table)
    server.serving_layout = table
    server.current = table


class Server:
    """Continuous-batching executor of grouped aggregations over a resident, versioned table."""

    def __init__(self, table: TableVersion, n_slots: int, max_rows: int, drift_ratio: float = 0.8,
                 sample_rows: int = 1 << 22, device="cuda"):
        self.device = torch.device(device)
        self.n_groups = table.n_groups
        self.max_rows = max_rows
        self.drift_ratio = drift_ratio
        self.sample_rows = sample_rows
        self.slots = []
        for _ in range(n_slots):
            ws = skew.workspace(skew.SKEW_OP_GROUP, max_rows, self.n_groups, self.device)
            out = (torch.empty(self.n_groups, dtype=torch.int64, device=self.device),
                   torch.empty(self.n_groups, dtype=torch.int64, device=self.device))
            self.slots.append(Slot(torch.cuda.Stream(self.device), ws, out, torch.cuda.Event(enable_timing=False)))
        self.side = torch.cuda.Stream(self.device)  # layout rebuilds
        self.build_ws = None
        self.current = table
        self.serving_layout: TableVersion | None = None  # the version whose layout queries use
        self.rebuild: dict | None = None
        self.events: list[dict] = []
        self.t0 = time.perf_counter()

    # ---- time
    def now(self) -> float:
        return time.perf_counter() - self.t0

    # ---- layout maintenance
    def build_layout(self, table: TableVersion, stream) -> None:
        """Frequency-ordered layout of `table` on `stream` (Section 3.1).  The build workspace and the layout's
        arrays are allocated on `stream`, the stream that uses them."""
        n = table.keys.numel()
        need = skew.workspace_bytes(skew.SKEW_OP_BUILD, n, self.n_groups)
        with torch.cuda.stream(stream):
            if self.build_ws is None or self.build_ws.numel() < need:
                self.build_ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            table.layout = skew.build_skew_layout(table.keys, self.n_groups, ws=self.build_ws)

    def measure_hot_share(self, table: TableVersion) -> None:
        """Share of the table's rows that its own layout sends to the hot prefix (after its build): the
        frequencies of the hot ranks, copied to the host and added there."""
        t = min(skew.max_hot_groups(), self.n_groups)
        cnt = table.layout.counts_by_rank[:t].cpu().numpy().astype(np.uint32).astype(np.int64)
        table.hot_share = float(cnt.sum()) / max(table.keys.numel(), 1)

    def hot_share_under(self, layout_table: TableVersion, table: TableVersion) -> float:
        """Share of a sample of `table`'s rows whose rank under layout_table's layout is below the hot
        threshold: selection (Q2) of the rows with rank[key] < t."""
        t = min(skew.max_hot_groups(), self.n_groups)
        n = min(self.sample_rows, table.keys.numel())
        _, cnt = skew.select_fact_rows(table.keys[:n], layout_table.layout.rank, t)
        return float(cnt.item()) / max(n, 1)

    def install(self, table: TableVersion, rebuild: bool = True) -> None:
        """A new version of the table arrives: serve it on the identity layout at once; rebuild if drifted."""
        old = self.serving_layout
        self.current = table
        self.events.append({"t": self.now(), "event": "version", "version": table.version})
        if not rebuild:
            return
        drift = True
        if old is not None and old.layout is not None:
            share = self.hot_share_under(old, table)
            drift = share < self.drift_ratio * old.hot_share
            self.events.append({"t": self.now(), "event": "drift_check", "old_share": old.hot_share,
                                "new_share": share, "drift": drift})
        if drift:
            # The build waits for its histogram (a range check) before it enqueues the rest, so it is issued
            # from a worker thread: admission and harvesting go on meanwhile.
            r = {"table": table, "event": torch.cuda.Event(enable_timing=True),
                 "start": torch.cuda.Event(enable_timing=True), "t": self.now(), "error": None}

            def work():
                try:
                    r["start"].record(self.side)
                    self.build_layout(table, self.side)
                    r["event"].record(self.side)
                except Exception as e:  # reported by poll_rebuild on the serving thread
                    r["error"] = e

            r["thread"] = threading.Thread(target=work, daemon=True)
            r["thread"].start()
            self.rebuild = r

    def insert(self, batch: InsertBatch) -> TableVersion:
        """Rows inserted into the table (Section 3.1, maintenance): the next version is the current one with the
        rows appended.  When the current version is served on its own layout, the new rows are recoded through that
        layout and the next version is served on it at once, with no rebuild; the new rows' frequencies are not
        counted, and drift detection decides later whether a rebuild pays."""
        old = self.current
        t0 = self.now()
        tab = TableVersion(old.version + 1, torch.cat([old.keys, batch.keys]), torch.cat([old.vals, batch.vals]),
                           old.n_groups)
        if self.serving_layout is old and old.layout is not None:
            layout, rec = skew.append_skew_layout(old.layout, old.n_groups, fact_keys_new=batch.keys)
            layout.fact_recoded = torch.cat([old.layout.fact_recoded, rec])
            tab.layout = layout
            tab.hot_share = old.hot_share
            self.serving_layout = tab
        self.current = tab
        torch.cuda.current_stream(self.device).synchronize()  # the new version is complete before it is served
        self.events.append({"t": t0, "event": "insert", "version": tab.version, "rows": batch.keys.numel(),
                            "served_on": "skew" if tab.layout is not None else "identity",
                            "ms": (self.now() - t0) * 1e3})
        return tab

    def poll_rebuild(self) -> None:
        r = self.rebuild
        if r is None or r["thread"].is_alive():
            return
        if r["error"] is not None:
            self.rebuild = None
            raise r["error"]
        if r["event"].query():
            self.measure_hot_share(r["table"])
            self.serving_layout = r["table"]
            self.events.append({"t": self.now(), "event": "layout_ready", "version": r["table"].version,
                                "rebuild_ms": r["start"].elapsed_time(r["event"]),
                                "hot_share": r["table"].hot_share})
            self.rebuild = None

    # ---- requests
    def launch(self, slot: Slot, req: Request) -> None:
        tab = self.current
        use_skew = self.serving_layout is tab and tab.layout is not None
        req.version = tab.version
        req.layout = "skew" if use_skew else "identity"
        req.admitted = self.now()
        req.rows = max(0, min(req.rows, tab.keys.numel() - req.start))
        a, n = req.start, req.rows
        out = req.out if req.out is not None else slot.out
        with torch.cuda.stream(slot.stream):
            if use_skew:
                skew.group_aggregate(tab.layout.fact_recoded[a:a + n], tab.vals[a:a + n], self.n_groups,
                                     hot_groups=skew.SKEW_HOT_AUTO, perm=tab.layout.perm, ws=slot.ws, out=out)
            else:
                skew.group_aggregate(tab.keys[a:a + n], tab.vals[a:a + n], self.n_groups, hot_groups=0,
                                     ws=slot.ws, out=out)
            slot.done.record(slot.stream)
        slot.req = req

    def harvest(self, slot: Slot) -> Request:
        """The slot's stream has passed its done event: the request's outputs are complete."""
        req = slot.req
        req.done = self.now()
        slot.req = None
        return req

    def run(self, requests: list[Request], versions: list[tuple[float, TableVersion | InsertBatch]] | None = None,
            idle_sleep: float = 0.0) -> list[Request]:
        """Serve `requests` at their arrival times (seconds from now); install table versions (or insert rows) at
        their times.  A request's row range is clipped to the rows of the version it is answered on."""
        versions = sorted(versions or [], key=lambda v: v[0])
        pending: list[Request] = []
        finished: list[Request] = []
        i = vi = 0
        self.t0 = time.perf_counter()
        while len(finished) < len(requests):
            now = self.now()
            while vi < len(versions) and versions[vi][0] <= now:
                if isinstance(versions[vi][1], InsertBatch):
                    self.insert(versions[vi][1])
                else:
                    self.install(versions[vi][1])
                vi += 1
            while i < len(requests) and requests[i].arrival <= now:
                pending.append(requests[i])
                i += 1
            self.poll_rebuild()
            for slot in self.slots:
                if slot.req is not None and slot.done.query():
                    finished.append(self.harvest(slot))
            for slot in self.slots:  # admit in arrival order into every free slot
                if slot.req is None and pending:
                    self.launch(slot, pending.pop(0))
            if idle_sleep and not pending:
                time.sleep(idle_sleep)
        torch.cuda.synchronize(self.device)
        if self.rebuild is not None:
            self.rebuild["thread"].join()
            torch.cuda.synchronize(self.device)
        self.poll_rebuild()
        return finished


def latency_report(done: list[Request]) -> dict:
    lat = np.array([r.done - r.arrival for r in done]) * 1e3
    rows = sum(r.rows for r in done)
    span = max(r.done for r in done) - min(r.arrival for r in done)
    # requests in flight at once (admitted, not yet harvested), and how many were admitted while another one ran
    ev = sorted([(r.admitted, 1) for r in done] + [(r.done, -1) for r in done], key=lambda e: (e[0], e[1]))
    depth = peak = 0
    overlapped = 0
    for _, d in ev:
        if d > 0 and depth > 0:
            overlapped += 1
        depth += d
        peak = max(peak, depth)
    return {"requests": len(done), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "rows": int(rows), "tuples_per_s": rows / span if span > 0 else 0.0,
            "served_on_skew": sum(r.layout == "skew" for r in done),
            "served_on_identity": sum(r.layout == "identity" for r in done),
            "max_in_flight": peak, "admitted_while_another_ran": overlapped}

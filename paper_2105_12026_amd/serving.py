"""Serving driver: feeds a stream of summarisation requests to the serving
core (``ebc.Server``: continuous batching at greedy-step granularity with
admission by device footprint) and accounts latency from arrival to the
result on the host.

The driver only schedules submissions and ticks; every step of the
computation runs in the library's kernels. It works with any object that
has the server's methods (``submit``, ``step``, ``poll``, ``stats``,
``now``), so its accounting can be checked on a virtual clock.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

__all__ = ["Record", "run_open_loop", "run_closed_loop", "summarize"]


@dataclass
class Record:
    index: int          # position in the request stream
    rid: int
    n: int
    k: int
    t_arrive: float
    t_admit: float
    t_done: float
    state: str

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive

    @property
    def wait(self) -> float:
        return self.t_admit - self.t_arrive


def _unpack(payload, dtype):
    """A payload is (x, k) or (x, k, dtype)."""
    if len(payload) == 3:
        return payload
    return payload[0], payload[1], dtype


def _collect(server, pending: dict, records: list, results: dict | None = None):
    for rid in list(pending):
        r = server.poll(rid)
        if r["state"] in ("done", "failed"):
            i, n, k = pending.pop(rid)
            records.append(Record(i, rid, n, k, r["t_arrive"], r["t_admit"], r["t_done"], r["state"]))
            if results is not None:
                results[i] = r


def run_open_loop(server, payloads, arrivals, dtype: str = "bf16", sleep=time.sleep, results: dict | None = None,
                  progress=None, progress_every: int = 250):
    """Open-loop stream: request i = payloads[i] = (x, k[, dtype]) arrives at
    ``arrivals[i]`` seconds after the start and is submitted, stamped with
    that arrival time, as soon as the driver reaches it; the server is ticked
    while it holds work, and the driver sleeps until the next arrival when it
    is idle. Returns the records (one per request, completion order) and the
    start time on the server clock. ``results`` (optional) receives each
    finished request's poll() output, keyed by stream index; ``progress``
    (optional) is called with (finished, total) every ``progress_every``
    finished requests."""
    arrivals = np.asarray(arrivals, dtype=np.float64)
    if len(arrivals) != len(payloads):
        raise ValueError("one arrival time per request")
    t0 = server.now()
    i, count = 0, len(payloads)
    pending: dict = {}
    records: list[Record] = []
    while i < count or pending:
        now = server.now()
        while i < count and t0 + arrivals[i] <= now:
            x, k, dt = _unpack(payloads[i], dtype)
            rid = server.submit(x, k, dt, t_arrival=t0 + arrivals[i])
            pending[rid] = (i, int(x.shape[0]), int(k))
            i += 1
        st = server.stats()
        if st["queued"] + st["active"] == 0:
            if pending:  # finished during the last tick but not collected yet
                _collect(server, pending, records, results)
                continue
            if i < count:
                sleep(max(0.0, t0 + arrivals[i] - server.now()))
            continue
        if server.step() > 0:
            before = len(records)
            _collect(server, pending, records, results)
            if progress and len(records) // progress_every > before // progress_every:
                progress(len(records), count)
    return records, t0


def run_closed_loop(server, payloads, dtype: str = "bf16", results: dict | None = None):
    """All requests submitted at once; the server runs until every one has
    finished. Returns (records, t0, t_end): the capacity is
    len(payloads) / (t_end - t0) requests per second."""
    t0 = server.now()
    pending = {}
    for i, p in enumerate(payloads):
        x, k, dt = _unpack(p, dtype)
        rid = server.submit(x, k, dt, t_arrival=t0)
        pending[rid] = (i, int(x.shape[0]), int(k))
    records: list[Record] = []
    while pending:
        if server.step() > 0:
            _collect(server, pending, records, results)
        else:
            st = server.stats()
            if st["queued"] + st["active"] == 0:  # only failed requests remain uncollected
                _collect(server, pending, records, results)
    return records, t0, server.now()


def summarize(records, t0: float) -> dict:
    """p50/p99 latency (arrival -> result on the host), queueing wait,
    completed requests per second over the span from t0 to the last
    completion, and the failure count."""
    ok = [r for r in records if r.state == "done"]
    if not ok:
        return {"completed": 0, "failed": len(records)}
    lat = np.array([r.latency for r in ok])
    wait = np.array([r.wait for r in ok])
    span = max(r.t_done for r in ok) - t0
    return {
        "completed": len(ok),
        "failed": len(records) - len(ok),
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()),
        "max_s": float(lat.max()),
        "wait_p50_s": float(np.percentile(wait, 50)),
        "wait_p99_s": float(np.percentile(wait, 99)),
        "req_per_s": len(ok) / span if span > 0 else float("inf"),
        "span_s": span,
    }

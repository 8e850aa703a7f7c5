"""Host-side parts of the serving core, on the CPU: the first-fit arena
allocator against a brute-force interval model, the request footprint, the
Poisson arrival generator, and the serving driver's latency accounting on a
virtual clock with a mock executor (which runs the oracle instead of the
device; the driver cannot tell the difference)."""
import numpy as np
import pytest

from paper_2105_12026_amd import serving
from paper_2105_12026_amd import workloads as W


@pytest.fixture(scope="module")
def ebc():
    from paper_2105_12026_amd import ebc as mod
    return mod


def _first_fit(used: dict, cap: int, size: int):
    """Lowest offset where a block of `size` fits between the used blocks."""
    pos = 0
    for off in sorted(used):
        if off - pos >= size:
            return pos
        pos = max(pos, off + used[off])
    return pos if cap - pos >= size else None


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_arena_matches_first_fit_model(ebc, seed):
    rng = np.random.default_rng(seed)
    cap = 1 << 20
    a = ebc.Arena(cap)
    used = {}
    for _ in range(600):
        if used and rng.random() < 0.45:
            off = list(used)[rng.integers(len(used))]
            a.free(off)
            del used[off]
        else:
            req = int(rng.integers(1, 90_000))
            size = (req + 255) // 256 * 256
            want = _first_fit(used, cap, size)
            got = a.alloc(req)
            assert got == want
            if got is not None:
                assert got % 256 == 0 and got + size <= cap
                used[got] = size
        assert a.free_bytes == cap - sum(used.values())
        gaps, pos = [], 0
        for off in sorted(used):
            gaps.append(off - pos)
            pos = off + used[off]
        gaps.append(cap - pos)
        assert a.largest_free == max(gaps)
    for off in list(used):
        a.free(off)
    assert a.free_bytes == cap and a.largest_free == cap  # fully coalesced


def test_arena_errors(ebc):
    a = ebc.Arena(4096)
    assert a.alloc(0) == 0  # rounds up to one 256-byte unit
    assert a.alloc(4096) is None
    with pytest.raises(ebc.EBCError):
        a.free(12345)
    a.free(0)
    with pytest.raises(ebc.EBCError):
        a.free(0)  # double free
    with pytest.raises(ebc.EBCError):
        ebc.Arena(0)


def test_request_bytes(ebc):
    base = ebc.request_bytes(10_000, 64, 10, "bf16")
    assert base > 10_000 * 64 * 4
    assert ebc.request_bytes(20_000, 64, 10, "bf16") > base
    assert ebc.request_bytes(10_000, 64, 50, "bf16") > base
    # float32: the caller's points plus the padded float32 copy; bf16: the points
    # plus the cast copy in row order and in grouped order (10240 padded rows)
    assert ebc.request_bytes(10_000, 64, 10, "f32") > 2 * 10_000 * 64 * 4
    assert base > 10_000 * 64 * 4 + 2 * 10_240 * 64 * 2
    assert ebc.request_bytes(10, 64, 11, "bf16") == 0       # k > n
    assert ebc.request_bytes(10, 4097, 5, "bf16") == 0      # d beyond the supported maximum
    assert ebc.request_bytes(1000, 3524, 5, "bf16") > 1000 * 3524 * 4
    assert base % 256 == 0


def test_poisson_arrivals():
    a = W.poisson_arrivals(5, 50.0, 20000)
    assert np.all(np.diff(a) > 0)
    gaps = np.diff(np.concatenate([[0.0], a]))
    assert abs(gaps.mean() - 1 / 50.0) < 0.03 / 50.0 * 5
    assert np.array_equal(a, W.poisson_arrivals(5, 50.0, 20000))
    with pytest.raises(ValueError):
        W.poisson_arrivals(5, 0.0, 3)


class MockServer:
    """The serving core's scheduling on a virtual clock: FIFO admission while
    a slot is free, one greedy step per tick for every active request, each
    tick costing `tick_s` of virtual time; results come from the oracle."""

    def __init__(self, slots, tick_s):
        self.slots, self.tick_s, self.t = slots, tick_s, 0.0
        self.queue, self.active, self.req, self.next = [], [], {}, 1
        self.ticks = 0

    def now(self):
        return self.t

    def sleep(self, dt):
        assert dt >= 0
        self.t += dt

    def submit(self, x, k, dtype, t_arrival=-1.0):
        rid = self.next
        self.next += 1
        self.req[rid] = {"x": x, "k": k, "t": 0, "state": "queued", "t_arrive": t_arrival if t_arrival >= 0 else self.t,
                         "t_admit": 0.0, "t_done": 0.0}
        self.queue.append(rid)
        return rid

    def stats(self):
        return {"queued": len(self.queue), "active": len(self.active), "ticks": self.ticks}

    def step(self):
        from oracle import ebc_oracle as O
        while self.queue and len(self.active) < self.slots:
            rid = self.queue.pop(0)
            self.req[rid].update(state="active", t_admit=self.t)
            self.active.append(rid)
        if not self.active:
            return 0
        self.t += self.tick_s
        self.ticks += 1
        done = []
        for rid in self.active:
            r = self.req[rid]
            r["t"] += 1
            if r["t"] == r["k"]:
                sel, f, g = O.greedy(r["x"], r["k"])
                r.update(state="done", t_done=self.t, sel=sel, f=f, gain=g)
                done.append(rid)
        self.active = [r for r in self.active if r not in done]
        return len(done)

    def poll(self, rid):
        r = self.req[rid]
        return {k: r[k] for k in ("state", "t_arrive", "t_admit", "t_done", "sel", "f", "gain") if k in r}


def test_driver_latency_on_virtual_clock():
    x = np.random.default_rng(3).standard_normal((12, 3)).astype(np.float32)
    sv = MockServer(slots=1, tick_s=1.0)
    # request 0 at t=0 (k=2), request 1 at t=0.5 (k=1) waits for the slot,
    # request 2 at t=10 arrives to an idle server (the driver sleeps until then)
    payloads = [(x, 2), (x, 1), (x, 3)]
    arrivals = [0.0, 0.5, 10.0]
    results = {}
    recs, t0 = serving.run_open_loop(sv, payloads, arrivals, sleep=sv.sleep, results=results)
    by = {r.index: r for r in recs}
    assert t0 == 0.0
    assert (by[0].t_admit, by[0].t_done) == (0.0, 2.0)
    assert (by[1].t_arrive, by[1].t_admit, by[1].t_done) == (0.5, 2.0, 3.0)
    assert (by[2].t_arrive, by[2].t_admit, by[2].t_done) == (10.0, 10.0, 13.0)
    assert [r.latency for r in sorted(recs, key=lambda r: r.index)] == [2.0, 2.5, 3.0]
    s = serving.summarize(recs, t0)
    assert s["completed"] == 3 and s["failed"] == 0
    assert s["p50_s"] == 2.5 and abs(s["p99_s"] - (2.5 + 0.98 * 0.5)) < 1e-12
    assert s["req_per_s"] == 3 / 13.0
    from oracle import ebc_oracle as O
    sel, f, _ = O.greedy(x, 3)
    assert results[2]["sel"].tolist() == sel.tolist()


def test_closed_loop_capacity_on_virtual_clock():
    x = np.random.default_rng(4).standard_normal((10, 2)).astype(np.float32)
    sv = MockServer(slots=2, tick_s=0.25)
    recs, t0, t1 = serving.run_closed_loop(sv, [(x, 2)] * 5)
    # two at a time, 2 ticks each: pairs finish at 0.5, 1.0, then the last at 1.5
    assert sorted(r.t_done for r in recs) == [0.5, 0.5, 1.0, 1.0, 1.5]
    assert t1 - t0 == 1.5
    assert serving.summarize(recs, t0)["req_per_s"] == 5 / 1.5

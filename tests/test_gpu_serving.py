"""Serving core (continuous batching at greedy-step granularity, admission
by device footprint): every request's result equals its solo ebc_greedy run
bitwise, whatever the mix (short and long rows), the arrival pattern, the slot
count or the arena budget; the arena is never oversubscribed; the float32 requests also match
the oracle."""
import numpy as np
import pytest

from paper_2105_12026_amd import workloads as W

pytestmark = pytest.mark.gpu

# (n, d, dtype, k)
REQS = [(3000, 64, "bf16", 7), (700, 64, "f32", 4), (5000, 64, "bf16", 12), (1200, 16, "fp8", 3),
        (2600, 64, "f16", 9), (4100, 100, "f32", 6), (257, 64, "bf16", 1), (1800, 64, "bf16", 10),
        (900, 300, "f32", 5), (600, 520, "bf16", 4)]  # the last two: long rows


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2105_12026_amd import ebc
    assert torch.cuda.is_available()
    return torch, ebc


def _x(spec, i):
    n, d = spec[0], spec[1]
    return W.gaussian_mixture(np.random.default_rng([61, i]), n, d, 5).astype(np.float32)


@pytest.fixture(scope="module")
def solos(env):
    torch, ebc = env
    out = []
    for i, spec in enumerate(REQS):
        x = _x(spec, i)
        ds = ebc.Dataset(torch.from_numpy(x).cuda(), dtype=spec[2])
        res = [t.cpu().numpy() for t in ds.greedy(spec[3])]
        ds.sync()
        out.append((x, res))
    return out


def _check(results, solos, order):
    for j, i in enumerate(order):
        r = results[j]
        assert r["state"] == "done", (i, r)
        x, (sel, f, g) = solos[i]
        np.testing.assert_array_equal(r["sel"], sel, err_msg=str(REQS[i]))
        np.testing.assert_array_equal(r["f"], f, err_msg=str(REQS[i]))
        np.testing.assert_array_equal(r["gain"], g, err_msg=str(REQS[i]))


def _footprint(ebc, i):
    n, d, dt, k = REQS[i]
    return ebc.request_bytes(n, d, k, dt)


def test_all_at_once_equals_solo(env, solos, ref):
    torch, ebc = env
    from paper_2105_12026_amd import serving
    print(f"[gpu-case] serving: {len(REQS)} requests at once", flush=True)
    sv = ebc.Server(256 << 20, max_slots=16)
    free0 = sv.stats()["free_bytes"]
    results = {}
    payloads = [(solos[i][0], REQS[i][3], REQS[i][2]) for i in range(len(REQS))]
    recs, t0, t1 = serving.run_closed_loop(sv, payloads, results=results)
    assert len(recs) == len(REQS) and t1 > t0
    _check([results[i] for i in range(len(REQS))], solos, range(len(REQS)))
    st = sv.stats()
    assert st["active"] == 0 and st["queued"] == 0 and st["ticks"] == max(s[3] for s in REQS)
    assert st["free_bytes"] == free0
    for i, spec in enumerate(REQS):
        if spec[2] == "f32":
            rsel, rf, _ = ref.greedy(solos[i][0], spec[3])
            assert solos[i][1][0].tolist() == rsel.tolist()
            np.testing.assert_allclose(solos[i][1][1], rf, rtol=1e-5)
    sv.close()


def test_staggered_arrivals_equal_solo(env, solos):
    """Requests join while others are mid-run (different steps in one tick)."""
    torch, ebc = env
    print("[gpu-case] serving: staggered arrivals", flush=True)
    sv = ebc.Server(256 << 20, max_slots=8)
    ids = {}
    order = [2, 0, 8, 5, 7, 1, 9, 4, 3, 6]
    for tick in range(40):
        if tick < len(order):
            i = order[tick]
            ids[i] = sv.submit(solos[i][0], REQS[i][3], REQS[i][2])
        sv.step()
        if tick >= len(order) and sv.stats()["completed"] == len(REQS):
            break
    assert sv.stats()["completed"] == len(REQS)
    _check([sv.poll(ids[i]) for i in range(len(REQS))], solos, range(len(REQS)))
    sv.close()


@pytest.mark.parametrize("slots", [1, 3])
def test_small_budget_never_oversubscribes(env, solos, slots):
    """An arena that holds only about two requests: the rest queue, admission
    follows arrival order, the arena is never oversubscribed, and every
    result still equals its solo run."""
    torch, ebc = env
    print(f"[gpu-case] serving: small budget, slots={slots}", flush=True)
    sizes = [_footprint(ebc, i) for i in range(len(REQS))]
    tables = 64 << 10
    budget = tables + sorted(sizes)[-1] + sorted(sizes)[-2] + 4096
    sv = ebc.Server(budget, max_slots=slots)
    free0 = sv.stats()["free_bytes"]
    ids = [sv.submit(solos[i][0], REQS[i][3], REQS[i][2]) for i in range(len(REQS))]
    max_active = 0
    admitted_order = []
    seen = set()
    for _ in range(400):
        sv.step()
        st = sv.stats()
        assert st["active"] <= slots
        active = [j for j, r in enumerate(ids) if sv.poll(r)["state"] == "active"]
        used = sum((sizes[j] + 255) // 256 * 256 for j in active)
        assert used <= free0
        assert free0 - st["free_bytes"] == used
        for j in active:
            if j not in seen:
                seen.add(j)
                admitted_order.append(j)
        max_active = max(max_active, st["active"])
        if st["completed"] == len(REQS):
            break
    assert sv.stats()["completed"] == len(REQS)
    assert sv.stats()["free_bytes"] == free0
    # first come, first served: admission order is the submission order
    admits = [sv.poll(r)["t_admit"] for r in ids]
    assert admits == sorted(admits)
    _check([sv.poll(r) for r in ids], solos, range(len(REQS)))
    sv.close()


def test_oversized_request_is_refused(env):
    torch, ebc = env
    sv = ebc.Server(4 << 20, max_slots=4)
    x = np.zeros((20000, 64), np.float32)
    with pytest.raises(ebc.EBCError) as ei:
        sv.submit(x, 5, "bf16")
    assert ei.value.code == 5
    with pytest.raises(ebc.EBCError):
        sv.submit(x[:10], 11, "bf16")  # k > n
    sv.close()


def test_open_loop_driver_accounts_latency(env, solos):
    torch, ebc = env
    from paper_2105_12026_amd import serving
    print("[gpu-case] serving: open-loop driver", flush=True)
    sv = ebc.Server(256 << 20, max_slots=8)
    idx = [0, 2, 6, 7, 0, 2]
    payloads = [(solos[i][0], REQS[i][3]) for i in idx]
    arrivals = W.poisson_arrivals(5, 200.0, len(payloads))
    results = {}
    recs, t0 = serving.run_open_loop(sv, payloads, arrivals, dtype="bf16", results=results)
    assert len(recs) == len(payloads)
    for r in recs:
        assert r.state == "done"
        assert r.t_arrive <= r.t_admit <= r.t_done
        assert abs(r.t_arrive - (t0 + arrivals[r.index])) < 1e-9
    for j, i in enumerate(idx):
        np.testing.assert_array_equal(results[j]["sel"], solos[i][1][0])
        np.testing.assert_array_equal(results[j]["f"], solos[i][1][1])
    s = serving.summarize(recs, t0)
    assert s["completed"] == len(payloads) and s["p99_s"] >= s["p50_s"] > 0
    sv.close()

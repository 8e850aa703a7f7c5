"""Batched greedy (many instances, one launch per kernel bucket and stage per
tick) against solo runs: selections, f and gains bitwise equal, for a mix of
sizes, dimensions (short and long rows), distance dtypes, tile variants and k
(including k = 0), eager and graph mode; the float32 instances also against
the oracle. A sample of the 512-instance batched workload (its first 32
instances, k = 20) against the stored float64 oracle runs: FP32 selections
identical, BF16 quality gap at most 1e-3 with f exact for the chosen sets."""
import json
import os

import numpy as np
import pytest

from paper_2105_12026_amd import workloads as W

pytestmark = pytest.mark.gpu

# (n, d, dtype, variant, k)
MIX = [(300, 16, "f32", 0, 5), (1000, 100, "bf16", 0, 7), (2500, 64, "bf16", 2, 12), (700, 5, "fp8", 0, 3),
       (1500, 33, "f16", 1, 0), (4000, 128, "f32", 0, 9), (257, 64, "bf16", 0, 4), (2049, 64, "fp8", 2, 6),
       (3100, 64, "bf16", 3, 8), (1800, 128, "fp8", 3, 5), (2300, 112, "f16", 3, 6),
       # float32 rows whose last 4 padded slots are empty (shortened last K step)
       (1300, 100, "f32", 0, 6), (800, 3, "f32", 0, 4),
       # long rows (padded length above 128)
       (1000, 300, "f32", 0, 6), (900, 200, "bf16", 1, 5), (500, 520, "fp8", 0, 4)]


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2105_12026_amd import ebc
    assert torch.cuda.is_available()
    return torch, ebc


def _make(env, spec, seed):
    torch, ebc = env
    n, d, dt, var, k = spec
    x = W.gaussian_mixture(np.random.default_rng(seed), n, d, 6).astype(np.float32)
    ds = ebc.Dataset(torch.from_numpy(x).cuda(), dtype=dt)
    ds.set_variant(var)
    return x, ds


def _solo(env, spec, seed):
    x, ds = _make(env, spec, seed)
    out = [t.cpu().numpy() for t in ds.greedy(spec[4])]
    ds.sync()
    return x, out


@pytest.mark.parametrize("graph", [False, True])
def test_batched_equals_solo(env, ref, graph):
    torch, ebc = env
    print(f"[gpu-case] batched mix of {len(MIX)} instances, graph={graph}", flush=True)
    solos = [_solo(env, s, 100 + i) for i, s in enumerate(MIX)]
    dss = [_make(env, s, 100 + i)[1] for i, s in enumerate(MIX)]
    batch = ebc.Batch(dss)
    if graph:
        batch.set_graph(True)
    info = batch.info()
    assert info["buckets"] >= 5
    ks = [s[4] for s in MIX]
    for rep in range(3 if graph else 1):
        outs = batch.greedy(ks)
        for ds in dss:
            ds.sync()
        for (x, so), bo, spec in zip(solos, outs, MIX):
            for a, b in zip(so, bo):
                np.testing.assert_array_equal(b.cpu().numpy(), a, err_msg=str(spec))
    # float32 instances against the oracle
    for (x, so), spec in zip(solos, MIX):
        if spec[2] == "f32":
            rsel, rf, _ = ref.greedy(x, spec[4])
            assert so[0].tolist() == rsel.tolist()
            np.testing.assert_allclose(so[1], rf, rtol=1e-5)


def test_batched_k_change_same_ticks(env):
    torch, ebc = env
    print("[gpu-case] batched graph replay with changed k", flush=True)
    specs = [(600, 16, "bf16", 0, 6), (900, 24, "f32", 0, 2), (1200, 8, "fp8", 0, 4)]
    dss = [_make(env, s, 200 + i)[1] for i, s in enumerate(specs)]
    batch = ebc.Batch(dss)
    batch.set_graph(True)
    first = batch.greedy([6, 2, 4])
    firstn = [[t.cpu().numpy() for t in o] for o in first]
    second = batch.greedy([3, 6, 1])   # same number of ticks: graph replayed
    for ds in dss:
        ds.sync()
    np.testing.assert_array_equal(second[0][0].cpu().numpy(), firstn[0][0][:3])
    np.testing.assert_array_equal(second[2][0].cpu().numpy(), firstn[2][0][:1])
    solo = _solo(env, (900, 24, "f32", 0, 6), 201)[1]
    np.testing.assert_array_equal(second[1][0].cpu().numpy(), solo[0])
    np.testing.assert_array_equal(second[1][1].cpu().numpy(), solo[1])


@pytest.mark.parametrize("dt", ["bf16", "fp8", "f16"])
def test_variants_are_bitwise_identical_and_autotune(env, dt, tmp_path):
    torch, ebc = env
    print(f"[gpu-case] gains variants {dt} n=3000 d=64 + autotune", flush=True)
    x = W.gaussian_mixture(np.random.default_rng(300), 3000, 64, 6).astype(np.float32)
    ds = ebc.Dataset(torch.from_numpy(x).cuda(), dtype=dt)
    m = torch.from_numpy(np.sum(x.astype(np.float64) ** 2, axis=1) * 0.3)
    outs = []
    for v in range(ebc.Dataset.variant_count(dt)):
        ds.set_variant(v)
        outs.append(ds.marginal_gains(m=m).cpu().numpy())
    ds.sync()
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    r = ds.autotune(reps=2, force=True)
    assert 0 <= r["variant"] < ebc.Dataset.variant_count(dt)
    assert all(t > 0 for t in r["times_ms"])
    path = str(tmp_path / "tune.txt")
    ebc.tune_cache_save(path)
    assert ebc.tune_cache_load(path)
    assert ebc.tune_cache_size() >= 1
    r2 = ds.autotune(reps=2)                  # served from the table
    assert r2["variant"] == r["variant"]


def test_batched_sample_against_oracle(env, ref):
    """The first 32 instances of the batched workload (n 2000..50000, d in
    {8..128}), batched in one graph: FP32 picks the oracle's points in the
    oracle's order; BF16 (the workload's dtype) reaches the oracle's f(S_20)
    within 1e-3 relative, and its f values are those of its own selections
    (float64 minima, checked with the C oracle)."""
    torch, ebc = env
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "batched512_first32_k20.json")))
    insts = W.batched_instances(seed=4, count=32)
    for p, g in zip(insts, gold["instances"]):
        assert W.sha256_of(p.x) == g["sha256_x"], p.name
    for dt in ("f32", "bf16"):
        print(f"[gpu-case] batched sample of 32 instances, {dt}, graph mode", flush=True)
        dss = [ebc.Dataset(torch.from_numpy(p.x).cuda(), dtype=dt) for p in insts]
        batch = ebc.Batch(dss)
        batch.set_graph(True)
        outs = batch.greedy([p.k for p in insts])
        for ds in dss:
            ds.sync()
        agree, gaps = [], []
        for p, g, (sel, f, _) in zip(insts, gold["instances"], outs):
            sel = sel.cpu().numpy()
            f = f.cpu().numpy()
            if dt == "f32":
                assert sel.tolist() == g["sel"], p.name
                np.testing.assert_allclose(f, g["f"], rtol=1e-12, err_msg=p.name)
                continue
            # f(S_t) of the BF16 run is the float64 f of its own sets
            m = ref.min_dist(p.x, sel)
            l0 = float(np.mean(ref.min_dist(p.x, [])))
            np.testing.assert_allclose(f[-1], l0 - float(np.mean(m)), rtol=1e-10, err_msg=p.name)
            gap = (g["f"][-1] - f[-1]) / g["f"][-1]
            gaps.append(gap)
            agree.append(len(set(sel.tolist()) & set(g["sel"])) / p.k)
            assert gap <= 1e-3, (p.name, gap)
        if dt == "bf16":
            print(f"[gpu-result] batched BF16 sample: max quality gap {max(gaps):.2e}, "
                  f"mean selection agreement {np.mean(agree):.3f}, min {min(agree):.2f}", flush=True)
        del batch, dss

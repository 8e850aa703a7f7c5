"""The seeded generators are deterministic and have the stated shapes."""
import numpy as np

from paper_2105_12026_amd import workloads as W


def test_small_normal_shapes_and_determinism():
    a, b = W.small_normal(seed=0), W.small_normal(seed=0)
    assert a.x.shape == (1000, 16) and a.x.dtype == np.float32
    assert np.array_equal(a.x, b.x) and np.array_equal(a.idx, b.idx)
    assert a.offsets.tolist() == list(range(0, 321, 5))
    for j in range(64):
        s = a.idx[a.offsets[j]:a.offsets[j + 1]]
        assert len(set(s.tolist())) == 5 and s.min() >= 0 and s.max() < 1000


def test_mixture_and_outliers():
    p = W.precision_sweep(seed=3, n=20000, d=8, n_comp=5, k=3)
    assert p.x.shape == (20000, 8)
    big = np.abs(p.x).max(axis=1) > 12  # outliers are uniform in [-20, 20]^d
    assert 100 <= big.sum() <= 210


def test_batched_and_serving_regenerate_alone():
    insts = W.batched_instances(count=3)
    again = W.batched_instances(count=3)
    for a, b in zip(insts, again):
        assert np.array_equal(a.x, b.x)
        assert 2000 <= a.n <= 50000 and a.d in (8, 16, 32, 64, 128) and a.k == 20
    reqs = W.serving_requests(count=2)
    assert all(r.x.shape[1] == 64 and 5 <= r.k <= 50 for r in reqs)

"""Seeded synthetic inputs for the exemplar-based-clustering (EBC) workloads.

This module only draws random numbers. It holds none of the method's
arithmetic (no distances, no losses, no gains), so that the CPU oracle and
the HIP path can both be fed from it without sharing any computation.

Every generator uses NumPy's PCG64 (``numpy.random.default_rng``), draws in
float64 and casts once to float32. The float32 array is the input of record
for both sides. The paper's experiments use random data of unstated
distribution (Sec. 5, experimental setup) and proprietary injection-moulding
curves (Sec. 6); the recipes below are synthetic stand-ins with the sizes of
the paper's workloads and of the benchmark configurations.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem",
    "gaussian_mixture",
    "random_sets",
    "process_curves",
    "small_normal",
    "greedy_fp32",
    "precision_sweep",
    "batched_instances",
    "serving_requests",
    "poisson_arrivals",
    "paper_sets",
    "sha256_of",
]


@dataclass
class Problem:
    """One EBC instance: ground set ``x`` (float32, row-major [n, d]) and greedy bound ``k``."""

    x: np.ndarray
    k: int = 0
    name: str = ""
    # Optional CSR-packed sets S_1..S_l (indices into the rows of x).
    offsets: np.ndarray | None = None
    idx: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def d(self) -> int:
        return int(self.x.shape[1])


def sha256_of(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def gaussian_mixture(rng: np.random.Generator, n: int, d: int, n_comp: int,
                     mean_std: float = 2.0, comp_std: float = 1.0) -> np.ndarray:
    """Gaussian mixture: weights ~ Dirichlet(1), means ~ N(0, mean_std^2 I),
    each point = its component mean + N(0, comp_std^2 I). Returns float64 [n, d]."""
    pi = rng.dirichlet(np.ones(n_comp))
    mu = rng.standard_normal((n_comp, d)) * mean_std
    z = rng.choice(n_comp, size=n, p=pi)
    return mu[z] + rng.standard_normal((n, d)) * comp_std


def random_sets(rng: np.random.Generator, n: int, l: int, set_size: int,
                replace: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """l random subsets of {0..n-1}, each of ``set_size`` indices, CSR-packed.

    Returns (offsets int64 [l+1], idx int32 [l*set_size])."""
    idx = np.empty(l * set_size, dtype=np.int32)
    for j in range(l):
        idx[j * set_size:(j + 1) * set_size] = rng.choice(n, set_size, replace=replace)
    offsets = np.arange(l + 1, dtype=np.int64) * set_size
    return offsets, idx


def small_normal(seed: int = 0, n: int = 1000, d: int = 16, n_sets: int = 64,
                 set_size: int = 5, k: int = 5) -> Problem:
    """Smallest instance: n i.i.d. N(0,1) points in d dims, then n_sets random
    sets of set_size distinct indices (drawn after x), greedy bound k."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d)).astype(np.float32)
    offsets, idx = random_sets(rng, n, n_sets, set_size)
    return Problem(x=x, k=k, name=f"normal_n{n}_d{d}", offsets=offsets, idx=idx,
                   meta={"seed": seed, "sets": n_sets, "set_size": set_size})


def greedy_fp32(seed: int = 2, n: int = 100_000, d: int = 100, n_comp: int = 20,
                k: int = 50) -> Problem:
    """FP32 greedy workload: n points from a 20-component Gaussian mixture in
    d=100 dims (means N(0,4I), unit isotropic variance, Dirichlet(1) weights)."""
    rng = np.random.default_rng(seed)
    x = gaussian_mixture(rng, n, d, n_comp).astype(np.float32)
    return Problem(x=x, k=k, name=f"gmm{n_comp}_n{n}_d{d}", meta={"seed": seed})


def precision_sweep(seed: int = 3, n: int = 200_000, d: int = 64, n_comp: int = 50,
                    outlier_frac: float = 0.01, k: int = 100) -> Problem:
    """Precision-sweep workload: a 50-component Gaussian mixture plus 1% uniform
    outliers in [-20, 20]^d, rows shuffled."""
    rng = np.random.default_rng(seed)
    n_out = int(round(n * outlier_frac))
    inl = gaussian_mixture(rng, n - n_out, d, n_comp)
    out = rng.uniform(-20.0, 20.0, size=(n_out, d))
    x = np.concatenate([inl, out], axis=0)
    x = x[rng.permutation(n)].astype(np.float32)
    return Problem(x=x, k=k, name=f"gmm{n_comp}+out_n{n}_d{d}", meta={"seed": seed})


def batched_instances(seed: int = 4, count: int = 512, n_lo: int = 2000, n_hi: int = 50_000,
                      dims=(8, 16, 32, 64, 128), k: int = 20, comp_lo: int = 5,
                      comp_hi: int = 30) -> list[Problem]:
    """Many independent problems of uneven size; instance i is drawn from
    default_rng([seed, i]) so that any one instance can be regenerated alone."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.choice(np.asarray(dims)))
        c = int(rng.integers(comp_lo, comp_hi + 1))
        x = gaussian_mixture(rng, n, d, c).astype(np.float32)
        out.append(Problem(x=x, k=k, name=f"inst{i}", meta={"seed": [seed, i], "comp": c}))
    return out


def process_curves(rng: np.random.Generator, n: int, d: int = 64,
                   noise_var: float = 0.05, anomaly_frac: float = 0.05) -> np.ndarray:
    """Synthetic process curves of length d: each request has 3 base Gaussian
    bumps (centre U(0.1,0.9), width U(0.03,0.15), height U(0.5,2)); each curve
    jitters the centres by N(0, 0.02^2) and widths/heights by a factor
    1+N(0, 0.1^2), adds N(0, noise_var) noise, and 5% of curves carry an added
    drift ramp a*t with a ~ U(0.2, 0.6). Returns float64 [n, d]."""
    t = np.arange(d, dtype=np.float64) / (d - 1)
    c0 = rng.uniform(0.1, 0.9, 3)
    w0 = rng.uniform(0.03, 0.15, 3)
    h0 = rng.uniform(0.5, 2.0, 3)
    c = c0[None, :] + rng.normal(0.0, 0.02, (n, 3))
    w = w0[None, :] * (1.0 + rng.normal(0.0, 0.1, (n, 3)))
    h = h0[None, :] * (1.0 + rng.normal(0.0, 0.1, (n, 3)))
    curves = np.zeros((n, d))
    for b in range(3):
        curves += h[:, b:b + 1] * np.exp(-0.5 * ((t[None, :] - c[:, b:b + 1]) / w[:, b:b + 1]) ** 2)
    curves += rng.normal(0.0, np.sqrt(noise_var), (n, d))
    anom = rng.random(n) < anomaly_frac
    a = rng.uniform(0.2, 0.6, n)
    curves[anom] += a[anom, None] * t[None, :]
    return curves


def serving_requests(seed: int = 5, count: int = 2000, n_lo: int = 5000, n_hi: int = 100_000,
                     d: int = 64, k_lo: int = 5, k_hi: int = 50, materialize: bool = True):
    """Summarisation requests of process curves: N ~ U{n_lo..n_hi}, d=64,
    k ~ U{k_lo..k_hi}. Request i uses default_rng([seed, i])."""
    reqs = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        n = int(rng.integers(n_lo, n_hi + 1))
        k = int(rng.integers(k_lo, k_hi + 1))
        x = process_curves(rng, n, d).astype(np.float32) if materialize else None
        reqs.append(Problem(x=x, k=k, name=f"req{i}", meta={"seed": [seed, i], "n": n}))
    return reqs


def poisson_arrivals(seed: int, rate: float, count: int) -> np.ndarray:
    """Arrival offsets (seconds from the start) of a Poisson stream of
    ``count`` requests at ``rate`` per second: cumulative sums of i.i.d.
    exponential gaps of mean 1/rate, drawn from default_rng([seed, 7])."""
    if rate <= 0:
        raise ValueError("rate must be positive")
    rng = np.random.default_rng([seed, 7])
    return np.cumsum(rng.exponential(1.0 / rate, count))


def paper_sets(seed: int = 6, n: int = 50_000, l: int = 5000, set_size: int = 10, d: int = 100) -> Problem:
    """Multi-set evaluation in the shape of the paper's runtime sweep (Sec. 5.1
    defaults: |V| = 50000, l = 5000 sets of k = 10 points, d = 100; the paper's
    data is "randomly generated" with no distribution given): i.i.d. N(0,1)
    points, then l sets of set_size distinct random indices, CSR-packed."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d)).astype(np.float32)
    idx = np.empty(l * set_size, dtype=np.int32)
    for j in range(l):
        idx[j * set_size:(j + 1) * set_size] = rng.choice(n, set_size, replace=False)
    offsets = np.arange(l + 1, dtype=np.int64) * set_size
    return Problem(x=x, k=0, name=f"paper_sets_n{n}_l{l}_k{set_size}_d{d}", offsets=offsets, idx=idx,
                   meta={"seed": seed, "sets": l, "set_size": set_size})


def case_study_curves(seed: int = 8, n: int = 1000, d: int = 3524, k: int = 50) -> Problem:
    """Long-row workload in the shape of the paper's case study (Sec. 6:
    summaries of size k from N = 1000 process series of d = 3524 samples;
    the injection-moulding data is not available): one machine's curves from
    ``process_curves`` (shared bumps, per-curve jitter, noise, 5% drifted
    anomalies) at length d."""
    rng = np.random.default_rng(seed)
    x = process_curves(rng, n, d).astype(np.float32)
    return Problem(x=x, k=k, name=f"curves_n{n}_d{d}_k{k}", meta={"seed": seed})

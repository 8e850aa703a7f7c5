"""FP64 CPU oracle for exemplar-based clustering (EBC).

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or
link this module; only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it. It shares no code with the HIP library.

Everything here is the plain definition from the paper, in float64, with
direct differences (never the norm expansion), so that it can be checked
against the paper by eye:

* k-medoids loss, Sec. 4, Definition "k-medoids loss" (Eq. k_medoids_loss):
  L(S) = |V|^-1 sum_{v in V} min_{s in S} d(v, s).
* Exemplar-based clustering, Sec. 4, Definition "Exemplar-based clustering"
  (Eq. exemplar_based_clustering): f(S) = L({e0}) - L(S u {e0}), with the
  auxiliary vector e0 the zero vector by default (the paper's example) or
  any d-vector passed as ``e0``.
* CPU evaluation, Sec. 4.1, Algorithm 1: per ground point a running minimum
  over the set, a sum over the ground points, division by |V|.
* Discrete derivative, Sec. 3, Definition "Discrete derivative":
  Delta(e | S) = f(S u {e}) - f(S).
* Greedy for the cardinality-constrained problem, Sec. 3 (Eq.
  submodular_function_optimization_cardinality_constraint and the text after
  it) and Sec. 4.1 (greedy picks the not-yet-selected item of largest
  marginal gain).
* The dissimilarity d is the squared Euclidean distance of the paper's
  experiments, Sec. 5 (experimental setup), by default. Sec. 4 defines L and
  f for any dissimilarity; ``dist="l1"`` selects the L1 (Manhattan)
  distance sum_k |a_k - b_k| instead. f stays monotone and submodular for
  any non-negative dissimilarity (it is a facility-location function), so
  the same pins apply.

Readings where the paper is silent (each listed in the design notes):
e0 is the zero vector unless given; ties in the greedy argmax go to the lowest index;
greedy keeps picking (gain 0) once every point is covered; sets are lists of
row indices into V, may be empty and may repeat an index.

Pins: tests/test_oracle_pins.py checks every function here against closed
forms, hand-derived tiny cases, exhaustive search, a library distance
routine and the submodularity/monotonicity invariants.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = [
    "sqdist",
    "l1dist",
    "dissim",
    "loss",
    "f_value",
    "eval_sets",
    "marginal_gain",
    "gains",
    "greedy",
    "exhaustive",
    "min_dist_to_set",
    "sieve_thresholds",
    "three_sieves",
    "sieve_streaming",
]


def sqdist(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Squared Euclidean distance d(a, b) = sum_k (a_k - b_k)^2 (Sec. 5), in
    float64 by direct differences. ``a`` is [n, d] or [d]; ``b`` is [d]."""
    diff = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return np.sum(diff * diff, axis=-1)


def l1dist(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """L1 (Manhattan) distance d(a, b) = sum_k |a_k - b_k| in float64 by
    direct differences. ``a`` is [n, d] or [d]; ``b`` is [d]."""
    diff = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return np.sum(np.abs(diff), axis=-1)


DISSIMILARITIES = {"sqeuclidean": sqdist, "l1": l1dist}


def dissim(a: np.ndarray, b: np.ndarray, dist: str = "sqeuclidean") -> np.ndarray:
    """The dissimilarity d(a, b) named by ``dist`` ("sqeuclidean" or "l1")."""
    if dist not in DISSIMILARITIES:
        raise ValueError(f"dist must be one of {sorted(DISSIMILARITIES)}")
    return DISSIMILARITIES[dist](a, b)


def loss(x: np.ndarray, s_vectors, dist: str = "sqeuclidean") -> float:
    """k-medoids loss L(V, S) as in Algorithm 1 (function L): for every ground
    point v a running minimum t over the vectors of S, then the sum of the t's
    divided by |V|. The running minimum starts at +inf (Algorithm 1 uses the
    largest float). ``s_vectors`` is an iterable of d-vectors; S must be
    non-empty for the result to be finite."""
    x = np.asarray(x, dtype=np.float64)
    t = np.full(x.shape[0], np.inf)
    for s in s_vectors:
        t = np.minimum(t, dissim(x, s, dist))
    return float(np.sum(t) / x.shape[0])


def _aux(x: np.ndarray, e0) -> np.ndarray:
    """The auxiliary vector e0 (Sec. 4): the zero vector unless given."""
    return np.zeros(x.shape[1]) if e0 is None else np.asarray(e0, dtype=np.float64).reshape(x.shape[1])


def f_value(x: np.ndarray, s_idx, e0=None, dist: str = "sqeuclidean") -> float:
    """f(S) = L({e0}) - L(S u {e0}) (Eq. exemplar_based_clustering;
    Algorithm 1, return statement). ``s_idx`` lists row indices of x forming
    S (may be empty)."""
    x = np.asarray(x, dtype=np.float64)
    e0 = _aux(x, e0)
    members = [x[int(i)] for i in s_idx]
    return loss(x, [e0], dist) - loss(x, [e0] + members, dist)


def eval_sets(x: np.ndarray, offsets: np.ndarray, idx: np.ndarray, e0=None, dist: str = "sqeuclidean") -> np.ndarray:
    """f(S_j) for every set of a CSR-packed family S_multi = {S_1, .., S_l}
    (Sec. 4.1: optimisers score many sets per step). Set j holds
    idx[offsets[j]:offsets[j+1]]."""
    l = len(offsets) - 1
    out = np.empty(l)
    for j in range(l):
        out[j] = f_value(x, idx[offsets[j]:offsets[j + 1]], e0, dist)
    return out


def min_dist_to_set(x: np.ndarray, s_idx, e0=None, dist: str = "sqeuclidean") -> np.ndarray:
    """m_v = min(d(v, e0), min_{s in S} d(v, s)) for every v: the per-point
    term inside L(S u {e0}) (Eq. loss_decomposed, times |V|)."""
    x = np.asarray(x, dtype=np.float64)
    m = dissim(x, _aux(x, e0), dist)
    for i in s_idx:
        m = np.minimum(m, dissim(x, x[int(i)], dist))
    return m


def marginal_gain(x: np.ndarray, m: np.ndarray, c: int, dist: str = "sqeuclidean") -> float:
    """Delta(c | S) given m = min_dist_to_set(x, S).

    From the definitions: f(S u {c}) - f(S) = L(S u {e0}) - L(S u {c} u {e0})
    = |V|^-1 sum_v [m_v - min(m_v, d(v, c))] = |V|^-1 sum_v max(0, m_v - d(v, c)).
    The tests check this against the literal difference of two f_value calls.
    """
    x = np.asarray(x, dtype=np.float64)
    dc = dissim(x, x[int(c)], dist)
    return float(np.sum(np.maximum(0.0, m - dc)) / x.shape[0])


def gains(x: np.ndarray, m: np.ndarray, cand=None, dist: str = "sqeuclidean") -> np.ndarray:
    """Delta(c | S) for every candidate c (default: every row of x)."""
    n = x.shape[0]
    cand = range(n) if cand is None else cand
    return np.array([marginal_gain(x, m, c, dist) for c in cand], dtype=np.float64)


def greedy(x: np.ndarray, k: int, e0=None, dist: str = "sqeuclidean"):
    """Greedy maximisation of f under |S| <= k (Sec. 3; Sec. 4.1).

    Each step scores every not-yet-selected point by its marginal gain,
    picks the largest (lowest index among equal float64 values), and extends
    S. Returns (selected indices [k], f(S_1..S_k) [k], gains [k])."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    l0 = float(np.sum(dissim(x, _aux(x, e0), dist)) / n)
    m = min_dist_to_set(x, [], e0, dist)
    chosen = np.zeros(n, dtype=bool)
    sel, fs, gs = [], [], []
    for _ in range(k):
        g = gains(x, m, dist=dist)
        g[chosen] = -np.inf
        c = int(np.argmax(g))  # first maximum = lowest index on ties
        sel.append(c)
        gs.append(float(g[c]))
        chosen[c] = True
        m = np.minimum(m, dissim(x, x[c], dist))
        fs.append(l0 - float(np.sum(m) / n))
    return np.array(sel, dtype=np.int64), np.array(fs), np.array(gs)


def exhaustive(x: np.ndarray, k: int, e0=None, dist: str = "sqeuclidean"):
    """max_{S subset V, |S| <= k} f(S) by enumerating every subset (Eq.
    submodular_function_optimization_cardinality_constraint). Tiny n only.
    Returns (best value, best subset as a tuple)."""
    n = x.shape[0]
    best, arg = 0.0, ()
    for size in range(0, k + 1):
        for s in itertools.combinations(range(n), size):
            v = f_value(x, s, e0, dist)
            if v > best:
                best, arg = v, s
    return best, arg


def sieve_thresholds(m: float, k: int, eps: float) -> list:
    """Guesses of the optimum for a threshold rule (the sieve grid of the
    streaming optimisers the paper cites in Sec. 2 and runs in Sec. 6): every
    power (1+eps)^i with m <= (1+eps)^i <= k*m, where m is the largest
    singleton value max_e f({e}); largest first. Empty when m <= 0."""
    if m <= 0.0:
        return []
    base = math.log1p(eps)
    lo = math.ceil(math.log(m) / base)
    hi = math.floor(math.log(k * m) / base)
    return [(1.0 + eps) ** i for i in range(hi, lo - 1, -1)]


def three_sieves(x: np.ndarray, k: int, eps: float, T: int, m=None, order=None, e0=None, dist: str = "sqeuclidean"):
    """Three Sieves: one summary S built from a stream of the points of V.

    The threshold v starts at the largest guess of sieve_thresholds. An
    arriving point e joins S when |S| < k and
        Delta(e | S) >= (v/2 - f(S)) / (k - |S|);
    otherwise a counter of consecutive rejections grows, and after T of them
    v moves to the next smaller guess (the counter restarts; it also restarts
    on every acceptance; at the smallest guess v stays). The stream ends
    early once |S| = k. ``m`` is the largest singleton value (computed when
    None); ``order`` the stream as indices into x (default 0..n-1).
    Returns (accepted indices, f(S) after each acceptance, v at each
    acceptance, number of points examined)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    order = range(n) if order is None else [int(i) for i in order]
    mv = min_dist_to_set(x, [], e0, dist)
    l0 = float(np.sum(mv) / n)
    if m is None:
        m = max(marginal_gain(x, mv, c, dist) for c in range(n))
    grid = sieve_thresholds(m, k, eps)
    sel, fs, vs = [], [], []
    if not grid or k <= 0:
        return sel, fs, vs, 0
    j, t, fS, seen = 0, 0, 0.0, 0
    for e in order:
        if len(sel) == k:
            break
        seen += 1
        v = grid[j]
        g = marginal_gain(x, mv, e, dist)
        if g >= (v / 2.0 - fS) / (k - len(sel)):
            sel.append(e)
            mv = np.minimum(mv, dissim(x, x[e], dist))
            fS = l0 - float(np.sum(mv) / n)
            fs.append(fS)
            vs.append(v)
            t = 0
        else:
            t += 1
            if t >= T and j + 1 < len(grid):
                j += 1
                t = 0
    return sel, fs, vs, seen


def sieve_streaming(x: np.ndarray, k: int, eps: float, m=None, order=None, e0=None, dist: str = "sqeuclidean"):
    """Sieve Streaming (the paper names it, Sec. 2 and Sec. 4.1, as an
    optimiser that scores many sets per step): one summary S_v per guess v of
    sieve_thresholds. Every arriving point is offered to every summary,
    and joins S_v when |S_v| < k and Delta(e | S_v) >= (v/2 - f(S_v)) /
    (k - |S_v|). The stream ends early once every summary is full. Returns
    (indices of the best summary, f after each of its acceptances, its v,
    number of points examined); the best summary is the first, in grid
    order (largest v first), with the largest f."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    order = range(n) if order is None else [int(i) for i in order]
    m0 = min_dist_to_set(x, [], e0, dist)
    l0 = float(np.sum(m0) / n)
    if m is None:
        m = max(marginal_gain(x, m0, c, dist) for c in range(n))
    grid = sieve_thresholds(m, k, eps)
    if not grid or k <= 0:
        return [], [], 0.0, 0
    mv = [m0.copy() for _ in grid]
    sel = [[] for _ in grid]
    fs = [[] for _ in grid]
    fS = [0.0] * len(grid)
    seen = 0
    for e in order:
        if all(len(s) == k for s in sel):
            break
        seen += 1
        for j, v in enumerate(grid):
            if len(sel[j]) == k:
                continue
            g = marginal_gain(x, mv[j], e, dist)
            if g >= (v / 2.0 - fS[j]) / (k - len(sel[j])):
                sel[j].append(e)
                mv[j] = np.minimum(mv[j], dissim(x, x[e], dist))
                fS[j] = l0 - float(np.sum(mv[j]) / n)
                fs[j].append(fS[j])
    best = 0
    for j in range(len(grid)):
        if fS[j] > fS[best]:
            best = j
    return sel[best], fs[best], grid[best], seen

"""Write the stored expected values under tests/golden/ by calling only the
oracle (oracle/ebc_oracle.py and oracle/ebc_ref.c) on the seeded synthetic
workloads. Nothing here touches the HIP library.

    python tests/golden/make_golden.py small      # seconds
    python tests/golden/make_golden.py gmm100k    # ~2 h on 8 cores (FP64 greedy, k=50)
    python tests/golden/make_golden.py sweep200k  # ~15 min on 8 cores (lazy FP64 greedy, k=100)
    python tests/golden/make_golden.py batched_sample  # ~5 min on 8 cores (32 instances, lazy, k=20)

Each JSON file records the generator, its seed, the SHA-256 of the float32
input of record, the oracle entry point used, its thread count and wall time.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import build_ref, ebc_oracle, ref  # noqa: E402
from paper_2105_12026_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _dump(name, obj):
    path = os.path.join(HERE, name)
    with open(path, "w") as fh:
        json.dump(obj, fh, indent=1)
    print("wrote", path, flush=True)


def small():
    p = W.small_normal(seed=0)
    t0 = time.time()
    f_sets = ebc_oracle.eval_sets(p.x, p.offsets, p.idx)
    sel, f, g = ebc_oracle.greedy(p.x, p.k)
    _dump("normal_n1000_d16.json", {
        "workload": "small_normal(seed=0): 1000 x 16 N(0,1), 64 sets of 5, greedy k=5",
        "sha256_x": W.sha256_of(p.x), "sha256_idx": W.sha256_of(p.idx),
        "oracle": "oracle.ebc_oracle (NumPy, float64, direct differences)",
        "seconds": time.time() - t0,
        "f_sets": f_sets.tolist(), "sel": sel.tolist(), "f": f.tolist(), "gain": g.tolist(),
    })


def gmm100k():
    p = W.greedy_fp32(seed=2)
    t0 = time.time()
    sel, f, g = ref.greedy(p.x, p.k)
    _dump("gmm20_n100000_d100_k50.json", {
        "workload": "greedy_fp32(seed=2): 100000 x 100, 20-component Gaussian mixture, greedy k=50",
        "sha256_x": W.sha256_of(p.x),
        "oracle": "oracle/ebc_ref.c ebc_ref_greedy (C, float64, direct differences)",
        "threads": ref.threads(), "seconds": time.time() - t0,
        "sel": sel.tolist(), "f": f.tolist(), "gain": g.tolist(),
    })


def sweep200k():
    p = W.precision_sweep(seed=3)
    t0 = time.time()
    # lazy evaluation of the same greedy: bitwise the plain loop's run (pinned in
    # tests/test_oracle_pins.py, and on the 100000 x 100 run above)
    sel, f, g, evals = ref.greedy_lazy(p.x, p.k)
    _dump("gmm50+out_n200000_d64_k100.json", {
        "workload": "precision_sweep(seed=3): 198000 x 64 50-component mixture + 2000 uniform [-20,20] outliers, "
                    "shuffled; greedy k=100",
        "sha256_x": W.sha256_of(p.x),
        "oracle": "oracle/ebc_ref.c ebc_ref_greedy_lazy (C, float64, direct differences, lazy re-evaluation)",
        "threads": ref.threads(), "seconds": time.time() - t0, "gain_evaluations": evals,
        "sel": sel.tolist(), "f": f.tolist(), "gain": g.tolist(),
    })


def batched_sample():
    """The first 32 of the 512 batched instances (k = 20), each through the
    lazy float64 greedy: the reference of the batched path's quality check."""
    insts = W.batched_instances(seed=4, count=32)
    t0 = time.time()
    out = []
    for p in insts:
        sel, f, g, evals = ref.greedy_lazy(p.x, p.k)
        out.append({"name": p.name, "seed": p.meta["seed"], "n": int(p.x.shape[0]), "d": int(p.x.shape[1]),
                    "k": p.k, "sha256_x": W.sha256_of(p.x), "sel": sel.tolist(), "f": f.tolist(),
                    "gain_evaluations": int(evals)})
        print(p.name, p.x.shape, f"{time.time() - t0:.0f} s", flush=True)
    _dump("batched512_first32_k20.json", {
        "workload": "batched_instances(seed=4): instances 0..31 of 512 (n in [2000, 50000], d in "
                    "{8, 16, 32, 64, 128}, 5-30 components), greedy k=20 each",
        "oracle": "oracle/ebc_ref.c ebc_ref_greedy_lazy (C, float64, direct differences, lazy re-evaluation)",
        "threads": ref.threads(), "seconds": time.time() - t0, "instances": out,
    })


if __name__ == "__main__":
    build_ref.build()
    what = sys.argv[1:] or ["small"]
    for w in what:
        globals()[w]()

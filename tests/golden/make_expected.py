"""Write oracle results for the full-size workloads to expected_*.json.

Calls only ``oracle/`` and the seeded generators in ``synth.py``; nothing
from the GPU engine.  The GPU parity tests and the benchmark regenerate the
same seeded inputs on the GPU machine, check that their bytes hash to the
SHA-256 recorded here, and compare against these values.

Usage:  python tests/golden/make_expected.py NAME [NAME ...]
Names:  uniform_n1000 normal_n8000 normal_n8192 wishart_n16384
        wishart_batch512 wishart_batch64
Each name writes tests/golden/expected_<name>.json:

* ``sha256_f64`` / ``sha256_f32``: the input's bytes (FP64, and the
  FP32-rounded copy where the workload has an FP32 variant);
* ``f64`` / ``f32``: the oracle's (sign, log|det|, info) on the FP64 input
  and on the FP32-rounded input (the FP32 engine's own input values);
* single matrices: ``piv_col`` (the oracle's pivot column per step on the
  FP64 input), ``min_gap`` and ``gap_safe_steps`` (steps before the first
  whose pivot beats the runner-up by a relative margin below 1e-9, the
  prefix on which a rounding-level difference cannot change a choice);
* wishart_batch64: ``grad_samples``, per member 16 seeded entries (i, j) of
  A^{-T} from the oracle's Gauss-Jordan inverse (FP64 input and the
  FP32-rounded input).
The oracle runs with one OpenMP thread per processor over the rows of each
step (its results do not depend on the thread count).
"""

from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

GAP_SAFE = 1e-9
GRAD_SAMPLES = 16


def _one(a: np.ndarray, pivots: bool = False) -> dict:
    t = time.time()
    if pivots:
        r, gap = O.slogdet_gaps(a)
    else:
        r = O.slogdet(a)
    out = {"sign": r.sign, "logabsdet": r.logabsdet, "info": r.info,
           "oracle_seconds": round(time.time() - t, 3)}
    if pivots:
        small = np.flatnonzero(gap < GAP_SAFE)
        out["piv_col"] = [int(c) for c in r.piv_col]
        out["min_gap"] = float(gap.min()) if gap.size else 1.0
        out["gap_safe_steps"] = int(small[0]) if small.size else int(a.shape[0])
    return out


def grad_samples(a: np.ndarray, seed: int) -> dict:
    n = a.shape[0]
    g = np.random.default_rng(seed)
    ij = g.integers(0, n, size=(GRAD_SAMPLES, 2))
    ij[0] = (0, 0)
    ij[1] = (n - 1, n - 1)
    inv64 = O.inverse(a)
    inv32 = O.inverse(a.astype(np.float32).astype(np.float64))
    # d log|det A| / dA = A^{-T}: entry (i, j) is A^{-1}[j, i]
    return {"ij": [[int(i), int(j)] for i, j in ij],
            "f64": [float(inv64[j, i]) for i, j in ij],
            "f32": [float(inv32[j, i]) for i, j in ij]}


def run(name: str) -> dict:
    spec = dict(synth.CONFIGS[name])
    out = {"workload": name, "spec": spec,
           "generator": "synth.py (numpy default_rng / PCG64)",
           "oracle": "oracle/mc_oracle.c, top-down rows, largest-|a| column",
           "host": platform.processor() or platform.machine(),
           "oracle_threads": O.num_procs()}
    data = synth.make(name)
    if spec["kind"] == "wishart_batch":
        sizes, mats = data
        out["sizes"] = sizes
        out["sha256_f64"] = synth.sha256_of(mats)
        out["sha256_f32"] = synth.sha256_of([m.astype(np.float32) for m in mats])
        out["f64"] = [_one(m) for m in mats]
        out["f32"] = [_one(m.astype(np.float32)) for m in mats]
        if name == "wishart_batch64":
            out["grad_samples"] = [grad_samples(m, 9000 + k)
                                   for k, m in enumerate(mats)]
    else:
        a = data
        out["sha256_f64"] = synth.sha256_of(a)
        out["f64"] = _one(a, pivots=True)
        if spec["kind"] == "wishart":
            out["sha256_f32"] = synth.sha256_of(a.astype(np.float32))
            out["f32"] = _one(a.astype(np.float32))
    return out


def main(names):
    O.set_threads(O.num_procs())
    for name in names:
        res = run(name)
        path = os.path.join(HERE, f"expected_{name}.json")
        with open(path, "w") as f:
            json.dump(res, f, indent=1)
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["uniform_n1000"])

"""Write oracle results for the full-size workloads to expected_*.json.

Calls only ``oracle/`` and the seeded generators in ``synth.py``; nothing
from the GPU engine.  The GPU parity tests regenerate the same seeded
inputs on the GPU machine and compare against these values.

Usage:  python tests/golden/make_expected.py NAME [NAME ...]
Names:  uniform_n1000 normal_n8000 normal_n8192 wishart_n16384
        wishart_batch512 wishart_batch64
Each name writes tests/golden/expected_<name>.json.  FP32 variants are the
oracle on the FP32-rounded input (the FP32 engine's own input values).
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


def _one(a: np.ndarray) -> dict:
    t = time.time()
    r = O.slogdet(a)
    return {"sign": r.sign, "logabsdet": r.logabsdet, "info": r.info,
            "oracle_seconds": round(time.time() - t, 3)}


def run(name: str) -> dict:
    spec = dict(synth.CONFIGS[name])
    out = {"workload": name, "spec": spec,
           "generator": "synth.py (numpy default_rng / PCG64)",
           "oracle": "oracle/mc_oracle.c, top-down rows, largest-|a| column",
           "host": platform.processor() or platform.machine()}
    data = synth.make(name)
    if spec["kind"] == "wishart_batch":
        sizes, mats = data
        out["sizes"] = sizes
        out["f64"] = [_one(m) for m in mats]
        out["f32"] = [_one(m.astype(np.float32)) for m in mats]
    else:
        a = data
        out["f64"] = _one(a)
        if spec["kind"] == "wishart":
            out["f32"] = _one(a.astype(np.float32))
    return out


def main(names):
    for name in names:
        res = run(name)
        path = os.path.join(HERE, f"expected_{name}.json")
        with open(path, "w") as f:
            json.dump(res, f, indent=1)
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["uniform_n1000"])

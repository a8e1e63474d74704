"""Write sampled oracle solutions of the full-size workloads to tests/golden/*.json.

Calls only the CPU oracle and the seeded input generators.  Each file holds, for a few
right-hand-side columns, the oracle's X at sampled row indices (float64 as repr strings).
Usage: python tests/golden/make_golden.py [workload ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth   # noqa: E402

SPECS = {
    # workload: (columns, samples per column)
    "varcoef_n2048_m256_k512": ([0, 257, 511], 1500),
    "adjoint_n1024_m256_k256": ([0, 128, 255], 1500),
    "mixed_n4096_m512_k1024": ([0, 1023], 1500),
}


def make(name):
    cols, ns = SPECS[name]
    w = synth.WORKLOADS[name]
    sys_ = synth.workload_system(name)
    n = sys_.N * sys_.M
    F = synth.rhs_columns(w["seed"], sys_.N, sys_.M, cols)
    t0 = time.time()
    X = oracle.solve(sys_, F)
    rng = np.random.default_rng(12345)
    out = {"workload": name, "N": sys_.N, "M": sys_.M, "seed": w["seed"], "columns": cols,
           "generator": "tests/golden/make_golden.py (oracle block-Thomas, float64)", "samples": []}
    for t, k in enumerate(cols):
        idx = np.sort(rng.choice(n, ns, replace=False))
        idx = np.unique(np.concatenate([idx, [0, n - 1]]))
        out["samples"].append({"column": k, "index": idx.tolist(), "value": [repr(float(v)) for v in X[t, idx]],
                               "col_norm": repr(float(np.linalg.norm(X[t])))})
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"{name}: oracle {time.time() - t0:.1f} s -> {path}")


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["varcoef_n2048_m256_k512", "adjoint_n1024_m256_k256"]):
        make(name)

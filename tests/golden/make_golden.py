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

def tile_columns(K, tiles, step=32):
    """One column in each of `tiles` groups of `step` columns, at a different position in each group
    (so that every column tile of the solve kernels, and lanes across the tile, are sampled), plus the
    first and the last column."""
    cols = {0, K - 1}
    for t in range(tiles):
        cols.add(min(K - 1, t * (K // tiles) + (7 * t + 3) % step))
    return sorted(cols)


SPECS = {
    # workload: (columns, samples per column)
    "varcoef_n2048_m256_k512": (tile_columns(512, 16), 500),
    "adjoint_n1024_m256_k256": (tile_columns(256, 8), 800),
    "mixed_n4096_m512_k1024": (tile_columns(1024, 8), 800),
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


BATCH_LARGEST = 8        # systems of the batched workload with the most sweep work (N M^2 K)


def largest_batch_shapes(count=BATCH_LARGEST):
    """The `count` systems of the 64-system batched workload with the largest N M^2 K, in that order."""
    return sorted(synth.batch_shapes(), key=lambda t: -t[0] * t[1] * t[1] * t[2])[:count]


def make_batched(samples=500):
    """Oracle samples for the largest systems of the batched workload (coefficients of the tiny
    workload, C = tridiag(-1, 4.5, -1), A = B = I; right-hand sides from each system's seed):
    columns 0, K//2 and K-1 of each."""
    out = {"workload": "batched_64_largest", "generator": "tests/golden/make_golden.py (oracle block-Thomas, float64)",
           "systems": []}
    rng = np.random.default_rng(54321)
    t0 = time.time()
    for N, M, K, seed in largest_batch_shapes():
        sys_ = synth.laplace_system(N, M, 4.5)
        n = N * M
        cols = [0, K // 2, K - 1]
        F = synth.rhs_columns(seed, N, M, cols)
        X = oracle.solve(sys_, F)
        ent = {"N": N, "M": M, "K": K, "seed": seed, "samples": []}
        for t, k in enumerate(cols):
            idx = np.unique(np.concatenate([np.sort(rng.choice(n, samples, replace=False)), [0, n - 1]]))
            ent["samples"].append({"column": k, "index": idx.tolist(), "value": [repr(float(v)) for v in X[t, idx]]})
        out["systems"].append(ent)
        print(f"  N={N} M={M} K={K}: {time.time() - t0:.1f} s", flush=True)
    path = os.path.join(HERE, "batched_64_largest.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"batched_64_largest -> {path}")


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["varcoef_n2048_m256_k512", "adjoint_n1024_m256_k256", "mixed_n4096_m512_k1024"]):
        if name == "batched_64_largest":
            make_batched()
        else:
            make(name)

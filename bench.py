"""Benchmark: right-hand-side solves per second of the block-tridiagonal solver on one MI355X.

One step = one solve (Algorithm 2, step 2: subdomain sweeps, interface right-hand side,
dichotomy, superposition) of the K right-hand sides of the workload, on a plan factored
once before the timed region (the factor time is reported beside it).  Inputs are seeded
synthetic data already resident in device memory.

Prints one JSON line.  `roofline` is for the kernel with the largest measured time in the
timed region (HIP events on the solve's stream); `cpu_baseline` times the CPU oracle on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RHS solves/sec & %MFMA peak; FP64 vs mixed+refine at rel. residual ≤1e-10"
PEAK_F64_MFMA = 78.6   # TFLOP/s, MI355X dense float64 matrix
PEAK_F32_MFMA = 157.3
PEAK_HBM = 8000.0      # GB/s

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (FETCH_SIZE scaled by 2.0 and
# WRITE_SIZE by 1.0, the factors a 1 GiB device copy shows), valid only for the kernel sources they
# were taken on (profiles/solve_f64_n4096_m512_k1024.md, profiles/scalar_dichotomy_n65536_k1024.md).
KERNEL_SOURCES = {
    "f64": ["kernels_f64.hip", "tile_bodies.h", "device_common.h", "internal.h"],
    "scalar": ["kernels_scalar.hip", "device_common.h", "internal.h"],
}
MEASURED_TRAFFIC = {
    # (kernel, workload): (source set, source hash (kernel_source_hash), read bytes, write bytes)
    ("sweep", "mixed_n4096_m512_k1024"): ("f64", "0a99f9263b833a11", 54.0047e9, 32.7995e9),
    ("superposition", "mixed_n4096_m512_k1024"): ("f64", "0a99f9263b833a11", 50.5494e9, 16.6430e9),
    ("scalar_subtrees", "scalar_n65536_k1024"): ("scalar", "ad931b9574f73499", 0.55359e9, 0.53687e9),
}


def kernel_source_hash(which="f64"):
    """sha256 prefix over the sources that define the kernels of a measured-traffic entry."""
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES[which]:
        with open(os.path.join(ROOT, "paper_1108_4181_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    rec = MEASURED_TRAFFIC.get((kernel, workload))
    if rec is None:
        return None
    return rec[2] + rec[3] if kernel_source_hash(rec[0]) == rec[1] else None


def partition(N, p):
    base, extra = divmod(N, p)
    ks, k = [], 0
    for s in range(p):
        ks.append(k)
        k += base + (1 if s < extra else 0)
    return ks + [N]


def algorithmic_work(N, M, K, p):
    """Flops and HBM bytes per solve that the method itself needs (A, B diagonal; C tridiagonal).

    sweep:         forward  beta_i = D_i^{-1}(F_i + a_i o beta_{i-1}) : 2 M^2 K per interior row
                   backward W_i = alpha_i W_{i+1} + beta_i          : 2 M^2 K per interior row but the last
                   bytes: D^{-1}, alpha once (8 M^2 per row each), F read, beta written, beta read,
                   W written (8 M K per row each)
    superposition: X_i = W_i + U_i X_{k_s} + V_i X_{k_{s+1}}         : 4 M^2 K per interior row (2 M^2 K in
                   the last subdomain, whose right boundary value is zero)
                   bytes: U, V once (16 M^2 per row), W read, X written (8 M K per row each)
    """
    ks = partition(N, p)
    n = [ks[s + 1] - ks[s] - 1 for s in range(p)]
    fwd = sum(n)
    bwd = sum(max(v - 1, 0) for v in n)
    sweep_flops = 2.0 * M * M * K * (fwd + bwd)
    sweep_bytes = 8.0 * (M * M * (fwd + bwd) + M * K * (N + 3 * fwd))
    sup_flops = 4.0 * M * M * K * fwd - 2.0 * M * M * K * n[-1]
    sup_bytes = 8.0 * (2 * M * M * fwd + 2 * M * K * fwd)
    depth = 0
    q = p
    while q > 0:
        depth += 1
        q >>= 1
    dich_flops = 2.0 * M * M * K * p * (depth + 2)
    dich_bytes = 8.0 * (M * M * p * depth + 3 * p * M * K)   # stored inverse rows once, F~ and X rows
    return dict(sweep_flops=sweep_flops, sweep_bytes=sweep_bytes, sup_flops=sup_flops, sup_bytes=sup_bytes,
                dich_flops=dich_flops, dich_bytes=dich_bytes, total_flops=sweep_flops + sup_flops + dich_flops)


def factor_work(N, M, p):
    """Flops of the factor that the method itself defines (A, B diagonal; C tridiagonal), counting
    a dense M x M product or a Gauss-Jordan inversion as 2 M^3:
      subdomain elimination, per interior row: D_i^{-1}, and Gamma_i = D_i^{-1} a_i Gamma_{i-1}
                             (no product on a subdomain's first row)
      backward chains, per interior row but a subdomain's last: U_i = alpha_i U_{i+1} + Gamma_i,
                             V_i = alpha_i V_{i+1}
      dichotomy tree, per element of a node's left or right chain: the chain matrix (none for the
                             chain's first), its inverse, alpha, and the row G_j (two products);
                             per node: S_m (one product per present side), its inverse, the maps H
    """
    ks = partition(N, p)
    n = [ks[s + 1] - ks[s] - 1 for s in range(p)]
    c = 2.0 * float(M) ** 3
    fl = sum(c * (2 * v - min(v, 1)) for v in n)           # inversions, Gamma products
    fl += sum(c * 2 * max(v - 1, 0) for v in n)             # U, V
    nodes = []

    def build(l, r):
        m = (l + r) // 2
        nodes.append((l, r, m))
        if m > l:
            build(l, m - 1)
        if m < r:
            build(m + 1, r)

    build(0, p - 1)
    for l, r, m in nodes:
        for length in (m - l, r - m):
            if length > 0:
                fl += c * (4 * length - 1) + c * 2 * length    # chain, inverse, alpha; rows G_j
        fl += c * ((m > l) + (m < r)) + c                    # S_m, its inverse
        fl += c * ((l > 0) + (r < p - 1))                    # H^L, H^R
    return fl


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, rows, cols, cols_1t, threads):
    """The CPU oracle (plain float64 block Thomas, OpenMP over right-hand sides) on a bounded sample of
    the workload: the leading `rows` block rows of the same matrix (a truncated system; the oracle's
    solve cost per right-hand side is linear in the number of block rows, so its time is scaled by
    N / rows), with `cols` right-hand sides on `threads` threads and `cols_1t` on one thread.  The
    factor (not part of the metric) is timed once, on `threads` threads."""
    import numpy as np

    import oracle
    import synth

    full = synth.workload_system(w["name"])
    N, M = full.N, full.M
    rows = N if rows <= 0 else min(rows, N)
    sub = synth.System(rows, M, full.A[:rows], full.B[:rows], full.C[:rows], full.fmt_A, full.fmt_B, full.fmt_C)
    F = np.ascontiguousarray(synth.rhs_columns(w["seed"], N, M, range(cols))[:, : rows * M])
    t0 = time.perf_counter()
    fac = oracle.Factor(sub, threads)
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    fac.solve(F)
    ts = time.perf_counter() - t0
    print(f"bench: oracle sample on {threads} threads {ts:.1f} s", file=sys.stderr, flush=True)
    fac.threads = 1
    F1 = np.ascontiguousarray(F[:cols_1t])
    t0 = time.perf_counter()
    fac.solve(F1)
    ts1 = time.perf_counter() - t0
    scale = N / rows
    per_rhs = ts * scale / cols
    per_rhs_1t = ts1 * scale / cols_1t
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {
        "value": 1.0 / per_rhs,
        "unit": "RHS/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle block-Thomas solve of the leading {rows} of {N} block rows (M={M}; same coefficients) "
                   f"with {cols} of {w['K']} right-hand sides on {threads} threads and {cols_1t} on 1 thread; "
                   f"solve seconds per right-hand side scaled x{scale:g} to N={N}"
                   + (" (extrapolated)" if rows < N else "") + "; factor timed separately"),
        "extrapolated": rows < N,
        "value_1thread": 1.0 / per_rhs_1t,
        "solve_s_per_rhs": per_rhs,
        "solve_s_per_rhs_1thread": per_rhs_1t,
        "sample_factor_s": tf,
        "factor_s_scaled": tf * scale,
        "nproc": os.cpu_count(),
        "affinity_cpus": affinity,
        "cpu_model": _cpu_model(),
    }


def bench_batched(args):
    """64 uneven systems: one persistent launch replayed from a HIP graph (float32 sweeps, float64
    reduced systems and refinement to 1e-10) against per-system float64 solves."""
    import torch

    import synth
    import paper_1108_4181_amd as td

    shapes = synth.batch_shapes()
    dev = torch.device("cuda:0")
    # autotune the subdomain length for every (M, K bucket) of the batch (timed search in the library)
    t0 = time.perf_counter()
    tuned = {}
    prec = "f32"   # float64 plans of all 64 systems with their workspaces exceed one GPU's HBM
    passes = args.batch_passes
    for M, Kb in sorted({(m, td._kbucket(k)) for _, m, k, _ in shapes}):
        # (the batch's work items have fixed tiles: only the subdomain length is searched)
        tuned[f"M{M}|K{Kb}"] = td.autotune(M, Kb, prec, probe_N=1024, candidates=(16, 32, 64), tiles=False)["L"]
    tune_s = time.perf_counter() - t0
    plans, Fs, Xs, systems = [], [], [], []
    t0 = time.perf_counter()
    for N, M, K, seed in shapes:
        sysq = synth.laplace_system(N, M, 4.5)
        p = td.choose_subdomains(N, M, K, prec)
        plans.append(td.Plan.from_system(sysq, device=dev, subdomains=p, sweep_prec=prec))
        Fs.append(synth.rhs_torch(seed, N, M, K, dev))
        Xs.append(torch.zeros_like(Fs[-1]))
        systems.append((N, M, K, p))
    torch.cuda.synchronize()
    factor_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan_bytes = sum(pl.plan_info()["device_bytes"] for pl in plans)
    batch = td.Batch(plans, Fs, Xs, passes=passes, tol=1e-10)
    build_s = time.perf_counter() - t0
    batch.solve()
    infos, ok = batch.info()
    for _ in range(args.warmup):
        batch.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1e3 / args.steps
    totK = sum(k for _, _, k, _ in systems)
    flops = sum(8.0 * m * m * k * (n - p) for n, m, k, p in systems)
    batch.close()
    for pl in plans:
        pl.close()
    del plans, batch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    # baseline: the same systems solved one after another with per-system float64 launches
    base_ms = 0.0
    for (N, M, K, p), F, X in zip(systems, Fs, Xs):
        pl = td.Plan.from_system(synth.laplace_system(N, M, 4.5), device=dev, subdomains=p)
        pl.solve(F, X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, args.steps // 4)):
            pl.solve(F, X)
        torch.cuda.synchronize()
        base_ms += (time.perf_counter() - t0) * 1e3 / max(1, args.steps // 4)
        pl.close()
    worst = max(i["max_col_rel_residual"] for i in infos)
    out = {
        "metric": METRIC, "value": totK / (ms / 1e3), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "batched_64_uneven", "systems": len(systems), "total_rhs": totK,
                   "sweep_prec": prec, "passes": passes, "subdomains": "autotuned"},
        "plan_device_bytes": plan_bytes,
        "per_system_f64_ms": base_ms, "per_system_f64_rhs_per_s": totK / (base_ms / 1e3),
        "speedup_vs_per_system_f64": base_ms / ms, "all_converged": ok, "max_col_rel_residual": worst,
        "max_passes_used": 1 + max(i["iterations"] for i in infos), "algorithmic_tflops": flops / (ms * 1e-3) / 1e12,
        "factor_s": factor_s, "graph_build_s": build_s, "autotune_s": tune_s, "tuned_subdomain_length": tuned,
    }
    print(json.dumps(out))


def band_storage(n, kl, ku, seed):
    """General band storage (rows = diagonals, (kl+ku+1) x n) of a diagonally dominant band matrix."""
    import numpy as np

    import synth

    ab = synth.uniform_range(seed, 11, 0, (kl + ku + 1) * n, -1.0, 1.0).reshape(kl + ku + 1, n)
    ab[ku, :] = (kl + ku + 1) * 1.5 + np.abs(ab[ku, :])
    j = np.arange(n)
    for d in range(kl + ku + 1):
        i = j - (ku - d)
        ab[d, (i < 0) | (i >= n)] = 0.0
    return ab


def bench_band(args):
    """A band matrix (n, kl, ku) solved through its block-tridiagonal form (blocks of size max(kl, ku),
    dense triangular couplings, float64), K right-hand sides."""
    import numpy as np
    import torch

    import synth
    import paper_1108_4181_amd as td

    n, kl, ku, K = (int(v) for v in args.band.split(","))
    dev = torch.device("cuda:0")
    ab = torch.as_tensor(np.ascontiguousarray(band_storage(n, kl, ku, 4242).T), device=dev)
    F = synth.rhs_torch(4243, n, 1, K, dev)
    M = max(kl, ku, 1)
    N = -(-n // M)
    p = args.subdomains or td.choose_subdomains(N, M, K)
    t0 = time.perf_counter()
    solver = td.BandSolver(ab, kl, ku, subdomains=p)
    torch.cuda.synchronize()
    factor_ms = (time.perf_counter() - t0) * 1e3
    Fp = solver._pad(F)
    X = torch.empty_like(Fp)
    _, info = solver.plan.solve(Fp, X, info=True)
    for _ in range(args.warmup):
        solver.plan.solve(Fp, X)
    torch.cuda.synchronize()
    solver.plan.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.plan.solve(Fp, X)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    stages = solver.plan.stage_times()
    # dense couplings: the forward sweep is G = D^{-1} F (2 M^2 K per interior row) plus the recurrence
    # with E (2 M^2 K), the backward sweep 2 M^2 K, the superposition 4 M^2 K
    work = algorithmic_work(N, M, K, p)
    fwd = N - p
    flops = work["total_flops"] + 2.0 * M * M * K * fwd
    out = {
        "metric": METRIC, "value": K / (ms / 1e3), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "band", "n": n, "kl": kl, "ku": ku, "K": K, "block": M, "N": N, "subdomains": p},
        "stages_ms": {k: v for k, v in stages.items() if k != "count"},
        "whole_solve_tflops": flops / (ms * 1e-3) / 1e12,
        "factor_ms": factor_ms, "max_col_rel_residual": info["max_col_rel_residual"],
    }
    print(json.dumps(out))


def bench_schur(args):
    """Schur-complement CG on interface block rows (Sec. 3): a 2-D five-point operator
    (C_j = tridiag(-1, 4 + s, -1), A = B = I, s = 0.01) on a rectangle of N columns of M nodes cut
    into strips by interface columns; probing preconditioner of half-bandwidth `band`.  Compared
    with the direct float64 solve of the whole system by one plan."""
    import numpy as np
    import torch

    import synth
    import paper_1108_4181_amd as td

    N, M, nstrip, K, band = (int(v) for v in args.schur.split(","))
    width = (N - (nstrip - 1)) // nstrip
    icol = [(k + 1) * width + k for k in range(nstrip - 1)]
    dev = torch.device("cuda:0")
    sysw = synth.laplace_system(N, M, 4.01)
    A, B, C = (torch.as_tensor(np.ascontiguousarray(x), device=dev) for x in (sysw.A, sysw.B, sysw.C))
    F = synth.rhs_torch(4251, N, M, K, dev)
    t0 = time.perf_counter()
    solver = td.SchurSolver(A, B, C, icol, band=band)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    X, info = solver.solve(F, tol=1e-10, info=True)
    for _ in range(args.warmup):
        solver.solve(F, tol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.solve(F, tol=1e-10)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # one application of S to K interface vectors (scatter, interior solve, gather)
    V = torch.ones((K, len(icol) * M), dtype=torch.float64, device=dev)
    solver.apply(V)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.apply(V)
    torch.cuda.synchronize()
    apply_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # the same system by one plan (direct Algorithm 2 on the whole domain)
    plan = td.Plan.from_system(sysw, device=dev, subdomains=max(1, N // 32))
    Xd = torch.empty_like(F)
    plan.solve(F, Xd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.solve(F, Xd)
    torch.cuda.synchronize()
    direct_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    diff = float(torch.linalg.norm(X - Xd) / torch.linalg.norm(Xd))
    out = {
        "metric": METRIC, "value": K / (ms / 1e3), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "schur_cg", "N": N, "M": M, "strips": nstrip, "interfaces": len(icol), "K": K,
                   "probe_band": band, "shift": 0.01},
        "cg_iterations": info["iterations"], "cg_max_rel_residual": info["max_rel_residual"],
        "apply_ms": apply_ms, "setup_ms": setup_ms,
        "direct_plan_ms": direct_ms, "direct_plan_rhs_per_s": K / (direct_ms / 1e3),
        "rel_diff_vs_direct": diff,
    }
    solver.close()
    plan.close()
    print(json.dumps(out))


# The paper's Tables 1-2 (Sec. 2.3), smallest printed value over the process counts of each column:
# solve time "Exe" (seconds, presumably one right-hand side) with its process count, and preliminary
# time "Pre" (the factor) with its process count, on the MBC-100k cluster (Fortran-90 + MPI, node CPU
# not stated).  Taken as printed, also where a value breaks its column's trend (4096 x 150: 2.6e-3 s
# at 256 processes between 4.8e-2 and 1.3e-2; 4096 x 60: 1.3e-4 s at 2048).
PAPER_BEST = {
    # (N, M): (Exe, processes, Pre, processes)
    (2048, 60): (4.6e-4, 1024, 1.0, 32), (2048, 150): (4e-3, 1024, 15.0, 64),
    (4096, 60): (1.3e-4, 2048, 1.9, 32), (4096, 150): (2.6e-3, 256, 22.0, 64),
    (8192, 60): (1e-3, 512, 3.0, 64), (8192, 150): (1.4e-2, 1024, 30.0, 128),
    (16384, 60): (8.8e-4, 1024, 4.1, 256), (16384, 150): (2.7e-2, 1024, 44.0, 128),
    (32768, 60): (2e-3, 2048, 5.0, 256), (32768, 150): (5.5e-2, 1024, 60.0, 256),
    (65536, 60): (6.6e-3, 2048, 6.9, 256), (65536, 150): (0.1, 1024, 89.0, 256),
}


def bench_paper(args):
    """The paper's problem sizes (N = 2^11 .. 2^16 block rows, M = 60 and 150; Sec. 2.3) with the
    variable-coefficient family: factor time, the time of a one-right-hand-side solve (the paper's
    Exe) and the rate at K right-hand sides, next to the paper's best Exe on its cluster."""
    import torch

    import synth
    import paper_1108_4181_amd as td

    dev = torch.device("cuda:0")
    K = args.paper_k
    rows = []
    # one untimed factor first, so that the first size's factor time holds no one-time start-up cost
    td.Plan.from_system(synth.varcoef_system(64, 60, 1), device=dev, subdomains=4).close()
    torch.cuda.synchronize()
    for (N, M), (exe, nproc, pre, nproc_pre) in sorted(PAPER_BEST.items(), key=lambda kv: (kv[0][1], kv[0][0])):
        sysw = synth.varcoef_system(N, M, 7000 + N + M)
        p = td.default_subdomains(N, K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = td.Plan.from_system(sysw, device=dev, subdomains=p)
        torch.cuda.synchronize()
        fac_s = time.perf_counter() - t0
        res = {}
        for k in (1, K):
            F = synth.rhs_torch(7100 + N + M, N, M, k, dev)
            X = torch.empty_like(F)
            _, info = plan.solve(F, X, info=True)
            for _ in range(args.warmup):
                plan.solve(F, X)
            torch.cuda.synchronize()
            n = max(3, args.steps)
            t0 = time.perf_counter()
            for _ in range(n):
                plan.solve(F, X)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / n
            res[k] = (ms, info["max_col_rel_residual"])
            del F, X
        plan.close()
        del plan
        torch.cuda.empty_cache()
        rows.append({"N": N, "M": M, "subdomains": p, "factor_s": fac_s, "solve_ms_k1": res[1][0],
                     f"solve_ms_k{K}": res[K][0], f"rhs_per_s_k{K}": K / (res[K][0] * 1e-3),
                     "max_col_rel_residual": max(res[1][1], res[K][1]),
                     "paper_best_exe_s": exe, "paper_nproc": nproc,
                     "k1_speedup_vs_paper_exe": exe / (res[1][0] * 1e-3),
                     "paper_best_pre_s": pre, "paper_nproc_pre": nproc_pre,
                     "factor_speedup_vs_paper_pre": pre / fac_s})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    tot = sum(r[f"solve_ms_k{K}"] for r in rows)
    out = {
        "metric": METRIC, "value": len(rows) * K / (tot * 1e-3), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": tot, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "paper_sizes", "sizes": "N 2^11..2^16 x M 60, 150", "K": K,
                   "coefficients": "varcoef", "paper_hardware": "MBC-100k cluster, Fortran-90 + MPI (Sec. 2.3)"},
        "sizes": rows,
    }
    print(json.dumps(out))


def progress(msg):
    """One line per finished stage on stderr, so that a long run shows that it is alive."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mixed_n4096_m512_k1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=256, help="block rows of the oracle sample (0 = all)")
    ap.add_argument("--cpu-cols", type=int, default=128, help="right-hand sides of the oracle sample")
    ap.add_argument("--cpu-cols-1t", type=int, default=16, help="right-hand sides of the one-thread oracle sample")
    ap.add_argument("--mixed", default="f32,bf16",
                    help="low-precision sweep types to time with float64 refinement ('' = none)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="bytes of a plain device-to-device copy run before the timed region (counter calibration)")
    ap.add_argument("--batch-passes", type=int, default=3)
    ap.add_argument("--paper-k", type=int, default=256, help="right-hand sides of the paper-size sweep's rate")
    ap.add_argument("--subdomains", type=int, default=0,
                    help="override the workload's subdomain count (= N: Algorithm 1 on the whole system)")
    ap.add_argument("--band", default="65536,60,60,256",
                    help="band workload n,kl,ku,K (with --workload band)")
    ap.add_argument("--schur", default="2047,256,16,64,4",
                    help="Schur-complement workload N,M,strips,K,probe band (with --workload schur)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU (asked for --gpus {args.gpus}); sharding over "
              "several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched_64":
        bench_batched(args)
        return
    if args.workload == "paper_sizes":
        bench_paper(args)
        return
    if args.workload == "band":
        bench_band(args)
        return
    if args.workload == "schur":
        bench_schur(args)
        return

    import torch

    import synth
    import paper_1108_4181_amd as td

    w = dict(synth.WORKLOADS[args.workload])
    w["name"] = args.workload
    N, M, K, p = w["N"], w["M"], w["K"], w["p"]
    if args.subdomains:
        p = min(N, args.subdomains)
    dev = torch.device("cuda:0")
    sysw = synth.workload_system(args.workload)
    F = synth.rhs_torch(w["seed"], N, M, K, dev)
    X = torch.empty_like(F)
    torch.cuda.synchronize()

    if args.copy_calibration > 0:
        n8 = args.copy_calibration // 8
        src_buf = torch.ones(n8, dtype=torch.float64, device=dev)
        dst_buf = torch.empty_like(src_buf)
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        del src_buf, dst_buf

    # a small factor of the same block size first: a process's first launches of the factor's
    # kernels load their code, a one-time cost that factor_ms leaves out
    wn = 64 if (M == 1 and p == N) else 16
    td.Plan.from_system(synth.varcoef_system(wn, M, 1), device=dev, subdomains=wn if M == 1 and p == N else 4).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = td.Plan.from_system(sysw, device=dev, subdomains=p)
    torch.cuda.synchronize()
    factor_ms = (time.perf_counter() - t0) * 1e3
    first_lib_ms = plan.plan_info()["factor_ms"]
    # the same factor again, its memory now in torch's cache (the first one also grows the cache):
    # the time of a repeated factor, e.g. after a change of the matrix
    plan.close()
    del plan
    t0 = time.perf_counter()
    plan = td.Plan.from_system(sysw, device=dev, subdomains=p)
    torch.cuda.synchronize()
    factor_repeat_ms = (time.perf_counter() - t0) * 1e3
    pinfo = plan.plan_info()
    progress(f"factor {factor_ms:.1f} ms, repeated {factor_repeat_ms:.1f} ms")

    _, info = plan.solve(F, X, info=True)
    # timed: plain solves, as a caller runs them (the library replays a captured HIP graph)
    for _ in range(args.warmup):
        plan.solve(F, X)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.solve(F, X)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = K / (ms_per_step / 1e3)
    # the same solves launched eagerly with HIP events around every stage (per-kernel times)
    plan.set_profiling(True)
    torch.cuda.synchronize()
    n_prof = max(1, min(args.steps, 10))
    t0 = time.perf_counter()
    for _ in range(n_prof):
        plan.solve(F, X)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3 / n_prof
    stages = plan.stage_times()
    plan.set_profiling(False)
    progress(f"float64 solves timed: {ms_per_step:.2f} ms per step")

    work = algorithmic_work(N, M, K, p)
    scalar = M == 1 and p == N
    if scalar:
        # Algorithm 1 on the scalar system: the subtree kernel reads F and writes X once (the HBM
        # bound; the stored inverse rows, 8 (depth) N bytes, stay in cache across column groups);
        # the top levels' kernels read F once more for the subtree parts of the top nodes' sums
        depth = max(1, int(N).bit_length())
        sub_bytes = 2.0 * 8 * N * K
        top_bytes = 8.0 * N * K
        sub_flops = 2.0 * N * K * depth
        kern = {"scalar_subtrees": (stages["dichotomy_levels"], sub_flops, sub_bytes),
                "scalar_top_levels": (stages["dichotomy_partial"], 2.0 * N * K * depth, top_bytes)}
        dom = "scalar_subtrees"
        t_ms, fl, by = kern[dom]
        achieved = by / (t_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM, "unit": "GB/s",
                    "frac": achieved / PEAK_HBM, "traffic": measured_traffic(dom, args.workload),
                    "algorithmic_flops_per_launch": fl, "algorithmic_bytes_per_launch": by,
                    "avg_launch_ms": t_ms}
        other = {k: {"avg_launch_ms": v[0], "gbs": v[2] / (v[0] * 1e-3) / 1e9} for k, v in kern.items()}
        args.mixed = ""
    else:
        kern = {
            "sweep": (stages["sweep"], work["sweep_flops"], work["sweep_bytes"]),
            "superposition": (stages["superposition"], work["sup_flops"], work["sup_bytes"]),
            "dichotomy": (stages["dichotomy_partial"] + stages["dichotomy_levels"], work["dich_flops"],
                          work["dich_bytes"]),
        }
        dom = max(kern, key=lambda k: kern[k][0])
        t_ms, fl, by = kern[dom]
        achieved = fl / (t_ms * 1e-3) / 1e12
        roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": PEAK_F64_MFMA, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_F64_MFMA, "traffic": measured_traffic(dom, args.workload),
                    "algorithmic_flops_per_launch": fl, "algorithmic_bytes_per_launch": by,
                    "avg_launch_ms": t_ms}
        other = {k: {"avg_launch_ms": v[0], "tflops": v[1] / (v[0] * 1e-3) / 1e12,
                     "frac_f64_peak": v[1] / (v[0] * 1e-3) / 1e12 / PEAK_F64_MFMA} for k, v in kern.items()}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "M": M, "K": K, "subdomains": p, "precision": "f64",
                   "coefficients": w["family"]},
        "roofline": roofline,
        "kernels": other,
        "stages_ms": {k: v for k, v in stages.items() if k != "count"},
        "whole_solve_tflops": (None if scalar else work["total_flops"] / (ms_per_step * 1e-3) / 1e12),
        "eager_profiled_ms_per_step": eager_ms,
        "factor_ms": factor_ms,
        "factor_repeat_ms": factor_repeat_ms,
        "max_col_rel_residual": info["max_col_rel_residual"],
        "plan_device_bytes": pinfo["device_bytes"],
    }
    if not scalar:
        # the factor's rate: its algorithmic flops over the library's own time of the repeated factor
        fw = factor_work(N, M, p)
        out["factor"] = {"ms_library_first": first_lib_ms, "ms_library": pinfo["factor_ms"],
                         "algorithmic_tflop": fw / 1e12, "tflops": fw / (pinfo["factor_ms"] * 1e-3) / 1e12,
                         "frac_f64_peak": fw / (pinfo["factor_ms"] * 1e-3) / 1e12 / PEAK_F64_MFMA}
    if args.workload.startswith("adjoint"):
        # one gradient step of a caller: forward solve, adjoint solve, diagonal-shift gradient
        del plan
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        aplan = td.Plan.from_system(sysw, device=dev, subdomains=p, adjoint=True)
        torch.cuda.synchronize()
        afac = (time.perf_counter() - t0) * 1e3
        G = synth.rhs_torch(w["seed"] + 1, N, M, K, dev)
        Lam = torch.empty_like(G)

        def grad_step():
            aplan.solve(F, X)
            aplan.solve_adjoint(G, Lam)
            return td.diag_grad(Lam, X)

        for _ in range(args.warmup):
            grad_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            grad_step()
        torch.cuda.synchronize()
        ams = (time.perf_counter() - t0) * 1e3 / args.steps
        out["adjoint"] = {"ms_forward_backward": ams, "rhs_per_s": K / (ams / 1e3), "factor_ms": afac,
                          "step": "forward solve + adjoint solve + diagonal-shift gradient, float64"}
        aplan.close()
        del aplan
        plan = None
    # mixed precision + float64 refinement to the same residual bar, same workload
    mixed = {}
    for prec in [m for m in args.mixed.split(",") if m]:
        del plan
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mplan = td.Plan.from_system(sysw, device=dev, subdomains=p, sweep_prec=prec)
        torch.cuda.synchronize()
        mfac = (time.perf_counter() - t0) * 1e3
        ref = {"tol": 1e-10, "max_iter": 20}
        _, minfo = mplan.solve(F, X, refine=ref, info=True)
        for _ in range(args.warmup):
            mplan.solve(F, X, refine=ref)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            mplan.solve(F, X, refine=ref)
        torch.cuda.synchronize()
        mel = time.perf_counter() - t0
        mms = mel * 1e3 / args.steps
        # stage times from separate, untimed solves with HIP events around every stage
        mplan.set_profiling(True)
        for _ in range(max(1, min(args.steps, 5))):
            mplan.solve(F, X, refine=ref)
        torch.cuda.synchronize()
        mst = mplan.stage_times()
        mplan.set_profiling(False)
        mixed[prec] = {"value": K / (mms / 1e3), "unit": "RHS/s", "ms_per_step": mms,
                       "speedup_vs_f64": ms_per_step / mms, "iterations": minfo["iterations"],
                       "max_col_rel_residual": minfo["max_col_rel_residual"], "factor_ms": mfac,
                       "last_pass_stages_ms": {k: v for k, v in mst.items() if k != "count"}}
        mplan.close()
        del mplan
        plan = None
        progress(f"{prec} + refinement timed: {mms:.2f} ms per step")
    out["mixed_refined"] = mixed
    if not args.no_cpu_baseline:
        import oracle

        # the scalar system's oracle (the Thomas algorithm) solves every row of the sample quickly
        rows = 0 if M == 1 else args.cpu_rows
        progress("oracle sample on the host")
        out["cpu_baseline"] = cpu_baseline(w, rows, args.cpu_cols, args.cpu_cols_1t, oracle.default_threads())
    print(json.dumps(out))


if __name__ == "__main__":
    main()

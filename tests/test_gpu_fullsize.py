"""Parity at the full workload sizes, in the launch configuration bench.py times.

The oracle cannot re-solve these sizes inside a test, so sampled entries of its solution are
stored in tests/golden/*.json (written by tests/golden/make_golden.py, which calls only the
oracle).  Every column is also checked by the float64 residual, a property at any size.
Bar: max |X - X_oracle| over the samples <= 1e-12 * max |X_oracle| for float64 solves;
<= 1e-9 for mixed precision refined to a relative residual of 1e-10.
"""
import json
import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1108_4181_amd as m

    m.load_library()
    return m


def _golden(name):
    path = os.path.join(HERE, "golden", f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


def _check_samples(X, gold, tol):
    worst = 0.0
    for smp in gold["samples"]:
        k = smp["column"]
        idx = torch.as_tensor(smp["index"], dtype=torch.int64, device=X.device)
        got = X[k].index_select(0, idx).cpu().numpy()
        ref = np.array([float(v) for v in smp["value"]])
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    assert worst <= tol, worst
    return worst


def _inputs(name):
    w = synth.WORKLOADS[name]
    sys = synth.workload_system(name)
    F = synth.rhs_torch(w["seed"], sys.N, sys.M, w["K"], "cuda")
    return w, sys, F


def test_device_generator_matches_host():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    w = synth.WORKLOADS["varcoef_n2048_m256_k512"]
    F = synth.rhs_torch(w["seed"], 2048, 256, 3, "cuda").cpu().numpy()
    ref = synth.rhs_columns(w["seed"], 2048, 256, range(3))
    assert np.array_equal(F, ref)


def test_varcoef_fullsize_f64(td):
    name = "varcoef_n2048_m256_k512"
    gold = _golden(name)
    w, sys, F = _inputs(name)
    plan = td.Plan.from_system(sys, subdomains=w["p"])
    X, info = plan.solve(F, info=True)
    assert info["max_col_rel_residual"] <= 1e-13 and info["nonfinite"] == 0
    _check_samples(X, gold, 1e-12)


def test_adjoint_workload_fullsize_forward_and_transpose(td):
    """The differentiation workload's matrix is symmetric, so P^{-T} F = P^{-1} F: the same samples
    pin both the forward and the transposed solve."""
    name = "adjoint_n1024_m256_k256"
    gold = _golden(name)
    w, sys, F = _inputs(name)
    plan = td.Plan.from_system(sys, subdomains=w["p"], adjoint=True)
    X = plan.solve(F)
    _check_samples(X, gold, 1e-12)
    Lam = plan.solve_adjoint(F)
    _check_samples(Lam, gold, 1e-12)


def test_mixed_workload_fullsize_f64(td):
    """The 4096 x 512 workload (K = 1024, 128 subdomains) solved in float64 as bench.py times it
    (plain solve, replayed graph): samples against the oracle <= 1e-12, every column's residual
    <= 1e-13 (checked by an eager solve with a report on the same plan)."""
    name = "mixed_n4096_m512_k1024"
    gold = _golden(name)
    w, sys, F = _inputs(name)
    plan = td.Plan.from_system(sys, subdomains=w["p"])
    X = torch.empty_like(F)
    plan.solve(F, X)                       # captured
    plan.solve(F, X)                       # replayed
    torch.cuda.synchronize()
    _check_samples(X, gold, 1e-12)
    Y, info = plan.solve(F, info=True)
    assert info["max_col_rel_residual"] <= 1e-13 and info["nonfinite"] == 0
    assert torch.equal(X, Y)
    del plan, X, Y, F
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_fullsize_refined(td, prec):
    name = "mixed_n4096_m512_k1024"
    gold = _golden(name)
    w, sys, F = _inputs(name)
    plan = td.Plan.from_system(sys, subdomains=w["p"], sweep_prec=prec)
    X, info = plan.solve(F, refine={"tol": 1e-10, "max_iter": 20}, info=True)
    assert info["converged"] and info["max_col_rel_residual"] <= 1e-10
    _check_samples(X, gold, 1e-9)
    del plan, X, F
    torch.cuda.empty_cache()

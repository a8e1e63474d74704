"""Mixed precision (float32 / bfloat16 sweeps and superposition, float64 pivots, reduced system
and residual) with float64 iterative refinement, through the C ABI, against the CPU oracle.

Bars: after refinement the max column relative residual is <= 1e-10 (checked by the library in
float64 and recomputed here with the oracle's P X), and the error vs the float64 oracle is within
the conditioning of the system (<= 1e-9 relative).  Without refinement the float32 path carries
its rounding error only (<= 1e-4 relative).
"""
import numpy as np
import pytest

import oracle
import synth
from dense_ref import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1108_4181_amd as m

    m.load_library()
    return m


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _colres(sys, X, F):
    R = F - oracle.apply(sys, X)
    return float(np.max(np.linalg.norm(R, axis=1) / np.linalg.norm(F, axis=1)))


@pytest.mark.parametrize("prec,maxit", [("f32", 3), ("bf16", 10)])
@pytest.mark.parametrize("N,M,K,p", [(128, 64, 20, 8), (64, 16, 8, 4), (96, 48, 37, 6), (48, 256, 70, 4),
                                     (40, 224, 33, 5), (24, 320, 17, 3), (20, 384, 100, 4), (12, 512, 70, 3)])
def test_refined_to_1e10(td, prec, maxit, N, M, K, p):
    """(The last two: float32 above block size 256 with more than 32 columns, whose first pass runs the
    superposition with half of the interface panel in LDS: one full and one ragged 64-column tile.)"""
    sys = synth.varcoef_system(N, M, seed=200 + N + M)
    F = synth.rhs_columns(200 + N, N, M, range(K))
    plan = td.Plan.from_system(sys, subdomains=p, sweep_prec=prec)
    X, info = plan.solve(_dev(F), refine={"tol": 1e-10, "max_iter": maxit}, info=True)
    X = X.cpu().numpy()
    assert info["converged"] and info["max_col_rel_residual"] <= 1e-10
    assert info["iterations"] <= maxit
    assert _colres(sys, X, F) <= 1e-10
    assert rel_err(X, oracle.solve(sys, F)) <= 1e-9


def test_f32_without_refinement(td):
    sys = synth.workload_system("tiny_n64_m16_k8")
    F = synth.rhs_columns(1, 64, 16, range(8))
    plan = td.Plan.from_system(sys, subdomains=4, sweep_prec="f32")
    X = plan.solve(_dev(F)).cpu().numpy()
    err = rel_err(X, oracle.solve(sys, F))
    assert 1e-12 < err <= 1e-4     # float32 rounding is visible, and small


def test_refinement_counts(td):
    """float32 needs at most 2 correction passes to 1e-10 on a well conditioned system;
    bfloat16 needs more than float32."""
    sys = synth.varcoef_system(128, 128, seed=33)
    F = synth.rhs_columns(33, 128, 128, range(16))
    its = {}
    for prec in ("f32", "bf16"):
        plan = td.Plan.from_system(sys, subdomains=8, sweep_prec=prec)
        _, info = plan.solve(_dev(F), refine={"tol": 1e-10, "max_iter": 12}, info=True)
        assert info["converged"]
        its[prec] = info["iterations"]
    assert its["f32"] <= 2
    assert its["bf16"] > its["f32"]


def test_f64_plan_refine_is_noop(td):
    sys = synth.varcoef_system(64, 32, seed=34)
    F = synth.rhs_columns(34, 64, 32, range(5))
    plan = td.Plan.from_system(sys, subdomains=4)
    _, info = plan.solve(_dev(F), refine=True, info=True)
    assert info["iterations"] == 0 and info["max_col_rel_residual"] < 1e-14


@pytest.mark.parametrize("N,M,K,p", [(70, 40, 37, 6), (20, 384, 40, 4)])
def test_f64_correction_pass_adds_to_x(td, N, M, K, p):
    """An unreachable tolerance forces one correction pass on a float64 plan: the superposition and
    the dichotomy's last level then add to X (their accumulating forms; above block size 256 the
    adding superposition is the 16-column kernel, the writing one the half-panel 32-column kernel),
    and X must stay the float64 solution."""
    sys = synth.varcoef_system(N, M, seed=36)
    F = synth.rhs_columns(36, N, M, range(K))
    plan = td.Plan.from_system(sys, subdomains=p)
    X, info = plan.solve(_dev(F), refine={"tol": 1e-300, "max_iter": 1}, info=True)
    assert info["iterations"] == 1 and not info["converged"]
    assert rel_err(X.cpu().numpy(), oracle.solve(sys, F)) < 1e-12


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("N,M,K,p", [(3, 1, 1, 1), (9, 5, 1, 3), (12, 33, 2, 4)])
def test_refined_degenerate_sizes(td, prec, N, M, K, p):
    sys = synth.varcoef_system(N, M, seed=300 + N + M)
    F = synth.rhs_columns(300 + N + M, N, M, range(K))
    plan = td.Plan.from_system(sys, subdomains=p, sweep_prec=prec)
    X, info = plan.solve(_dev(F), refine={"tol": 1e-10, "max_iter": 12}, info=True)
    assert info["converged"] and info["max_col_rel_residual"] <= 1e-10
    assert rel_err(X.cpu().numpy(), oracle.solve(sys, F)) < 1e-9


def test_noconvergence_reported(td):
    """max_iter = 1 with a bfloat16 plan cannot reach 1e-14: TD_ENOCONV (reported through info)."""
    sys = synth.varcoef_system(64, 32, seed=35)
    F = synth.rhs_columns(35, 64, 32, range(4))
    plan = td.Plan.from_system(sys, subdomains=4, sweep_prec="bf16")
    _, info = plan.solve(_dev(F), refine={"tol": 1e-14, "max_iter": 1}, info=True)
    assert not info["converged"] and info["iterations"] == 1
    with pytest.raises(td.TridiagError) as e:
        plan.solve(_dev(F), refine={"tol": 1e-14, "max_iter": 1})
    assert e.value.code == 4


def test_plan_bytes_count_released_buffers(td):
    """A float32 plan releases its float64 sweep matrices after rounding them, so it holds less
    device memory than the float64 plan of the same system (the report counts held memory)."""
    sys = synth.varcoef_system(96, 64, seed=36)
    b64 = td.Plan.from_system(sys, subdomains=6).plan_info()["device_bytes"]
    b32 = td.Plan.from_system(sys, subdomains=6, sweep_prec="f32").plan_info()["device_bytes"]
    assert 0 < b32 < b64

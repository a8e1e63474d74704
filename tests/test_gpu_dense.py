"""Dense coupling blocks A_j, B_j (format DENSE) on the GPU against the CPU oracle.

With a dense A or B every coupling of Algorithm 2 is a block product: D_i = C_i - A_i alpha_{i-1},
alpha_i = D_i^{-1} B_i, Gamma_i = D_i^{-1} A_i Gamma_{i-1}, the reduced blocks of eq. (red1), the
interface right-hand side and the forward sweep (as the recurrence beta_i = E_i beta_{i-1} +
D_i^{-1} F_i with E_i = D_i^{-1} A_i).  Float64, relative error <= 1e-12; shapes cover ragged
block sizes (padded internally), one subdomain, every row an interface, mixed formats, the
transposed solve and the low-precision rejection.
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


def _mixed(sys, which):
    """Replace A or B of a dense system by its diagonal (format DIAG)."""
    N, M = sys.N, sys.M
    diag = lambda X: np.ascontiguousarray(np.stack([np.diagonal(X[j]) for j in range(N)]))
    A, fA = (diag(sys.A), "diag") if which == "A" else (sys.A, "dense")
    B, fB = (diag(sys.B), "diag") if which == "B" else (sys.B, "dense")
    return synth.System(N, M, A, B, sys.C, fA, fB, sys.fmt_C)


@pytest.mark.parametrize("N,M,K,p", [
    (24, 16, 5, 4), (37, 50, 9, 6), (64, 48, 33, 8), (33, 32, 7, 1), (12, 16, 4, 12), (70, 64, 40, 9),
])
def test_dense_matches_oracle(td, N, M, K, p):
    sys = synth.dense_system(N, M, seed=700 + N)
    F = synth.rhs_columns(700 + N, N, M, range(K))
    plan = td.Plan.from_system(sys, subdomains=p)
    X = plan.solve(_dev(F)).cpu().numpy()
    assert rel_err(X, oracle.solve(sys, F)) <= 1e-12


@pytest.mark.parametrize("which", ["A", "B"])
def test_dense_mixed_formats(td, which):
    sys = _mixed(synth.dense_system(45, 32, seed=811), which)
    F = synth.rhs_columns(811, 45, 32, range(11))
    plan = td.Plan.from_system(sys, subdomains=5)
    X = plan.solve(_dev(F)).cpu().numpy()
    assert rel_err(X, oracle.solve(sys, F)) <= 1e-12


def test_dense_tridiagonal_C(td):
    base = synth.dense_system(40, 24, seed=823)
    C = np.zeros((40, 3, 24))
    C[:, 0, 1:] = -1.0
    C[:, 1, :] = 5.0
    C[:, 2, :-1] = -1.0
    sys = synth.System(40, 24, base.A, base.B, C, "dense", "dense", "tridiag")
    F = synth.rhs_columns(823, 40, 24, range(6))
    plan = td.Plan.from_system(sys, subdomains=4)
    X = plan.solve(_dev(F)).cpu().numpy()
    assert rel_err(X, oracle.solve(sys, F)) <= 1e-12


def test_dense_adjoint_and_residual(td):
    sys = synth.dense_system(50, 40, seed=831)
    F = synth.rhs_columns(831, 50, 40, range(8))
    G = synth.rhs_columns(832, 50, 40, range(8))
    plan = td.Plan.from_system(sys, subdomains=5, adjoint=True)
    X, info = plan.solve(_dev(F), info=True)
    assert info["max_col_rel_residual"] <= 1e-13
    Lam = plan.solve_adjoint(_dev(G)).cpu().numpy()
    assert rel_err(Lam, oracle.solve_adjoint(sys, G)) <= 1e-12
    lhs, rhs = float(np.sum(X.cpu().numpy() * G)), float(np.sum(F * Lam))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_dense_needs_float64(td):
    sys = synth.dense_system(16, 16, seed=841)
    with pytest.raises(td.TridiagError) as e:
        td.Plan.from_system(sys, subdomains=2, sweep_prec="f32")
    assert e.value.code == 7


def test_dense_singular_block_reported(td):
    sys = synth.dense_system(20, 16, seed=851)
    C = sys.C.copy()
    C[9] = 0.0   # an interior row of subdomain 1 of 4 (rows 5..9: interface 5, interior 6..9)
    sing = synth.System(20, 16, np.zeros_like(sys.A), np.zeros_like(sys.B), C, "dense", "dense", "dense")
    with pytest.raises(td.TridiagError) as e:
        td.Plan.from_system(sing, subdomains=4)
    assert e.value.code == 3

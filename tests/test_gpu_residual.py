"""The float64 stencil residual (diagonal A, B; tridiagonal C) that drives refinement and the
reported max column relative residual, against the oracle's P X.

A bfloat16 plan solved without refinement leaves a residual near 1e-3, so the value the library
reports measures its residual kernel, not rounding noise: it must agree with
max_k ||F_k - P X_k|| / ||F_k|| computed from the oracle's P X to 1e-9 relative.  Shapes cover a
single row per block (M = 1), a single block row (N = 1), row counts that leave a partial
work-group of rows, column counts that leave a partial group of columns, and the largest block
size (M = 512).  Coefficients that the problem ignores (A of the first block row, B of the last,
the corner entries of the tridiagonal C) are planted with large values: results must not see them.
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


def _planted(N, M, seed):
    """A variable-coefficient system whose ignored coefficients hold 1e6."""
    s = synth.varcoef_system(N, M, seed=seed)
    A, B, C = s.A.copy(), s.B.copy(), s.C.copy()
    A[0, :] = 1e6
    B[N - 1, :] = 1e6
    C[:, 0, 0] = 1e6          # sub-diagonal entry of each block's first row
    C[:, 2, M - 1] = 1e6      # super-diagonal entry of each block's last row
    return synth.System(N, M, A, B, C, s.fmt_A, s.fmt_B, s.fmt_C)


@pytest.mark.parametrize("N,M,K,p", [
    (3, 1, 1, 1), (1, 5, 3, 1), (7, 300, 17, 2), (9, 512, 33, 3), (40, 64, 16, 4), (33, 96, 50, 5),
])
def test_reported_residual_matches_oracle(td, N, M, K, p):
    sys = _planted(N, M, seed=900 + N + M)
    F = synth.rhs_columns(900 + N, N, M, range(K))
    plan = td.Plan.from_system(sys, subdomains=p, sweep_prec="bf16")
    X, info = plan.solve(_dev(F), info=True)
    ref = _colres(sys, X.cpu().numpy(), F)
    assert ref > 1e-8 or N * M < 8       # the unrefined bfloat16 residual is far above rounding noise
    assert abs(info["max_col_rel_residual"] - ref) <= 1e-9 * ref + 1e-16


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ignored_coefficients_do_not_reach_results(td, prec):
    N, M, K, p = 48, 40, 19, 4
    sys = _planted(N, M, seed=951)
    F = synth.rhs_columns(951, N, M, range(K))
    plan = td.Plan.from_system(sys, subdomains=p, sweep_prec=prec)
    X, info = plan.solve(_dev(F), refine={"tol": 1e-10, "max_iter": 4}, info=True)
    X = X.cpu().numpy()
    assert info["converged"] and info["max_col_rel_residual"] <= 1e-10
    assert _colres(sys, X, F) <= 1e-10
    assert rel_err(X, oracle.solve(sys, F)) <= (1e-12 if prec == "f64" else 1e-9)

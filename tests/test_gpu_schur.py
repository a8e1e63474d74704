"""Schur-complement solver on interface block rows (Sec. 3, eqs. (schur_decomp) and
(domains_equation)) on the GPU, through the C ABI, against the CPU oracle.

* tridiag_schur_apply against the oracle's dense S = A_GG - A_GI A_II^{-1} A_IG: <= 1e-12 relative.
* tridiag_schur_solve (CG on the interface system, tol 1e-12) against the oracle's block-Thomas
  solution of the whole system: <= 1e-9 relative (the CG stopping test bounds the interface
  residual; the conditioning of the systems here keeps the error within 1e-9).
Shapes cover one row per block (M = 1), strips of one interior row, uneven strips, no
preconditioner, several band widths, and many columns with a ragged count.  Nonsymmetric
matrices are rejected (CG needs a symmetric P).
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


def sym_varcoef(N, M, seed):
    """Symmetric, diagonally dominant: B_j = A_{j+1} = diag(b_j), C_j symmetric tridiagonal with
    varying off-diagonals."""
    u = synth.uniform_range(seed, 11, 0, 4 * N * M).reshape(4, N, M)
    b = 0.5 + 0.5 * u[0]
    A = np.empty((N, M))
    A[0] = 0.0
    A[1:] = b[:-1]
    B = b.copy()
    e = 0.2 + 0.8 * u[1]                       # |C_j(r, r-1)| = |C_j(r-1, r)| = e[j, r]
    C = np.zeros((N, 3, M))
    C[:, 0, 1:] = -e[:, 1:]
    C[:, 2, :-1] = -e[:, 1:]
    C[:, 1, :] = 2.0 + 2.0 * np.maximum(e, np.roll(e, -1, axis=1)) + 0.1 + u[2]
    return synth.System(N, M, A, B, C)


def _solver(td, sys, icol, band):
    return td.SchurSolver(_dev(sys.A), _dev(sys.B), _dev(sys.C), icol, band=band)


@pytest.mark.parametrize("N,M,icol,family", [
    (13, 6, [4, 8], "laplace"), (30, 16, [3, 10, 21, 27], "sym"), (9, 1, [2, 6], "laplace"), (21, 33, [1, 19], "sym"),
])
def test_apply_matches_oracle(td, N, M, icol, family):
    sys = synth.laplace_system(N, M, 4.5) if family == "laplace" else sym_varcoef(N, M, 71 + N)
    S = oracle.schur_complement(sys, icol)
    V = synth.uniform_range(72, 3, 0, 5 * len(icol) * M, -1.0, 1.0).reshape(5, len(icol) * M)
    s = _solver(td, sys, icol, -1)
    Y = s.apply(_dev(V)).cpu().numpy()
    assert rel_err(Y, V @ S.T) <= 1e-12


@pytest.mark.parametrize("N,M,icol,band,K,family", [
    (61, 16, [10, 20, 35, 50], 2, 7, "sym"),
    (129, 64, [16, 32, 48, 64, 80, 96, 112], 4, 9, "laplace"),
    (40, 1, [5, 15, 30], 0, 3, "sym"),
    (50, 32, [7, 30], -1, 4, "sym"),
    (24, 48, [2, 4, 6, 8, 10, 12, 14, 16, 18, 20], 3, 37, "laplace"),
])
def test_solve_matches_oracle(td, N, M, icol, band, K, family):
    sys = synth.laplace_system(N, M, 4.5) if family == "laplace" else sym_varcoef(N, M, 81 + N)
    F = synth.rhs_columns(82 + N, N, M, range(K))
    s = _solver(td, sys, icol, band)
    X, info = s.solve(_dev(F), tol=1e-12, info=True)
    assert info["converged"] and info["active"] == 0 and info["max_rel_residual"] <= 1e-12
    assert rel_err(X.cpu().numpy(), oracle.solve(sys, F)) <= 1e-9


def test_probing_reduces_iterations(td):
    """The probed band preconditioner cuts the CG iterations of the 5-point Laplacian's
    interface system (whose condition number grows with the block size)."""
    N, M = 127, 128
    icol = [15, 31, 47, 63, 79, 95, 111]
    sys = synth.laplace_system(N, M, 4.01)
    F = synth.rhs_columns(91, N, M, range(4))
    its = {}
    for band in (-1, 4):
        s = _solver(td, sys, icol, band)
        X, info = s.solve(_dev(F), tol=1e-10, info=True)
        assert info["converged"]
        assert rel_err(X.cpu().numpy(), oracle.solve(sys, F)) <= 1e-8
        its[band] = info["iterations"]
    assert its[4] < its[-1]


def test_nonsymmetric_rejected(td):
    sys = synth.varcoef_system(20, 8, seed=93)      # A_{j+1} != B_j
    with pytest.raises(td.TridiagError) as e:
        _solver(td, sys, [5, 12], 2)
    assert e.value.code == 1


def test_zero_rhs_and_repeated_solves(td):
    sys = sym_varcoef(33, 24, 95)
    icol = [8, 16, 24]
    s = _solver(td, sys, icol, 2)
    Z = np.zeros((3, 33 * 24))
    X, info = s.solve(_dev(Z), info=True)
    assert info["iterations"] <= 1 and np.all(X.cpu().numpy() == 0.0)
    for K in (5, 2):   # the workspace of the larger call serves the smaller one
        F = synth.rhs_columns(96 + K, 33, 24, range(K))
        X = s.solve(_dev(F), tol=1e-12)
        assert rel_err(X.cpu().numpy(), oracle.solve(sys, F)) <= 1e-9

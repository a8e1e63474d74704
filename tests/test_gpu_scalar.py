"""Algorithm 1 (Sec. 2.1) on a scalar tridiagonal system: block size 1 with every row an interface
row (subdomains = N) runs the scalar dichotomy (stored inverse rows per tree node, levels from the
root), not padded blocks.  Parity with the CPU oracle's scalar block-Thomas (Thomas algorithm) at
1e-12: sizes below and above the subtree size (1024 rows, one and several top levels), ragged column
counts, both coefficient families, a dense-format C, the transposed solve, refinement reports, and
the 65536-row, 1024-right-hand-side case (sampled columns against the oracle, every column by its
residual)."""
import numpy as np
import pytest

import oracle
import synth
from dense_ref import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1108_4181_amd as m

    m.load_library()
    return m


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _system(N, seed, family):
    return synth.varcoef_system(N, 1, seed) if family == "varcoef" else synth.laplace_system(N, 1, 2.5)


@pytest.mark.parametrize("N", [1, 2, 3, 7, 64, 1023, 1024, 1025, 3000, 9000])
@pytest.mark.parametrize("K", [1, 6])
def test_scalar_dichotomy_matches_oracle(td, N, K):
    sys = _system(N, 900 + N, "varcoef")
    F = synth.rhs_columns(900 + N + K, N, 1, range(K))
    plan = td.Plan.from_system(sys, subdomains=N)
    info = plan.plan_info()
    assert info["Mp"] == 1 and info["subdomains"] == N
    X = plan.solve(_dev(F)).cpu().numpy()
    assert rel_err(X, oracle.solve(sys, F)) < TOL


@pytest.mark.parametrize("K", [3, 4, 5, 33])
def test_scalar_column_groups(td, K):
    """Column counts around the four-column groups of the subtree kernels; laplace coefficients."""
    N = 2500
    sys = _system(N, 0, "laplace")
    F = synth.rhs_columns(950 + K, N, 1, range(K))
    plan = td.Plan.from_system(sys, subdomains=N)
    X = plan.solve(_dev(F)).cpu().numpy()
    assert rel_err(X, oracle.solve(sys, F)) < TOL


def test_scalar_columns_beyond_one_launch(td):
    """More right-hand sides than one launch's column groups hold (65535 groups of four): the solve
    runs in column chunks; columns on both sides of the chunk boundary against the oracle."""
    N, K = 64, 65535 * 4 + 41
    sys = _system(N, 77, "varcoef")
    F = synth.rhs_torch(977, N, 1, K, "cuda")
    plan = td.Plan.from_system(sys, subdomains=N)
    X = plan.solve(F)
    cols = [0, 1, 65535 * 4 - 1, 65535 * 4, 65535 * 4 + 1, K - 1]
    got = X[cols].cpu().numpy()
    assert rel_err(got, oracle.solve(sys, synth.rhs_columns(977, N, 1, cols))) < TOL
    del X, F
    torch.cuda.empty_cache()


def test_scalar_dense_c_and_adjoint(td):
    N, K = 1500, 5
    base = synth.varcoef_system(N, 1, 960)
    C = np.ascontiguousarray(base.C[:, 1, :].reshape(N, 1, 1))      # 1 x 1 blocks, dense format
    sys = synth.System(N, 1, base.A, base.B, C, "diag", "diag", "dense")
    F = synth.rhs_columns(961, N, 1, range(K))
    G = synth.rhs_columns(962, N, 1, range(K))
    plan = td.Plan.from_system(sys, subdomains=N, adjoint=True)
    assert rel_err(plan.solve(_dev(F)).cpu().numpy(), oracle.solve(sys, F)) < TOL
    assert rel_err(plan.solve_adjoint(_dev(G)).cpu().numpy(), oracle.solve_adjoint(sys, G)) < TOL


def test_scalar_refinement_report(td):
    N, K = 4000, 7
    sys = _system(N, 970, "varcoef")
    F = synth.rhs_columns(970, N, 1, range(K))
    plan = td.Plan.from_system(sys, subdomains=N)
    X, info = plan.solve(_dev(F), refine=True, info=True)
    assert info["max_col_rel_residual"] <= 1e-14 and info["iterations"] == 0
    assert rel_err(X.cpu().numpy(), oracle.solve(sys, F)) < TOL


def test_scalar_singular_reported(td):
    sys = _system(100, 980, "varcoef")
    C = sys.C.copy()
    C[:, 1, 0] = 0.0                     # c_j = 0 and a_j = b_j: the tree's pivots vanish
    A = np.zeros_like(sys.A)
    with pytest.raises(td.TridiagError) as e:
        td.Plan.from_system(synth.System(100, 1, A, A.copy(), C), subdomains=100)
    assert e.value.code == 3


def _stencil_residual_scalar(sys, X, F):
    a = torch.as_tensor(sys.A[:, 0], device=X.device)
    b = torch.as_tensor(sys.B[:, 0], device=X.device)
    c = torch.as_tensor(sys.C[:, 1, 0], device=X.device)
    px = c * X
    px[:, 1:] -= a[1:] * X[:, :-1]
    px[:, :-1] -= b[:-1] * X[:, 1:]
    return float(((F - px).norm(dim=1) / F.norm(dim=1)).max())


def test_scalar_fullsize(td):
    """N = 65536 rows, K = 1024 right-hand sides, every row an interface (the bench's scalar
    workload): 8 columns against the oracle, every column's residual <= 1e-14."""
    w = synth.WORKLOADS["scalar_n65536_k1024"]
    sys = synth.workload_system("scalar_n65536_k1024")
    F = synth.rhs_torch(w["seed"], sys.N, 1, w["K"], "cuda")
    plan = td.Plan.from_system(sys, subdomains=sys.N)
    X = torch.empty_like(F)
    plan.solve(F, X)
    plan.solve(F, X)
    torch.cuda.synchronize()
    cols = [0, 1, 3, 4, 511, 512, 1022, 1023]
    Fh = synth.rhs_columns(w["seed"], sys.N, 1, cols)
    assert rel_err(X[cols].cpu().numpy(), oracle.solve(sys, Fh)) < TOL
    assert _stencil_residual_scalar(sys, X, F) <= 1e-14

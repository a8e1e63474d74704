"""Parity of the HIP float64 path (through the C ABI) with the CPU oracle.

Tolerance: relative Frobenius error <= 1e-12 against the oracle for every float64
solve (the method is direct; both sides only differ in rounding order).
"""
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


def _solve(td, sys, F, p, **kw):
    plan = td.Plan.from_system(sys, subdomains=p, **kw)
    X = plan.solve(_dev(F)).cpu().numpy()
    return plan, X


def test_tiny_workload(td):
    w = synth.WORKLOADS["tiny_n64_m16_k8"]
    sys = synth.workload_system("tiny_n64_m16_k8")
    F = synth.rhs_columns(w["seed"], sys.N, sys.M, range(w["K"]))
    _, X = _solve(td, sys, F, w["p"])
    assert rel_err(X, oracle.solve(sys, F)) < TOL


@pytest.mark.parametrize("N,M,K,p", [
    (37, 16, 5, 6),      # uneven partition
    (40, 16, 3, 1),      # one subdomain: the reduced system is C~_0 only
    (24, 16, 2, 24),     # p = N: every row an interface row (Algorithm 1 on P itself)
    (50, 32, 33, 7),     # ragged column tail (33 = 32 + 1)
    (64, 20, 9, 5),      # M not a multiple of 16 (padded block)
    (96, 64, 40, 8),     # several row tiles per wave group
])
def test_varcoef_shapes(td, N, M, K, p):
    sys = synth.varcoef_system(N, M, seed=100 + N)
    F = synth.rhs_columns(100 + N, N, M, range(K))
    _, X = _solve(td, sys, F, p)
    assert rel_err(X, oracle.solve(sys, F)) < TOL


@pytest.mark.parametrize("N,M,K,p", [
    (1, 1, 1, 1),        # one block row: the reduced system is the whole problem
    (2, 1, 1, 2),        # scalar blocks, every row an interface
    (3, 1, 2, 1),        # scalar blocks, one subdomain with interior rows
    (5, 3, 1, 2),        # one right-hand side (column indices clamp to 0 in the epilogues)
    (7, 17, 1, 3),       # one row beyond a 16-row tile (padded to 32)
])
def test_degenerate_sizes(td, N, M, K, p):
    sys = synth.varcoef_system(N, M, seed=200 + N + M)
    F = synth.rhs_columns(200 + N + M, N, M, range(K))
    _, X = _solve(td, sys, F, p)
    assert rel_err(X, oracle.solve(sys, F)) < TOL


@pytest.mark.parametrize("M", [16, 48, 96, 256])
@pytest.mark.parametrize("K", [8, 16, 17, 64])
def test_tile_forms(td, M, K):
    """Every (row tiles, column tiles) form of the sweep and superposition kernels: blocks padded to
    16, 48, 96 and 256 rows (one, two and four row tiles per wave) and 8, 16, 17 and 64 columns
    (8-, 16- and 32-column tiles, one ragged); the LDS operand layout of each form is exercised."""
    N, p = 24, 4
    sys = synth.varcoef_system(N, M, seed=400 + M + K)
    F = synth.rhs_columns(400 + M + K, N, M, range(K))
    _, X = _solve(td, sys, F, p)
    assert rel_err(X, oracle.solve(sys, F)) < TOL


def test_block_150(td):
    """M = 150 (one of the paper's block sizes): padded to 160."""
    sys = synth.varcoef_system(48, 150, seed=7)
    F = synth.rhs_columns(7, 48, 150, range(10))
    _, X = _solve(td, sys, F, 6)
    assert rel_err(X, oracle.solve(sys, F)) < TOL


def test_m256_moderate(td):
    sys = synth.varcoef_system(128, 256, seed=8)
    F = synth.rhs_columns(8, 128, 256, range(40))
    _, X = _solve(td, sys, F, 8)
    assert rel_err(X, oracle.solve(sys, F)) < TOL


def test_residual_info_and_determinism(td):
    sys = synth.varcoef_system(64, 32, seed=9)
    F = synth.rhs_columns(9, 64, 32, range(12))
    plan = td.Plan.from_system(sys, subdomains=4)
    Fd = _dev(F)
    X1, info = plan.solve(Fd, info=True)
    X2 = plan.solve(Fd)
    assert torch.equal(X1, X2)
    assert info["max_col_rel_residual"] < 1e-13 and info["nonfinite"] == 0


def test_singular_reported(td):
    """A zero block C_i on the first interior row of a subdomain makes the first pivot block of that
    subdomain's sub-problems (eqs. sub1-sub3) zero: the factor must stop with TD_ESINGULAR."""
    sys = synth.varcoef_system(16, 16, seed=10)
    C = sys.C.copy()
    C[9] = 0.0                     # p = 2: interface rows 0 and 8, row 9 opens subdomain 1
    bad = synth.System(16, 16, sys.A, sys.B, C)
    with pytest.raises(td.TridiagError) as e:
        td.Plan.from_system(bad, subdomains=2)
    assert e.value.code == 3 and "block row 9" in str(e.value)


def test_nan_input_reported(td):
    sys = synth.varcoef_system(16, 16, seed=13)
    C = sys.C.copy()
    C[3, 1, 4] = np.nan
    with pytest.raises(td.TridiagError) as e:
        td.Plan.from_system(synth.System(16, 16, sys.A, sys.B, C), subdomains=2)
    assert e.value.code == 3


def test_adjoint_nonsymmetric(td):
    sys = synth.varcoef_system(40, 16, seed=11)
    G = synth.rhs_columns(11, 40, 16, range(6))
    plan = td.Plan.from_system(sys, subdomains=5, adjoint=True)
    Lam = plan.solve_adjoint(_dev(G)).cpu().numpy()
    assert rel_err(Lam, oracle.solve_adjoint(sys, G)) < TOL


def test_zero_columns(td):
    sys = synth.varcoef_system(16, 16, seed=12)
    plan = td.Plan.from_system(sys, subdomains=2)
    X = plan.solve(torch.empty((0, 256), dtype=torch.float64, device="cuda"))
    assert X.shape == (0, 256)


def test_solve_graph_replays_match_eager(td):
    """Plain solves replay a captured HIP graph: every replay, with eager work of the same plan
    between replays, equals the eager solve bitwise; new arguments or more columns recapture."""
    sys = synth.varcoef_system(96, 48, seed=71)
    F1 = _dev(synth.rhs_columns(71, 96, 48, range(9)))
    F2 = _dev(synth.rhs_columns(72, 96, 48, range(9)))
    plan = td.Plan.from_system(sys, subdomains=6)
    ref1, _ = plan.solve(F1, info=True)          # eager path (a report is requested)
    ref2, _ = plan.solve(F2, info=True)
    ref1, ref2 = ref1.clone(), ref2.clone()
    X = torch.empty_like(F1)
    for _ in range(3):
        X.zero_()
        plan.solve(F1, X)                         # captured once, then replayed
        torch.cuda.synchronize()
        assert torch.equal(X, ref1)
        Y, _ = plan.solve(F2, info=True)          # eager work of the same plan in between
        assert torch.equal(Y, ref2)
    Z = plan.solve(F2)                            # other arguments: a new capture
    assert torch.equal(Z, ref2)
    F3 = _dev(synth.rhs_columns(73, 96, 48, range(20)))   # more columns: workspace grows, recapture
    ref3, _ = plan.solve(F3, info=True)
    assert torch.equal(plan.solve(F3), ref3)
    assert rel_err(X.cpu().numpy(), oracle.solve(sys, F1.cpu().numpy())) <= TOL


@pytest.mark.parametrize("M", [288, 384, 448, 512])
@pytest.mark.parametrize("K", [17, 40])
def test_large_blocks_f64(td, M, K):
    """Block sizes above 256 (padded to 320, 384, 448 and 512): the superposition with half of the
    interface panel in LDS at a time (32-column tiles, lanes beyond K in the ragged tile) and the
    sweep with five to eight waves of 64 rows, which the 4096 x 512 workload's float64 solve runs;
    one full and one ragged 32-column tile."""
    N, p = 20, 4
    sys = synth.varcoef_system(N, M, seed=500 + M + K)
    F = synth.rhs_columns(500 + M + K, N, M, range(K))
    _, X = _solve(td, sys, F, p)
    assert rel_err(X, oracle.solve(sys, F)) < TOL


def test_large_block_laplace_f64(td):
    """The 4096 x 512 workload's coefficients (C = tridiag(-1, 4.5, -1), A = B = I) at a small N with
    the same subdomain length (32 rows) and 64 right-hand sides."""
    sys = synth.laplace_system(96, 512, 4.5)
    F = synth.rhs_columns(31, 96, 512, range(64))
    _, X = _solve(td, sys, F, 3)
    assert rel_err(X, oracle.solve(sys, F)) < TOL


def _pivoting_system(N, M, seed):
    """Dense blocks whose elimination needs row interchanges: C_j is a strictly diagonally dominant
    matrix with its rows cyclically shifted by M // 3 (so its diagonal is small and every pivot comes
    from another row), A_j and B_j small dense blocks (entries U[-1, 1] / (8 M))."""
    base = synth.dense_system(N, M, seed, dominance=2.0)
    C = np.empty_like(base.C)
    for j in range(N):
        rowmajor = base.C[j].T                     # stored column-major
        C[j] = np.roll(rowmajor, M // 3, axis=0).T
    return synth.System(N, M, base.A / 8.0, base.B / 8.0, np.ascontiguousarray(C), "dense", "dense", "dense")


@pytest.mark.parametrize("M", [64, 128, 192, 256, 320, 448, 512])
def test_row_interchanges_in_block_inverses(td, M):
    """Every diagonal block of the elimination needs row interchanges (Gauss-Jordan with partial
    pivoting inside each block), at the block sizes of the one-launch-per-panel Gauss-Jordan kernel
    (multiples of 64 from 128) and below it."""
    N, K, p = 9, 6, 3
    sys = _pivoting_system(N, M, 700 + M)
    F = synth.rhs_columns(700 + M, N, M, range(K))
    _, X = _solve(td, sys, F, p)
    assert rel_err(X, oracle.solve(sys, F)) < 1e-11


@pytest.mark.parametrize("M", [128, 256, 512])
def test_nan_input_reported_large(td, M):
    """A NaN on the diagonal of a subdomain's C block, in the last panel of the per-panel
    Gauss-Jordan kernel: the factor reports TD_ESINGULAR (a NaN pivot candidate ranks first)."""
    sys = synth.varcoef_system(12, M, seed=40 + M)
    C = sys.C.copy()
    C[8, 1, M - 3] = np.nan        # row M - 3 of block row 8 (tridiagonal format: sub, diag, super)
    with pytest.raises(td.TridiagError) as e:
        td.Plan.from_system(synth.System(12, M, sys.A, sys.B, C), subdomains=2)
    assert e.value.code == 3


@pytest.mark.parametrize("M", [64, 192, 256, 512])
def test_singular_block_large(td, M):
    """A zero C block that opens a subdomain: TD_ESINGULAR with its block row, at block sizes of both
    Gauss-Jordan kernels."""
    sys = synth.varcoef_system(12, M, seed=20 + M)
    C = sys.C.copy()
    C[7] = 0.0                     # p = 2: interface rows 0 and 6, row 7 opens subdomain 1
    with pytest.raises(td.TridiagError) as e:
        td.Plan.from_system(synth.System(12, M, sys.A, sys.B, C), subdomains=2)
    assert e.value.code == 3 and "block row 7" in str(e.value)


@pytest.mark.parametrize("M,p", [(256, 32), (384, 32), (448, 32), (512, 32), (384, 35), (512, 37)])
def test_row_interchanges_many_blocks_per_launch(td, M, p):
    """Row interchanges with 32 or more subdomains of three rows: each step of the subdomain
    elimination inverts that many blocks in one launch, which takes the Gauss-Jordan path with
    64-column panels at block sizes from 384 (two 32-column halves per panel in the lead
    work-group) and the one with 32-column panels at 256.  35 and 37 subdomains leave the
    work-group grid's last group of eight matrices partly empty."""
    N, K = 3 * p, 5
    sys = _pivoting_system(N, M, 900 + M + p)
    F = synth.rhs_columns(900 + M + p, N, M, range(K))
    _, X = _solve(td, sys, F, p)
    assert rel_err(X, oracle.solve(sys, F)) < 1e-11


@pytest.mark.parametrize("M,p", [(128, 3), (256, 32), (512, 32)])
def test_exact_pivot_ties(td, M, p):
    """Diagonal blocks C_j = H / sqrt(M), H a Sylvester Hadamard matrix (orthogonal once scaled),
    with the dense couplings of dense_system (norm about 1.15 / sqrt(M)): in the first block of every
    subdomain all candidates of each pivot column tie exactly in magnitude, so the pivot search's
    tie-break (the smaller row) decides every pivot; the per-panel Gauss-Jordan paths with 32-column
    panels (128, 256) and 64-column panels (512, 32 blocks per launch)."""
    from scipy.linalg import hadamard
    N, K = 3 * p, 4
    base = synth.dense_system(N, M, 1300 + M)
    H = hadamard(M).astype(np.float64) / np.sqrt(M)    # symmetric: the storage order does not matter
    C = np.ascontiguousarray(np.broadcast_to(H, (N, M, M)))
    sys = synth.System(N, M, base.A, base.B, C, "dense", "dense", "dense")
    F = synth.rhs_columns(1300 + M, N, M, range(K))
    _, X = _solve(td, sys, F, p)
    assert rel_err(X, oracle.solve(sys, F)) < 1e-11


@pytest.mark.parametrize("M", [256, 384, 512])
def test_singular_and_nan_many_blocks_per_launch(td, M):
    """TD_ESINGULAR with 32 blocks per launch (the 64-column-panel path from block size 384): a zero
    C block that opens subdomain 5 (block row 16) and, separately, a NaN on the diagonal of block row
    50 in the last panel."""
    N, p = 96, 32
    sys = synth.varcoef_system(N, M, seed=60 + M)
    C = sys.C.copy()
    C[16] = 0.0
    with pytest.raises(td.TridiagError) as e:
        td.Plan.from_system(synth.System(N, M, sys.A, sys.B, C), subdomains=p)
    assert e.value.code == 3 and "block row 16" in str(e.value)
    C = sys.C.copy()
    C[50, 1, M - 3] = np.nan
    with pytest.raises(td.TridiagError) as e:
        td.Plan.from_system(synth.System(N, M, sys.A, sys.B, C), subdomains=p)
    assert e.value.code == 3

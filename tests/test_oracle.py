"""Pins of the CPU oracle against mathematics that does not go through the oracle.

Each pin reduces a case to a library routine or a closed form: numpy's dense LU
solve of the matrix of eq. (main-eq) written out in full, the separable DST-I
eigen-solution of the constant-coefficient 5-point operator, scipy's banded
solver for M = 1, SuperLU on the assembled sparse matrix up to the bench workload's
size, manufactured solutions, linearity, the adjoint identity, central finite
differences and the Schur-complement identity behind eq. (red1).  The last test
plants mistakes in the oracle (a flipped sign, a dropped term, a transposed
block, a wrong index, a missing row interchange) and checks that every planted
mistake fails at least one pin.
"""
import os
import tempfile

import numpy as np
import pytest
import scipy.fft
import scipy.linalg

import oracle
import synth
from dense_ref import dense_matrix, dense_solve, rel_err


def _rhs(seed, sys, K):
    return synth.rhs_columns(seed, sys.N, sys.M, range(K))


def nonsym_tridiag_system(N, M, seed):
    """TRIDIAG C with sub != super, DIAG A != DIAG B: a nonsymmetric, dominant system."""
    u = synth.uniform_range(seed, 9, 0, 6 * N * M).reshape(6, N, M)
    C = np.empty((N, 3, M))
    C[:, 0, :] = -(0.2 + 0.8 * u[0])
    C[:, 2, :] = -(0.2 + 0.8 * u[1])
    C[:, 1, :] = 4.5 + u[2]
    C[:, 0, 0] = 0.0
    C[:, 2, M - 1] = 0.0
    A = 0.3 + 0.7 * u[3]
    B = 0.3 + 0.7 * u[4]
    return synth.System(N, M, A, B, C, "diag", "diag", "tridiag")


def pivoting_system(N, M, seed):
    """Dense blocks whose diagonal blocks have a zero (0,0) entry: elimination needs row interchanges."""
    s = synth.dense_system(N, M, seed)
    C = s.C.copy()
    for j in range(N):
        # C_j = (dominant matrix) with rows 0 and 1 interchanged -> C_j(0,0) small/zero
        Cj = C[j].T.copy()
        Cj[[0, 1]] = Cj[[1, 0]]
        Cj[0, 0] = 0.0
        C[j] = Cj.T
    return synth.System(N, M, s.A, s.B, np.ascontiguousarray(C), "dense", "dense", "dense")


# ---------------------------------------------------------------- dense LU pins

def test_dense_lu_tiny_laplace():
    sys = synth.workload_system("tiny_n64_m16_k8")
    F = _rhs(1, sys, 8)
    assert rel_err(oracle.solve(sys, F), dense_solve(sys, F)) < 1e-13


def test_dense_lu_varcoef_nonsymmetric():
    sys = synth.varcoef_system(40, 12, seed=7)
    P = dense_matrix(sys)
    assert np.abs(P - P.T).max() > 0.01          # the case is really nonsymmetric
    F = _rhs(7, sys, 5)
    assert rel_err(oracle.solve(sys, F), dense_solve(sys, F)) < 1e-13


def test_dense_lu_dense_blocks():
    sys = synth.dense_system(9, 7, seed=11)
    F = _rhs(11, sys, 4)
    assert rel_err(oracle.solve(sys, F), dense_solve(sys, F)) < 1e-13


def test_dense_lu_nonsym_tridiag():
    sys = nonsym_tridiag_system(30, 10, seed=3)
    F = _rhs(3, sys, 3)
    assert rel_err(oracle.solve(sys, F), dense_solve(sys, F)) < 1e-13


def test_pivoting_required():
    sys = pivoting_system(6, 5, seed=5)
    F = _rhs(5, sys, 3)
    assert rel_err(oracle.solve(sys, F), dense_solve(sys, F)) < 1e-12


# ---------------------------------------------------------------- closed forms

def dst_solve(N, M, d, F):
    """C_j = tridiag(-1,d,-1), A_j = B_j = I: the operator separates in the two grid directions and
    the orthonormal DST-I diagonalises both 1-D second differences (eigenvalues
    d - 2cos(pi a/(M+1)) - 2cos(pi b/(N+1)))."""
    a = np.arange(1, M + 1)
    b = np.arange(1, N + 1)
    lam = d - 2 * np.cos(np.pi * a / (M + 1))[None, :] - 2 * np.cos(np.pi * b / (N + 1))[:, None]
    X = np.empty_like(F)
    for k in range(F.shape[0]):
        Phi = F[k].reshape(N, M)
        X[k] = scipy.fft.dstn(scipy.fft.dstn(Phi, type=1, norm="ortho") / lam, type=1, norm="ortho").ravel()
    return X


@pytest.mark.parametrize("N,M,d", [(64, 16, 4.5), (200, 48, 4.5), (37, 5, 4.1)])
def test_dst_closed_form(N, M, d):
    sys = synth.laplace_system(N, M, d)
    F = _rhs(2, sys, 4)
    assert rel_err(oracle.solve(sys, F), dst_solve(N, M, d, F)) < 1e-13


def test_scalar_blocks_banded():
    """M = 1: the block system is a scalar tridiagonal system."""
    N = 500
    u = synth.uniform_range(4, 9, 0, 3 * N).reshape(3, N)
    a, b, c = 0.2 + u[0], 0.2 + u[1], 2.5 + u[2]
    sys = synth.System(N, 1, a.reshape(N, 1), b.reshape(N, 1), c.reshape(N, 1, 1).copy(), "diag", "diag", "dense")
    F = _rhs(4, sys, 3)
    ab = np.zeros((3, N))
    ab[0, 1:] = -b[:-1]          # super-diagonal: P(j, j+1) = -b_j
    ab[1] = c
    ab[2, :-1] = -a[1:]          # sub-diagonal: P(j+1, j) = -a_{j+1}
    ref = scipy.linalg.solve_banded((1, 1), ab, F.T).T
    assert rel_err(oracle.solve(sys, F), ref) < 1e-14


def test_block_diagonal():
    """A = B = 0: the blocks decouple, X_j = C_j^{-1} F_j."""
    s = synth.dense_system(5, 6, seed=21)
    sys = synth.System(5, 6, np.zeros_like(s.A), np.zeros_like(s.B), s.C, "dense", "dense", "dense")
    F = _rhs(21, sys, 3)
    ref = np.concatenate([np.linalg.solve(s.C[j].T, F[:, j * 6:(j + 1) * 6].T).T for j in range(5)], axis=1)
    assert rel_err(oracle.solve(sys, F), ref) < 1e-14


def test_single_block_row():
    s = synth.dense_system(1, 9, seed=22)
    F = _rhs(22, s, 2)
    assert rel_err(oracle.solve(s, F), np.linalg.solve(s.C[0].T, F.T).T) < 1e-14


def test_manufactured_solution():
    sys = synth.dense_system(20, 5, seed=23)
    Xs = synth.uniform_range(23, 7, 0, 3 * 100, -1, 1).reshape(3, 100)
    F = Xs @ dense_matrix(sys).T
    assert rel_err(oracle.solve(sys, F), Xs) < 1e-13


def test_apply_matches_definition():
    sys = nonsym_tridiag_system(12, 6, seed=8)
    X = _rhs(8, sys, 3)
    assert rel_err(oracle.apply(sys, X), X @ dense_matrix(sys).T) < 1e-15


# ---------------------------------------------------------------- errors

def test_singular_block_reported():
    s = synth.dense_system(4, 3, seed=24)
    C = s.C.copy()
    C[0] = 0.0
    sys = synth.System(4, 3, s.A, s.B, C, "dense", "dense", "dense")
    with pytest.raises(oracle.OracleError) as e:
        oracle.solve(sys, _rhs(1, sys, 1))
    assert e.value.code == oracle.ESINGULAR and "block 0" in str(e.value)


def test_singular_later_block_reported():
    """D_1 = C_1 regular but D_2 = C_2 - A_2 C_1^{-1} B_1 = 0."""
    M = 3
    C = np.stack([np.eye(M) * 2.0, np.eye(M) * 0.5, np.eye(M) * 3.0])
    A = np.ones((3, M))
    B = np.ones((3, M))
    sys = synth.System(3, M, A, B, np.ascontiguousarray(C), "diag", "diag", "dense")
    with pytest.raises(oracle.OracleError) as e:
        oracle.solve(sys, _rhs(1, sys, 1))
    assert "block 1" in str(e.value)


# ---------------------------------------------------------------- adjoint

def test_adjoint_identity_nonsymmetric():
    sys = nonsym_tridiag_system(25, 8, seed=31)
    F, G = _rhs(31, sys, 3), _rhs(32, sys, 3)
    X = oracle.solve(sys, F)
    Lam = oracle.solve_adjoint(sys, G)
    lhs, rhs = np.sum(X * G), np.sum(F * Lam)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    assert rel_err(Lam, np.linalg.solve(dense_matrix(sys).T, G.T).T) < 1e-13


def test_adjoint_dense_blocks():
    sys = synth.dense_system(8, 5, seed=33)
    G = _rhs(33, sys, 2)
    assert rel_err(oracle.solve_adjoint(sys, G), np.linalg.solve(dense_matrix(sys).T, G.T).T) < 1e-13


def test_adjoint_symmetric_equals_forward():
    sys = synth.laplace_system(30, 7, 4.5)
    G = _rhs(34, sys, 2)
    assert rel_err(oracle.solve_adjoint(sys, G), oracle.solve(sys, G)) < 1e-14


def test_diag_shift_gradient_finite_differences():
    """L = 0.5 ||X - Xt||^2 with P(sigma) = P0 + diag(sigma): dL/dsigma = -sum_k Lambda X, Lambda = P^{-T}(X - Xt)."""
    N, M, K = 12, 6, 3
    sigma = synth.shift_sigma(N, M, seed=41)
    sys = synth.shift_system(sigma)
    F = _rhs(41, sys, K)
    Xt = synth.rhs_columns(41, N, M, range(K), stream=synth.STREAM_XT)
    X = oracle.solve(sys, F)
    Lam = oracle.solve_adjoint(sys, X - Xt)
    g = oracle.diag_shift_grad(Lam, X, N, M)
    h = 1e-6
    for e in [(0, 0), (3, 2), (11, 5), (7, 0)]:
        sp, sm = sigma.copy(), sigma.copy()
        sp[e] += h
        sm[e] -= h
        Xp = oracle.solve(synth.shift_system(sp), F)
        Xm = oracle.solve(synth.shift_system(sm), F)
        dL = 0.5 * np.sum((Xp - Xm) * (Xp + Xm - 2 * Xt))
        fd = dL / (2 * h)
        assert abs(fd - g[e]) < 1e-6 * max(1.0, abs(g[e])), (e, fd, g[e])


# ---------------------------------------------------------------- Algorithm 2 parts

@pytest.mark.parametrize("N,p", [(37, 6), (24, 4), (10, 10), (9, 1)])
def test_superposition_parts_definitions(N, p):
    """U, V, W solve eqs. (sub1)-(sub3); the reduced matrix of eq. (red1) is the Schur complement of P
    onto the interface rows; the interface solution and eq. (superposition) give X."""
    sys = nonsym_tridiag_system(N, 4, seed=50 + N)
    M = 4
    F = _rhs(50 + N, sys, 2)
    parts = oracle.superposition_parts(sys, p, F)
    ks = parts["ks"]
    P = dense_matrix(sys)
    X = oracle.solve(sys, F)
    # Schur complement onto the interface block rows
    gam = np.concatenate([np.arange(k * M, (k + 1) * M) for k in ks[:-1]])
    inn = np.setdiff1d(np.arange(N * M), gam)
    S = P[np.ix_(gam, gam)]
    if inn.size:
        S = S - P[np.ix_(gam, inn)] @ np.linalg.solve(P[np.ix_(inn, inn)], P[np.ix_(inn, gam)])
    Pt = np.zeros((p * M, p * M))
    for s in range(p):
        r = slice(s * M, (s + 1) * M)
        Pt[r, r] = parts["Ct"][s]
        if s > 0:
            Pt[r, (s - 1) * M:s * M] = -parts["At"][s]
        if s < p - 1:
            Pt[r, (s + 1) * M:(s + 2) * M] = -parts["Bt"][s]
    assert np.abs(Pt - S).max() < 1e-13 * np.abs(S).max()
    Xg = np.linalg.solve(Pt, parts["Ft"].reshape(2, p * M).T).T.reshape(2, p, M)
    Xb = X.reshape(2, N, M)
    assert rel_err(Xg, Xb[:, ks[:-1], :]) < 1e-13
    # eq. (superposition) on every row
    Xi = np.concatenate([Xg, np.zeros((2, 1, M))], axis=1)
    rec = np.empty_like(Xb)
    for s in range(p):
        for i in range(ks[s], ks[s + 1]):
            rec[:, i, :] = Xi[:, s] @ parts["U"][i].T + Xi[:, s + 1] @ parts["V"][i].T + parts["W"][:, i]
    assert rel_err(rec, Xb) < 1e-13


# ---------------------------------------------------------------- sparse direct solve at scale


def _five_point_csr(sys):
    """The matrix of eq. (main-eq) for DIAG A, B and TRIDIAG C, assembled entry by entry as a sparse
    matrix (row j*M + r): -A_j on column (j-1)*M + r, C_j(r, r-1 / r / r+1), -B_j on (j+1)*M + r."""
    import scipy.sparse

    N, M = sys.N, sys.M
    rows, cols, vals = [], [], []
    for j in range(N):
        for r in range(M):
            g = j * M + r
            rows.append(g); cols.append(g); vals.append(sys.C[j, 1, r])
            if r > 0:
                rows.append(g); cols.append(g - 1); vals.append(sys.C[j, 0, r])
            if r < M - 1:
                rows.append(g); cols.append(g + 1); vals.append(sys.C[j, 2, r])
            if j > 0:
                rows.append(g); cols.append(g - M); vals.append(-sys.A[j, r])
            if j < N - 1:
                rows.append(g); cols.append(g + M); vals.append(-sys.B[j, r])
    return scipy.sparse.csc_matrix((vals, (rows, cols)), shape=(N * M, N * M))


@pytest.mark.parametrize("N,M,family", [(256, 256, "varcoef"), (1024, 64, "nonsym")])
def test_sparse_lu_at_scale(N, M, family):
    """65k unknowns: the oracle against scipy's sparse LU (SuperLU) of the assembled matrix."""
    import scipy.sparse.linalg

    sys = synth.varcoef_system(N, M, seed=91) if family == "varcoef" else nonsym_tridiag_system(N, M, seed=92)
    F = _rhs(93, sys, 4)
    ref = scipy.sparse.linalg.splu(_five_point_csr(sys)).solve(np.ascontiguousarray(F.T)).T
    assert rel_err(oracle.solve(sys, F), ref) <= 1e-12


def test_sparse_lu_bench_workload():
    """The bench workload itself (N=2048, M=256: 524k unknowns, variable coefficients, nonsymmetric):
    the oracle against SuperLU on 4 of its right-hand sides (about 20 s)."""
    import scipy.sparse.linalg

    sys = synth.workload_system("varcoef_n2048_m256_k512")
    F = synth.rhs_columns(synth.WORKLOADS["varcoef_n2048_m256_k512"]["seed"], sys.N, sys.M, range(4))
    ref = scipy.sparse.linalg.splu(_five_point_csr(sys)).solve(np.ascontiguousarray(F.T)).T
    assert rel_err(oracle.solve(sys, F), ref) <= 1e-12


def test_linearity_and_column_independence():
    """solve(F1 + F2) = solve(F1) + solve(F2), and K columns at once equal one column at a time."""
    sys = nonsym_tridiag_system(40, 24, seed=95)
    F1, F2 = _rhs(96, sys, 5), _rhs(97, sys, 5)
    X1, X2 = oracle.solve(sys, F1), oracle.solve(sys, F2)
    assert rel_err(oracle.solve(sys, F1 + F2), X1 + X2) <= 1e-14
    cols = np.concatenate([oracle.solve(sys, F1[k:k + 1]) for k in range(5)])
    assert np.array_equal(cols, X1)


def test_partition_uneven():
    assert oracle.partition(37, 6) == [0, 7, 13, 19, 25, 31, 37]
    assert oracle.partition(40, 6) == [0, 7, 14, 21, 28, 34, 40]
    assert oracle.partition(64, 4) == [0, 16, 32, 48, 64]
    assert oracle.partition(5, 5) == [0, 1, 2, 3, 4, 5]


def test_thread_count_invariance():
    sys = synth.varcoef_system(50, 20, seed=60)
    F = _rhs(60, sys, 9)
    assert np.array_equal(oracle.solve(sys, F, threads=1), oracle.solve(sys, F, threads=8))


# ---------------------------------------------------------------- planted mistakes

def _pins_pass(lib_path):
    """A compact set of the pins above, run against an oracle build at lib_path."""
    cases = [pivoting_system(6, 5, seed=5), synth.dense_system(9, 7, seed=11), nonsym_tridiag_system(20, 6, seed=3)]
    for sys in cases:
        F = _rhs(5, sys, 2)
        try:
            X = oracle.solve(sys, F, lib_path=lib_path)
        except oracle.OracleError:
            return False
        if not np.all(np.isfinite(X)) or rel_err(X, dense_solve(sys, F)) > 1e-12:
            return False
    return True


@pytest.mark.parametrize("N,M,icol,family", [
    (13, 6, [4, 8], "laplace"), (20, 5, [3, 9, 14], "varcoef"), (9, 1, [2, 6], "laplace"), (12, 4, [5], "nonsym"),
])
def test_schur_complement_pins(N, M, icol, family):
    """Sec. 3: the interface values of the block-Thomas solution solve S x_G = f_G - A_GI A_II^{-1} f_I
    (eq. schur_decomp), S^{-1} is the interface block of P^{-1} (block inversion), and eq.
    (domains_equation) rebuilds the interior rows; for symmetric P, S is symmetric positive definite."""
    sys = {"laplace": lambda: synth.laplace_system(N, M, 4.5),
           "varcoef": lambda: synth.varcoef_system(N, M, seed=61),
           "nonsym": lambda: nonsym_tridiag_system(N, M, 62)}[family]()
    F = _rhs(63, sys, 4)
    X = oracle.solve(sys, F)
    S = oracle.schur_complement(sys, icol)
    g, _ = oracle.schur_sets(sys, icol)
    assert S.shape == (len(icol) * M, len(icol) * M)
    assert rel_err(X[:, g] @ S.T, oracle.schur_rhs(sys, icol, F)) <= 1e-12
    Pinv = np.linalg.inv(dense_matrix(sys))
    assert rel_err(np.linalg.inv(S), Pinv[np.ix_(g, g)]) <= 1e-11
    assert rel_err(oracle.schur_interior(sys, icol, F, X[:, g]), X) <= 1e-12
    if family == "laplace":
        assert np.allclose(S, S.T, rtol=0, atol=1e-13)
        assert np.linalg.eigvalsh(S).min() > 0


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5, 6])
def test_planted_mistakes_are_caught(mutant):
    with tempfile.TemporaryDirectory() as d:
        so = os.path.join(d, f"liboracle_m{mutant}.so")
        oracle.build(out=so, extra=[f"-DORACLE_MUTANT={mutant}"])
        assert not _pins_pass(so)


def test_unmutated_build_passes_compact_pins():
    assert _pins_pass(oracle._SO)

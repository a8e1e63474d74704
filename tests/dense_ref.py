"""Test-side helpers that are independent of both the oracle and the HIP library.

`dense_matrix` writes the block-tridiagonal matrix of eq. (main-eq) (Sec. 1) out as
one dense (N*M) x (N*M) array, straight from its definition, so that library
routines (numpy's LU solve, scipy's banded and FFT routines) can pin the oracle.
"""
import numpy as np


def block(fmt, src, j, M):
    """Block j as a row-major numpy matrix."""
    if fmt == "diag":
        return np.diag(src[j])
    if fmt == "dense":
        return np.asarray(src[j]).T      # stored column-major
    t = src[j]
    return np.diag(t[1]) + np.diag(t[0][1:], -1) + np.diag(t[2][:-1], 1)


def dense_matrix(sys):
    N, M = sys.N, sys.M
    P = np.zeros((N * M, N * M))
    for j in range(N):
        r = slice(j * M, (j + 1) * M)
        P[r, r] = block(sys.fmt_C, sys.C, j, M)
        if j > 0:
            P[r, (j - 1) * M:j * M] = -block(sys.fmt_A, sys.A, j, M)
        if j < N - 1:
            P[r, (j + 1) * M:(j + 2) * M] = -block(sys.fmt_B, sys.B, j, M)
    return P


def dense_solve(sys, F):
    """F: [K][N*M] -> X: [K][N*M] through numpy's LU solve of the dense matrix."""
    P = dense_matrix(sys)
    return np.linalg.solve(P, F.T).T


def rel_err(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def max_col_rel_residual(sys, X, F):
    P = dense_matrix(sys)
    R = F - X @ P.T
    return float(np.max(np.linalg.norm(R, axis=1) / np.linalg.norm(F, axis=1)))

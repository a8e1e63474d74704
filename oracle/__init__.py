"""ORACLE -- test infrastructure, not part of the library.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps the plain float64 block-Thomas solver of
`block_thomas.c` (the definition X = P^{-1} F of eq. (main-eq), Sec. 1 of
Terekhov's paper) and adds the few other plain definitions the tests need:
the product P X, the transposed system P^T, the diagonal-shift gradient and
the sub-problem solutions U, V, W of eqs. (sub1)-(sub3) with the reduced
matrix of eq. (red1) (Sec. 2.2), and the Schur complement on interface block
rows with its right-hand side and back-substitution (Sec. 3, eqs.
(schur_decomp), (domains_equation)).  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "block_thomas.c")

FMT = {"dense": 0, "diag": 1, "tridiag": 2}
OK, EINVAL, ENOMEM, ESINGULAR = 0, 1, 2, 3


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


def build(cc: str = "gcc", out: str = _SO, extra=()) -> str:
    """Compile block_thomas.c into a shared library (plain C, float64, OpenMP)."""
    cmd = [cc, "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", *extra, _SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def load(path: str = _SO):
    global _lib
    if path == _SO and _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"oracle library {path} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    i64, i32, dp, vp = ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
    lib.oracle_factor.argtypes = [i64, i64, i32, i32, i32, dp, dp, dp, i32, ctypes.POINTER(vp), ctypes.POINTER(i64)]
    lib.oracle_factor.restype = i32
    lib.oracle_solve.argtypes = [vp, dp, i64, dp, i64, i64, i32]
    lib.oracle_solve.restype = i32
    lib.oracle_free.argtypes = [vp]
    lib.oracle_free.restype = None
    lib.oracle_solve_system.argtypes = [i64, i64, i32, i32, i32, dp, dp, dp, dp, i64, dp, i64, i64, i32,
                                        ctypes.POINTER(i64)]
    lib.oracle_solve_system.restype = i32
    lib.oracle_apply.argtypes = [i64, i64, i32, i32, i32, dp, dp, dp, dp, i64, dp, i64, i64, i32]
    lib.oracle_apply.restype = i32
    if path == _SO:
        _lib = lib
    return lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(st, what, bad=None):
    if st == OK:
        return
    if st == ESINGULAR:
        raise OracleError(st, f"{what}: singular pivot in block {bad}")
    raise OracleError(st, f"{what}: status {st}")


class Factor:
    """The oracle's factored system (LU of every D_j and alpha_j), reusable for many F."""

    def __init__(self, sys, threads=None, lib_path: str = _SO):
        self.lib = load(lib_path)
        self.N, self.M = sys.N, sys.M
        self.threads = threads or default_threads()
        self._keep = (_c(sys.A), _c(sys.B), _c(sys.C))
        h = ctypes.c_void_p()
        bad = ctypes.c_int64(-1)
        st = self.lib.oracle_factor(sys.N, sys.M, FMT[sys.fmt_A], FMT[sys.fmt_B], FMT[sys.fmt_C],
                                    _ptr(self._keep[0]), _ptr(self._keep[1]), _ptr(self._keep[2]),
                                    self.threads, ctypes.byref(h), ctypes.byref(bad))
        _check(st, "oracle_factor", bad.value)
        self.h = h

    def solve(self, F: np.ndarray) -> np.ndarray:
        """F: [K][N*M] (column-major (N*M) x K). Returns X of the same layout."""
        F = _c(F)
        K = F.shape[0]
        n = self.N * self.M
        assert F.shape == (K, n)
        X = np.empty_like(F)
        st = self.lib.oracle_solve(self.h, _ptr(F), n, _ptr(X), n, K, self.threads)
        _check(st, "oracle_solve")
        return X

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.oracle_free(h)
            self.h = None


def solve(sys, F: np.ndarray, threads=None, lib_path: str = _SO) -> np.ndarray:
    """X = P^{-1} F for the system `sys` (see synth.System); F is [K][N*M]."""
    return Factor(sys, threads, lib_path).solve(F)


def apply(sys, X: np.ndarray, threads=None, lib_path: str = _SO) -> np.ndarray:
    """Y = P X (eq. (main-eq)); X is [K][N*M]."""
    lib = load(lib_path)
    X = _c(X)
    K = X.shape[0]
    n = sys.N * sys.M
    Y = np.empty_like(X)
    A, B, C = _c(sys.A), _c(sys.B), _c(sys.C)
    st = lib.oracle_apply(sys.N, sys.M, FMT[sys.fmt_A], FMT[sys.fmt_B], FMT[sys.fmt_C], _ptr(A), _ptr(B), _ptr(C),
                          _ptr(X), n, _ptr(Y), n, K, threads or default_threads())
    _check(st, "oracle_apply")
    return Y


def transpose_system(sys):
    """Blocks of P^T, again block tridiagonal with the sign convention of eq. (main-eq).

    Block (j, j+1) of P is -B_j and block (j+1, j) is -A_{j+1}; transposing the whole
    matrix gives C'_j = C_j^T, A'_j = B_{j-1}^T and B'_j = A_{j+1}^T.
    """
    import synth

    N, M = sys.N, sys.M

    def shift_down(x):   # x'_j = x_{j-1}, x'_0 = 0
        y = np.zeros_like(x)
        y[1:] = x[:-1]
        return y

    def shift_up(x):     # x'_j = x_{j+1}, x'_{N-1} = 0
        y = np.zeros_like(x)
        y[:-1] = x[1:]
        return y

    def tr(x, fmt):
        if fmt == "diag":
            return x
        if fmt == "dense":    # [N][c][r] column-major blocks: transpose swaps the last two axes
            return np.ascontiguousarray(np.swapaxes(x, 1, 2))
        raise ValueError(fmt)

    A2 = shift_down(tr(sys.B, sys.fmt_B))
    B2 = shift_up(tr(sys.A, sys.fmt_A))
    if sys.fmt_C == "dense":
        C2 = tr(sys.C, "dense")
    else:  # tridiag: (C^T)(i,i-1) = C(i-1,i) = super[i-1];  (C^T)(i,i+1) = C(i+1,i) = sub[i+1]
        C2 = np.zeros_like(sys.C)
        C2[:, 1, :] = sys.C[:, 1, :]
        C2[:, 0, 1:] = sys.C[:, 2, :-1]
        C2[:, 2, :-1] = sys.C[:, 0, 1:]
    return synth.System(N, M, A2, B2, C2, sys.fmt_B, sys.fmt_A, sys.fmt_C)


def solve_adjoint(sys, G: np.ndarray, threads=None, lib_path: str = _SO) -> np.ndarray:
    """Lambda = P^{-T} G."""
    return solve(transpose_system(sys), G, threads, lib_path)


def diag_shift_grad(Lam: np.ndarray, X: np.ndarray, N: int, M: int) -> np.ndarray:
    """dL/dsigma for a shift sigma added to the diagonal of every C_j, given Lambda = P^{-T} dL/dX.

    P depends on sigma_{j,i} only through its diagonal entry (j,i), so
    dL/dsigma_{j,i} = -sum_k Lambda_{(j,i),k} X_{(j,i),k}.
    """
    return -(Lam * X).sum(axis=0).reshape(N, M)


def timed_factor_solve(sys, F, threads=None):
    """(factor seconds, solve seconds, X) -- the CPU baseline's measurement."""
    t0 = time.perf_counter()
    fac = Factor(sys, threads)
    t1 = time.perf_counter()
    X = fac.solve(F)
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1, X


# ---------------------------------------------------------------------------
# Sub-problems of Algorithm 2 (Sec. 2.2), each from its own definition.  Small
# sizes only: they build each subsystem and solve it with the oracle above.
# ---------------------------------------------------------------------------

def partition(N: int, p: int):
    """Interface rows k_s (0-based) of p subdomains: the first N mod p get ceil(N/p) rows."""
    base, extra = divmod(N, p)
    ks, k = [], 0
    for s in range(p):
        ks.append(k)
        k += base + (1 if s < extra else 0)
    return ks + [N]


def _block(sys, which, j):
    """Dense M x M block (row-major numpy array) of A, B or C at block row j."""
    M = sys.M
    fmt = {"A": sys.fmt_A, "B": sys.fmt_B, "C": sys.fmt_C}[which]
    src = {"A": sys.A, "B": sys.B, "C": sys.C}[which]
    if fmt == "diag":
        return np.diag(src[j])
    if fmt == "dense":
        return src[j].T.copy()         # stored column-major
    t = src[j]
    return np.diag(t[1]) + np.diag(t[0][1:], -1) + np.diag(t[2][:-1], 1)


def _subsystem(sys, lo, hi):
    """Block rows lo..hi-1 of P as a dense-block system (the restriction {P}_lo^hi of Sec. 2.1)."""
    import synth

    n = hi - lo
    M = sys.M
    A = np.zeros((n, M, M)); B = np.zeros((n, M, M)); C = np.zeros((n, M, M))
    for t in range(n):
        A[t] = _block(sys, "A", lo + t).T
        B[t] = _block(sys, "B", lo + t).T
        C[t] = _block(sys, "C", lo + t).T
    return synth.System(n, M, A, B, C, "dense", "dense", "dense")


def superposition_parts(sys, p: int, F: np.ndarray):
    """U_i, V_i (eqs. sub1, sub2), W_i (eq. sub3) for every block row, and the reduced system of eq. (red1).

    Returns dict with U, V: [N][M][M] (row-major matrices, zero on interface rows except U = I),
    W: [K][N][M], and the reduced blocks At, Ct, Bt: [p][M][M], Ft: [K][p][M].
    """
    N, M = sys.N, sys.M
    K = F.shape[0]
    ks = partition(N, p)
    U = np.zeros((N, M, M)); V = np.zeros((N, M, M)); W = np.zeros((K, N, M))
    Fb = F.reshape(K, N, M)
    for s in range(p):
        a, b = ks[s], ks[s + 1]
        U[a] = np.eye(M)
        if b - a < 2:
            continue
        sub = _subsystem(sys, a + 1, b)
        n = b - a - 1
        # sub1: homogeneous equations with U_{k_s} = I moved to the right-hand side of the first interior row
        R = np.zeros((M, n * M))
        R[:, 0:M] = _block(sys, "A", a + 1).T          # column c = A_{a+1} e_c
        Uc = solve(sub, R)                              # [M][n*M]
        for t in range(n):
            U[a + 1 + t] = Uc[:, t * M:(t + 1) * M].T
        # sub2: V_{k_{s+1}} = I on the right boundary (absent, i.e. zero, past the last row N)
        if b < N:
            R = np.zeros((M, n * M))
            R[:, (n - 1) * M:] = _block(sys, "B", b - 1).T
            Vc = solve(sub, R)
            for t in range(n):
                V[a + 1 + t] = Vc[:, t * M:(t + 1) * M].T
        # sub3: the right-hand side with zero boundary values
        Wc = solve(sub, Fb[:, a + 1:b, :].reshape(K, n * M))
        W[:, a + 1:b, :] = Wc.reshape(K, n, M)
    At = np.zeros((p, M, M)); Ct = np.zeros((p, M, M)); Bt = np.zeros((p, M, M))
    Ft = np.zeros((K, p, M))
    for s in range(p):
        k = ks[s]
        Ak, Bk, Ck = _block(sys, "A", k), _block(sys, "B", k), _block(sys, "C", k)
        Ct[s] = Ck.copy()
        Ft[:, s, :] = Fb[:, k, :]
        if k > 0:                     # neighbour k-1 lies in subdomain s-1
            At[s] = Ak @ U[k - 1]
            Ct[s] -= Ak @ V[k - 1] if (k - 1) != ks[s - 1] else 0.0
            Ft[:, s, :] += W[:, k - 1, :] @ Ak.T
        if k + 1 < N:                 # neighbour k+1: interior row of s, or the next interface row
            if k + 1 < ks[s + 1]:
                Ct[s] -= Bk @ U[k + 1]
                Bt[s] = Bk @ V[k + 1]
                Ft[:, s, :] += W[:, k + 1, :] @ Bk.T
            else:
                Bt[s] = Bk
    return dict(ks=ks, U=U, V=V, W=W, At=At, Ct=Ct, Bt=Bt, Ft=Ft)


# ---------------------------------------------------------------------------
# Schur complement on interface block rows (Sec. 3, eqs. (linear_decomp),
# (schur_decomp), (domains_equation)): the unknowns of the block rows listed in
# `icol` form the interface set Gamma, all others the interior set I.  Small
# sizes only: P is assembled densely and A_II^{-1} is numpy's dense solve.
# ---------------------------------------------------------------------------

def dense_P(sys) -> np.ndarray:
    """P of eq. (main-eq) as a dense row-major (N M) x (N M) array."""
    N, M = sys.N, sys.M
    P = np.zeros((N * M, N * M))
    for j in range(N):
        r = slice(j * M, (j + 1) * M)
        P[r, r] = _block(sys, "C", j)
        if j > 0:
            P[r, (j - 1) * M:j * M] = -_block(sys, "A", j)
        if j + 1 < N:
            P[r, (j + 1) * M:(j + 2) * M] = -_block(sys, "B", j)
    return P


def schur_sets(sys, icol):
    """Unknown indices of the interface set (block rows icol, in that order) and of the interior set."""
    M = sys.M
    g = np.concatenate([np.arange(c * M, (c + 1) * M) for c in icol]) if len(icol) else np.zeros(0, int)
    mask = np.ones(sys.N * M, bool)
    mask[g] = False
    return g, np.nonzero(mask)[0]


def schur_complement(sys, icol) -> np.ndarray:
    """S = A_GG - A_GI A_II^{-1} A_IG (eq. schur_decomp), dense (|G| x |G|)."""
    P = dense_P(sys)
    g, i = schur_sets(sys, icol)
    return P[np.ix_(g, g)] - P[np.ix_(g, i)] @ np.linalg.solve(P[np.ix_(i, i)], P[np.ix_(i, g)])


def schur_rhs(sys, icol, F: np.ndarray) -> np.ndarray:
    """Right-hand side f_G - A_GI A_II^{-1} f_I of eq. (schur_decomp) for every row of F ([K][N M])."""
    P = dense_P(sys)
    g, i = schur_sets(sys, icol)
    Y = np.linalg.solve(P[np.ix_(i, i)], F[:, i].T)
    return F[:, g] - (P[np.ix_(g, i)] @ Y).T


def schur_interior(sys, icol, F: np.ndarray, xG: np.ndarray) -> np.ndarray:
    """Full solution from the interface values: x_I = A_II^{-1}(f_I - A_IG x_G) (eq. domains_equation)."""
    P = dense_P(sys)
    g, i = schur_sets(sys, icol)
    X = np.zeros_like(F)
    X[:, g] = xG
    X[:, i] = np.linalg.solve(P[np.ix_(i, i)], (F[:, i] - xG @ P[np.ix_(i, g)].T).T).T
    return X

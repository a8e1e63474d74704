"""Python binding of the MI355X block-tridiagonal solver (libtridiag.so).

Argument marshalling only: every step of the factor and of the solve runs in the
HIP kernels behind the C ABI of include/tridiag.h.  Tensors are torch float64
tensors on the current HIP device; the current torch stream is passed to the
library.  The solver is Algorithm 2 of Terekhov's paper (Sec. 2.2) with the
dichotomy of Algorithm 1 (Sec. 2.1) on the reduced interface system.

Layouts: DIAG fields [N][M], TRIDIAG fields [N][3][M] (sub, diag, super), DENSE
fields [N][M][M] with each block column-major; right-hand sides are tensors of
shape (K, N*M) (row k = right-hand side k), i.e. column-major (N*M) x K.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtridiag.so")

FMT = {"dense": 0, "diag": 1, "tridiag": 2}
PREC = {"f64": 0, "f32": 1, "bf16": 2}
STATUS = {0: "TD_OK", 1: "TD_EINVAL", 2: "TD_ENOMEM", 3: "TD_ESINGULAR", 4: "TD_ENOCONV", 5: "TD_ENOADJ",
          6: "TD_EHIP", 7: "TD_ENOTSUP"}


class TridiagError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def _torch_alloc(ctx, nbytes, stream):
    """td_desc.dev_alloc: a block of torch's caching allocator on the current device, associated with
    the library call's stream; None (the library then reports TD_ENOMEM) when it cannot allocate."""
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=torch.cuda.current_device(),
                                                  stream=int(stream or 0))
    except Exception:
        return None


def _torch_free(ctx, ptr, stream):
    try:
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


# kept alive for the lifetime of the module: the library calls them until every plan is destroyed
TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
TORCH_FREE = _FREE_FN(_torch_free)


class _Desc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("M", ctypes.c_int64), ("subdomains", ctypes.c_int64),
                ("fmt_A", ctypes.c_int32), ("fmt_B", ctypes.c_int32), ("fmt_C", ctypes.c_int32),
                ("sweep_prec", ctypes.c_int32), ("adjoint", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("k_hint", ctypes.c_int64), ("dev_alloc", _ALLOC_FN), ("dev_free", _FREE_FN),
                ("alloc_ctx", ctypes.c_void_p)]


class _Refine(ctypes.Structure):
    _fields_ = [("enable", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("nonfinite", ctypes.c_int32),
                ("max_col_rel_residual", ctypes.c_double)]


class _Tiles(ctypes.Structure):
    _fields_ = [("sweep_cols", ctypes.c_int32), ("sweep_waves", ctypes.c_int32), ("sup_cols", ctypes.c_int32),
                ("sup_waves", ctypes.c_int32)]


TILE_FIELDS = ("sweep_cols", "sweep_waves", "sup_cols", "sup_waves")


class _PlanInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("M", ctypes.c_int64), ("subdomains", ctypes.c_int64),
                ("Mp", ctypes.c_int64), ("tree_depth", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("factor_ms", ctypes.c_double), ("sweep_prec", ctypes.c_int32), ("adjoint", ctypes.c_int32)]


# every symbol the header declares
EXPORTS = ["tridiag_factor", "tridiag_solve", "tridiag_solve_adjoint", "tridiag_diag_grad", "tridiag_destroy",
           "tridiag_plan_info", "tridiag_set_profiling", "tridiag_stage_times", "tridiag_status_string",
           "tridiag_last_error", "tridiag_batch_create", "tridiag_batch_solve", "tridiag_batch_info",
           "tridiag_batch_destroy", "tridiag_autotune", "tridiag_autotune_tiles", "tridiag_set_tiles",
           "tridiag_get_tiles", "tridiag_band_to_blocks", "tridiag_schur_create",
           "tridiag_schur_apply", "tridiag_schur_solve", "tridiag_schur_destroy", "tridiag_default_subdomains",
           "tridiag_plan_bytes", "tridiag_solve_batched", "tridiag_solve_noalloc"]

class _SchurInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("active", ctypes.c_int32), ("max_rel_residual", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtridiag.so; raise if it is not built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.tridiag_factor.argtypes = [ctypes.POINTER(_Desc), vp, vp, vp, vp, ctypes.POINTER(vp)]
    lib.tridiag_factor.restype = i32
    lib.tridiag_solve.argtypes = [vp, vp, i64, vp, i64, i64, ctypes.POINTER(_Refine), ctypes.POINTER(_Info), vp]
    lib.tridiag_solve.restype = i32
    lib.tridiag_solve_adjoint.argtypes = lib.tridiag_solve.argtypes
    lib.tridiag_solve_adjoint.restype = i32
    lib.tridiag_diag_grad.argtypes = [vp, i64, vp, i64, i64, i64, vp, vp]
    lib.tridiag_diag_grad.restype = i32
    lib.tridiag_destroy.argtypes = [vp]
    lib.tridiag_destroy.restype = i32
    lib.tridiag_plan_info.argtypes = [vp, ctypes.POINTER(_PlanInfo)]
    lib.tridiag_plan_info.restype = i32
    lib.tridiag_set_profiling.argtypes = [vp, ctypes.c_int]
    lib.tridiag_set_profiling.restype = i32
    lib.tridiag_stage_times.argtypes = [vp, ctypes.POINTER(dp), ctypes.c_int]
    lib.tridiag_stage_times.restype = i32
    lib.tridiag_status_string.argtypes = [i32]
    lib.tridiag_status_string.restype = ctypes.c_char_p
    lib.tridiag_last_error.argtypes = []
    lib.tridiag_last_error.restype = ctypes.c_char_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    lib.tridiag_batch_create.argtypes = [ctypes.c_int, pp, pp, pi64, pp, pi64, pi64, ctypes.c_int, dp, vp,
                                         ctypes.POINTER(vp)]
    lib.tridiag_batch_create.restype = i32
    lib.tridiag_batch_solve.argtypes = [vp, vp]
    lib.tridiag_batch_solve.restype = i32
    lib.tridiag_batch_info.argtypes = [vp, ctypes.POINTER(_Info)]
    lib.tridiag_batch_info.restype = i32
    lib.tridiag_batch_destroy.argtypes = [vp]
    lib.tridiag_batch_destroy.restype = i32
    lib.tridiag_autotune.argtypes = [i64, i64, i32, i64, pi64, ctypes.c_int, vp, pi64, ctypes.POINTER(dp)]
    lib.tridiag_autotune.restype = i32
    lib.tridiag_autotune_tiles.argtypes = [i64, i64, i32, i64, pi64, ctypes.c_int, vp, pi64, ctypes.POINTER(_Tiles),
                                           ctypes.POINTER(dp)]
    lib.tridiag_autotune_tiles.restype = i32
    lib.tridiag_set_tiles.argtypes = [vp, ctypes.POINTER(_Tiles)]
    lib.tridiag_set_tiles.restype = i32
    lib.tridiag_get_tiles.argtypes = [vp, ctypes.POINTER(_Tiles)]
    lib.tridiag_get_tiles.restype = i32
    lib.tridiag_band_to_blocks.argtypes = [i64, i32, i32, vp, i64, i64, vp, vp, vp, vp]
    lib.tridiag_band_to_blocks.restype = i32
    lib.tridiag_schur_create.argtypes = [i64, i64, vp, vp, vp, i64, pi64, i32, vp, ctypes.POINTER(vp)]
    lib.tridiag_schur_create.restype = i32
    lib.tridiag_schur_apply.argtypes = [vp, vp, i64, vp, i64, i64, vp]
    lib.tridiag_schur_apply.restype = i32
    lib.tridiag_schur_solve.argtypes = [vp, vp, i64, vp, i64, i64, dp, i32, ctypes.POINTER(_SchurInfo), vp]
    lib.tridiag_schur_solve.restype = i32
    lib.tridiag_schur_destroy.argtypes = [vp]
    lib.tridiag_schur_destroy.restype = i32
    lib.tridiag_default_subdomains.argtypes = [i64, i64, pi64]
    lib.tridiag_default_subdomains.restype = i32
    lib.tridiag_plan_bytes.argtypes = [ctypes.POINTER(_Desc), pi64]
    lib.tridiag_plan_bytes.restype = i32
    lib.tridiag_solve_batched.argtypes = [ctypes.c_int, pp, pp, pp, pi64, ctypes.POINTER(_Refine),
                                          ctypes.POINTER(_Info), vp]
    lib.tridiag_solve_batched.restype = i32
    lib.tridiag_solve_noalloc.argtypes = [vp, vp, i64, vp, i64, i64, vp]
    lib.tridiag_solve_noalloc.restype = i32
    _lib = lib
    return lib


def _check(code: int):
    if code != 0:
        msg = _lib.tridiag_last_error().decode()
        raise TridiagError(code, msg)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 tensor on a HIP device")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    return t


def _rhs(t: torch.Tensor, n: int, name: str):
    """(K, n) tensor with row stride >= n -> (pointer, ld, K)."""
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 tensor on a HIP device")
    if t.dim() != 2 or t.shape[1] != n or t.stride(1) != 1 or (t.shape[0] > 1 and t.stride(0) < n):
        raise TypeError(f"{name} must have shape (K, {n}) with unit column stride")
    ld = t.stride(0) if t.shape[0] > 1 else n
    return ctypes.c_void_p(t.data_ptr()), max(ld, n), t.shape[0]


class Plan:
    """A factored block-tridiagonal matrix (tridiag_factor) reusable for many right-hand sides."""

    def __init__(self, A, B, C, N, M, fmt_A="diag", fmt_B="diag", fmt_C="tridiag", subdomains=0,
                 sweep_prec="f64", adjoint=False, k_hint=512, torch_allocator=True, tiles="auto"):
        """subdomains = 0: choose_subdomains(N, M, k_hint, sweep_prec) (the autotuned length for the
        expected number of right-hand sides per solve, else the library's default rule).
        torch_allocator: the plan's device memory comes from torch's caching allocator (td_desc
        callbacks); False: the library's own hipMalloc.
        tiles: launch shapes of the sweeps and the superposition (tridiag_set_tiles): "auto" = the
        autotuner's cached shapes for (M, k_hint bucket, precision) when the plan also uses the cached
        subdomain length, else the library's rules; a dict of TILE_FIELDS; None = the rules."""
        self.lib = load_library()
        self.N, self.M = int(N), int(M)
        tuned = autotuned_entry(self.M, int(k_hint), sweep_prec)
        if not subdomains:
            subdomains = choose_subdomains(self.N, self.M, int(k_hint), sweep_prec)
            if tiles == "auto" and tuned and "tiles" in tuned and tuned.get("L"):
                tiles = tuned["tiles"]
        d = _Desc(self.N, self.M, int(subdomains), FMT[fmt_A], FMT[fmt_B], FMT[fmt_C], PREC[sweep_prec],
                  1 if adjoint else 0, 0, int(k_hint), TORCH_ALLOC if torch_allocator else _ALLOC_FN(),
                  TORCH_FREE if torch_allocator else _FREE_FN(), None)
        A, B, C = _dev(A, "A"), _dev(B, "B"), _dev(C, "C")
        if torch_allocator:
            # torch may hold freed blocks in its cache that the library's free-memory check cannot see
            need = ctypes.c_int64()
            _check(self.lib.tridiag_plan_bytes(ctypes.byref(d), ctypes.byref(need)))
            free, _ = torch.cuda.mem_get_info(A.device)
            if need.value > 0.9 * free:
                torch.cuda.empty_cache()
        h = ctypes.c_void_p()
        with torch.cuda.device(A.device):
            code = self.lib.tridiag_factor(ctypes.byref(d), ctypes.c_void_p(A.data_ptr()),
                                           ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(C.data_ptr()),
                                           _stream(), ctypes.byref(h))
        _check(code)
        self.h = h
        self.device = A.device
        if isinstance(tiles, dict):
            self.set_tiles(**tiles)

    def set_tiles(self, **tiles):
        """Launch shapes (TILE_FIELDS, 0 = the library's rule) of this plan and its transposed plan."""
        t = _Tiles(*(int(tiles.get(k, 0)) for k in TILE_FIELDS))
        _check(self.lib.tridiag_set_tiles(self.h, ctypes.byref(t)))

    def get_tiles(self) -> dict:
        t = _Tiles()
        _check(self.lib.tridiag_get_tiles(self.h, ctypes.byref(t)))
        return {k: int(getattr(t, k)) for k in TILE_FIELDS}

    @classmethod
    def from_system(cls, sys, device="cuda", **kw):
        """Factor a synth.System (numpy arrays in the C-ABI layouts)."""
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
        return cls(t(sys.A), t(sys.B), t(sys.C), sys.N, sys.M, sys.fmt_A, sys.fmt_B, sys.fmt_C, **kw)

    def _solve(self, fn, F, X, refine, info):
        n = self.N * self.M
        fp, ldf, K = _rhs(F, n, "F")
        if X is None:
            X = torch.empty((K, n), dtype=torch.float64, device=F.device)
        xp, ldx, K2 = _rhs(X, n, "X")
        if K2 != K:
            raise ValueError("F and X have different numbers of columns")
        rf = None
        if refine:
            if refine is True:
                refine = {}
            rf = _Refine(1, int(refine.get("max_iter", 10)), float(refine.get("tol", 1e-10)))
        inf = _Info() if info else None
        code = fn(self.h, fp, ldf, xp, ldx, K, ctypes.byref(rf) if rf else None,
                  ctypes.byref(inf) if inf else None, _stream())
        if code == 4 and info:  # no convergence: report instead of raising when the caller asked for info
            return X, {"iterations": inf.iterations, "nonfinite": inf.nonfinite,
                       "max_col_rel_residual": inf.max_col_rel_residual, "converged": False}
        _check(code)
        if info:
            return X, {"iterations": inf.iterations, "nonfinite": inf.nonfinite,
                       "max_col_rel_residual": inf.max_col_rel_residual, "converged": True}
        return X

    def solve(self, F, X=None, refine=None, info=False):
        """X = P^{-1} F.  F: (K, N*M) float64 on the device.  refine: None, True or dict(tol, max_iter)."""
        return self._solve(self.lib.tridiag_solve, F, X, refine, info)

    def solve_noalloc(self, F, X):
        """tridiag_solve_noalloc: X = P^{-1} F with the workspace in the library's fixed device array
        (no allocation; TD_EINVAL above its 64 MiB).  X must be given (K, N*M), like F."""
        n = self.N * self.M
        fp, ldf, K = _rhs(F, n, "F")
        xp, ldx, K2 = _rhs(X, n, "X")
        if K2 != K:
            raise ValueError("F and X have different numbers of columns")
        _check(self.lib.tridiag_solve_noalloc(self.h, fp, ldf, xp, ldx, K, _stream()))
        return X

    def solve_adjoint(self, G, Lam=None, refine=None, info=False):
        """Lam = P^{-T} G (needs adjoint=True at factor time)."""
        return self._solve(self.lib.tridiag_solve_adjoint, G, Lam, refine, info)

    def plan_info(self) -> dict:
        pi = _PlanInfo()
        _check(self.lib.tridiag_plan_info(self.h, ctypes.byref(pi)))
        return {f: getattr(pi, f) for f, _ in _PlanInfo._fields_}

    def set_profiling(self, on: bool = True):
        _check(self.lib.tridiag_set_profiling(self.h, 1 if on else 0))

    def stage_times(self) -> dict:
        """Average ms per solve of each stage over the solves profiled since the last call."""
        buf = (ctypes.c_double * 8)()
        _check(self.lib.tridiag_stage_times(self.h, buf, 8))
        names = ["sweep", "interface_rhs", "dichotomy_partial", "dichotomy_levels", "superposition",
                 "refinement", "total", "count"]
        return dict(zip(names, list(buf)))

    def close(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.tridiag_destroy(h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def diag_grad(Lam: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """out[r] = -sum_k Lam[k, r] X[k, r] (gradient w.r.t. a shift of the diagonal of the C_j)."""
    lib = load_library()
    n = Lam.shape[1]
    lp, ldl, K = _rhs(Lam, n, "Lam")
    xp, ldx, K2 = _rhs(X, n, "X")
    if K2 != K:
        raise ValueError("Lam and X have different numbers of columns")
    out = torch.empty(n, dtype=torch.float64, device=Lam.device)
    _check(lib.tridiag_diag_grad(lp, ldl, xp, ldx, n, K, ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


class ShiftedSolve(torch.autograd.Function):
    """X = P(sigma)^{-1} F for C_j = tridiag(sub_j, base_j + sigma_j, super_j) with fixed A_j, B_j.

    Backward: Lam = P^{-T} dL/dX (the factored transpose), dL/dF = Lam and
    dL/dsigma = -sum_k Lam o X (the diagonal entries of dL/dP = -Lam X^T).
    The plan comes from `solver` (a ShiftedSolver), which refactors only when sigma changes.
    """

    @staticmethod
    def forward(ctx, F, sigma, solver):
        plan = solver.plan_for(sigma)
        X = plan.solve(F.contiguous(), refine=solver.refine)
        ctx.plan = plan                 # kept alive until backward, even if the solver refactors
        ctx.refine = solver.refine
        ctx.save_for_backward(X)
        ctx.NM = tuple(sigma.shape)
        return X

    @staticmethod
    def backward(ctx, gX):
        (X,) = ctx.saved_tensors
        Lam = ctx.plan.solve_adjoint(gX.contiguous(), refine=ctx.refine)
        dsig = diag_grad(Lam, X).view(*ctx.NM)
        return Lam, dsig, None


class ShiftedSolver:
    """Differentiable X = P(sigma)^{-1} F for the shifted system C_j = tridiag(sub_j, base_j + sigma_j,
    super_j), A_j, B_j fixed (diagonal; base_C tridiagonal [N][3][M]).  The plan, with its transposed
    factor for the backward pass, is kept between calls and rebuilt only when sigma changes (compared
    by value on the device), so repeated gradient steps at one sigma pay one factor."""

    def __init__(self, base_C, A, B, subdomains=0, sweep_prec="f64", refine=None, k_hint=512):
        self.base_C, self.A, self.B = _dev(base_C, "base_C"), _dev(A, "A"), _dev(B, "B")
        self.subdomains, self.sweep_prec, self.refine, self.k_hint = subdomains, sweep_prec, refine, k_hint
        self._sigma = None
        self._plan = None
        self.factors = 0                # number of factorizations done

    def plan_for(self, sigma):
        sigma = sigma.detach()
        if self._plan is None or self._sigma.shape != sigma.shape or not torch.equal(self._sigma, sigma):
            N, M = sigma.shape
            C = self.base_C.clone()
            C[:, 1, :] += sigma
            self._plan = Plan(self.A, self.B, C.contiguous(), N, M, "diag", "diag", "tridiag",
                              subdomains=self.subdomains, sweep_prec=self.sweep_prec, adjoint=True,
                              k_hint=self.k_hint)
            self._sigma = sigma.clone()
            self.factors += 1
        return self._plan

    def __call__(self, F, sigma):
        return ShiftedSolve.apply(F, sigma, self)


def shifted_solve(F, sigma, base_C, A, B, subdomains=0, sweep_prec="f64", refine=None):
    """One-shot form of ShiftedSolver (factors P(sigma) on every call)."""
    return ShiftedSolver(base_C, A, B, subdomains, sweep_prec, refine)(F, sigma)


class Batch:
    """Many independent systems solved by one persistent launch replayed from a HIP graph.

    plans: Plan objects factored with sweep_prec="f32"; Fs, Xs: per-system (K_q, N_q*M_q) float64
    device tensors (the graph reads and writes exactly these buffers on every solve()).
    passes: solve passes (1 + correction passes); tol: residual bar for the per-system early exit.
    """

    def __init__(self, plans, Fs, Xs, passes=3, tol=1e-10):
        self.lib = load_library()
        n = len(plans)
        if not (n == len(Fs) == len(Xs)) or n == 0:
            raise ValueError("plans, Fs and Xs must have the same non-zero length")
        self._keep = (list(plans), list(Fs), list(Xs))
        P = (ctypes.c_void_p * n)(*[p.h.value for p in plans])
        fptr, ldf, K, xptr, ldx = [], [], [], [], []
        for p, F, X in zip(plans, Fs, Xs):
            n_ = p.N * p.M
            a, lf, k = _rhs(F, n_, "F")
            b, lx, k2 = _rhs(X, n_, "X")
            if k != k2:
                raise ValueError("F and X column counts differ")
            fptr.append(a.value); ldf.append(lf); K.append(k); xptr.append(b.value); ldx.append(lx)
        self.n = n
        h = ctypes.c_void_p()
        code = self.lib.tridiag_batch_create(
            n, P, (ctypes.c_void_p * n)(*fptr), (ctypes.c_int64 * n)(*ldf), (ctypes.c_void_p * n)(*xptr),
            (ctypes.c_int64 * n)(*ldx), (ctypes.c_int64 * n)(*K), int(passes), float(tol), _stream(),
            ctypes.byref(h))
        _check(code)
        self.h = h

    def solve(self):
        _check(self.lib.tridiag_batch_solve(self.h, _stream()))

    def info(self):
        """Per-system dicts; converged is False for a system that missed tol within the passes."""
        infos = (_Info * self.n)()
        code = self.lib.tridiag_batch_info(self.h, infos)
        if code not in (0, 4):
            _check(code)
        return [{"iterations": i.iterations, "max_col_rel_residual": i.max_col_rel_residual,
                 "nonfinite": i.nonfinite} for i in infos], code == 0

    def close(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.tridiag_batch_destroy(h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batched(plans, Fs, Xs, refine=None, info=False):
    """tridiag_solve_batched: X_q = P_q^{-1} F_q for every plan, through one captured batch that later
    calls with the same plans, tensors and refinement settings replay.  Fs, Xs: (K_q, N_q*M_q)
    contiguous float64 device tensors.  refine: None (one pass), True or dict(tol, max_iter).
    info=True: returns the per-system reports."""
    lib = load_library()
    n = len(plans)
    if not (n == len(Fs) == len(Xs)) or n == 0:
        raise ValueError("plans, Fs and Xs must have the same non-zero length")
    for p, F, X in zip(plans, Fs, Xs):
        nn = p.N * p.M
        for t, name in ((F, "F"), (X, "X")):
            _dev(t, name)
            if t.dim() != 2 or t.shape[1] != nn:
                raise TypeError(f"{name} must have shape (K, {nn})")
        if F.shape[0] != X.shape[0]:
            raise ValueError("F and X column counts differ")
    rf = None
    if refine:
        refine = {} if refine is True else refine
        rf = _Refine(1, int(refine.get("max_iter", 2)), float(refine.get("tol", 1e-10)))
    infos = (_Info * n)() if info else None
    code = lib.tridiag_solve_batched(n, (ctypes.c_void_p * n)(*[p.h.value for p in plans]),
                                     (ctypes.c_void_p * n)(*[F.data_ptr() for F in Fs]),
                                     (ctypes.c_void_p * n)(*[X.data_ptr() for X in Xs]),
                                     (ctypes.c_int64 * n)(*[F.shape[0] for F in Fs]),
                                     ctypes.byref(rf) if rf else None, infos, _stream())
    if code not in (0, 4) or (code == 4 and not info):
        _check(code)
    if info:
        return [{"iterations": i.iterations, "max_col_rel_residual": i.max_col_rel_residual,
                 "nonfinite": i.nonfinite} for i in infos], code == 0
    return None


def release_batched():
    """Drop the batch cached by solve_batched (tridiag_solve_batched with n = 0)."""
    _check(load_library().tridiag_solve_batched(0, None, None, None, None, None, None, None))


class BandSolver:
    """Solves with an n x n band matrix (kl sub-, ku super-diagonals) through its block-tridiagonal
    form (tridiag_band_to_blocks, then a float64 plan with DENSE blocks of size M).

    ab: float64 device tensor of shape (n, kl + ku + 1); row j holds column j of the general band
    storage, i.e. ab[j, ku + i - j] = a(i, j).  Right-hand sides are (K, n) tensors; they are
    padded with zeros to N*M rows for the solve and the solution is cut back to n rows."""

    def __init__(self, ab, kl: int, ku: int, M: int = 0, subdomains: int = 0, adjoint: bool = False):
        lib = load_library()
        ab = _dev(ab, "ab")
        self.n, self.kl, self.ku = int(ab.shape[0]), int(kl), int(ku)
        if ab.dim() != 2 or ab.shape[1] != self.kl + self.ku + 1:
            raise ValueError("ab must have shape (n, kl + ku + 1)")
        self.M = int(M) if M else max(self.kl, self.ku, 1)
        self.N = -(-self.n // self.M)
        blocks = [torch.empty((self.N, self.M, self.M), dtype=torch.float64, device=ab.device) for _ in range(3)]
        A, B, C = blocks
        _check(lib.tridiag_band_to_blocks(self.n, self.kl, self.ku, ctypes.c_void_p(ab.data_ptr()), ab.shape[1],
                                          self.M, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                          ctypes.c_void_p(C.data_ptr()), _stream()))
        self.plan = Plan(A, B, C, self.N, self.M, "dense", "dense", "dense", subdomains=subdomains, adjoint=adjoint)

    def _pad(self, F):
        Fp = torch.zeros((F.shape[0], self.N * self.M), dtype=torch.float64, device=F.device)
        Fp[:, : self.n] = F
        return Fp

    def solve(self, F, refine=None):
        return self.plan.solve(self._pad(F), refine=refine)[:, : self.n]

    def solve_adjoint(self, G, refine=None):
        return self.plan.solve_adjoint(self._pad(G), refine=refine)[:, : self.n]


class SchurSolver:
    """Schur-complement solver on interface block rows (tridiag_schur_*): the block rows `icol`
    of the system (diagonal A, B; tridiagonal C; symmetric) are the interfaces, solved by
    conjugate gradients on S = A_GG - A_GI A_II^{-1} A_IG with a probing preconditioner of
    half-bandwidth `band` (-1: none); the interiors by the stacked interior plan.

    A, B: (N, M) and C: (N, 3, M) float64 device tensors.  Vectors are (K, rows) tensors:
    full vectors have N*M rows, interface vectors len(icol)*M rows."""

    def __init__(self, A, B, C, icol, band: int = 4):
        lib = load_library()
        A, B, C = _dev(A, "A"), _dev(B, "B"), _dev(C, "C")
        self.N, self.M = int(A.shape[0]), int(A.shape[1])
        self.icol = [int(c) for c in icol]
        arr = (ctypes.c_int64 * len(self.icol))(*self.icol)
        h = ctypes.c_void_p()
        _check(lib.tridiag_schur_create(self.N, self.M, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                        ctypes.c_void_p(C.data_ptr()), len(self.icol), arr, int(band), _stream(),
                                        ctypes.byref(h)))
        self.lib, self.h = lib, h

    def apply(self, V):
        V = _dev(V, "V")
        Y = torch.empty_like(V)
        _check(self.lib.tridiag_schur_apply(self.h, ctypes.c_void_p(V.data_ptr()), V.shape[1],
                                            ctypes.c_void_p(Y.data_ptr()), Y.shape[1], V.shape[0], _stream()))
        return Y

    def solve(self, F, tol: float = 1e-10, max_iter: int = 500, info: bool = False):
        F = _dev(F, "F")
        X = torch.empty_like(F)
        inf = _SchurInfo()
        st = self.lib.tridiag_schur_solve(self.h, ctypes.c_void_p(F.data_ptr()), F.shape[1],
                                          ctypes.c_void_p(X.data_ptr()), X.shape[1], F.shape[0], float(tol),
                                          int(max_iter), ctypes.byref(inf), _stream())
        rep = {"iterations": inf.iterations, "active": inf.active, "max_rel_residual": inf.max_rel_residual,
               "converged": st == 0}
        if st != 4 or not info:
            _check(st)
        return (X, rep) if info else X

    def close(self):
        if getattr(self, "h", None):
            self.lib.tridiag_schur_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_subdomains(N: int, K: int) -> int:
    """The library's default subdomain count for N block rows and K right-hand sides
    (tridiag_default_subdomains): N / L with L the longest of 32, 16 and 8 rows that still gives the
    sweeps about 512 work-groups."""
    lib = load_library()
    p = ctypes.c_int64()
    _check(lib.tridiag_default_subdomains(int(N), int(K), ctypes.byref(p)))
    return int(p.value)


def choose_subdomains(N: int, M: int, K: int, sweep_prec: str = "f64") -> int:
    """Subdomain count for an N x M system with K right-hand sides: N / L with the subdomain length
    L from the autotuner's cached result for (M, K bucket, precision) when present, else the library's
    default rule (default_subdomains)."""
    L = autotuned_length(M, K, sweep_prec, default=0)
    if L <= 0:
        return default_subdomains(N, K)
    return max(1, min(N, N // L))


def _cache_path():
    return os.environ.get("TD_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "tridiag_autotune.json"))


def _kbucket(K):
    b = 16
    while b < K:
        b *= 2
    return b


def autotuned_entry(M, K, sweep_prec="f64"):
    """The cached autotuner result for (M, K bucket, precision), or None."""
    import json
    try:
        with open(_cache_path()) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        return None
    return cache.get(f"gfx950|M{M}|K{_kbucket(K)}|{sweep_prec}")


def autotuned_length(M, K, sweep_prec="f64", default=0):
    e = autotuned_entry(M, K, sweep_prec)
    return int(e.get("L", default)) if e else default


def autotune(M, K, sweep_prec="f64", probe_N=1024, candidates=(8, 16, 32, 64, 128), store=True, tiles=True):
    """Time the candidate subdomain lengths on a probe system (C++ search in the library) and
    record the fastest in the JSON cache keyed by (arch, M, K bucket, precision).  tiles: search the
    sweeps' and the superposition's launch shapes as well (tridiag_autotune_tiles) and record them."""
    import json
    lib = load_library()
    cand = [c for c in candidates if c <= probe_N]
    best = ctypes.c_int64()
    if tiles:
        t = _Tiles()
        bms = ctypes.c_double()
        _check(lib.tridiag_autotune_tiles(int(M), int(_kbucket(K)), PREC[sweep_prec], int(probe_N),
                                          (ctypes.c_int64 * len(cand))(*cand), len(cand), _stream(),
                                          ctypes.byref(best), ctypes.byref(t), ctypes.byref(bms)))
        result = {"L": int(best.value), "tiles": {k: int(getattr(t, k)) for k in TILE_FIELDS},
                  "ms_per_solve": float(bms.value), "probe_N": probe_N}
    else:
        ms = (ctypes.c_double * len(cand))()
        _check(lib.tridiag_autotune(int(M), int(_kbucket(K)), PREC[sweep_prec], int(probe_N),
                                    (ctypes.c_int64 * len(cand))(*cand), len(cand), _stream(), ctypes.byref(best), ms))
        result = {"L": int(best.value), "ms_per_solve": dict(zip(map(str, cand), list(ms))), "probe_N": probe_N}
    if store:
        path = _cache_path()
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        cache[f"gfx950|M{M}|K{_kbucket(K)}|{sweep_prec}"] = result
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return result

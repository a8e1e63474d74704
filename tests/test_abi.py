"""C-ABI checks that need no GPU: the library loads, exports every function that
include/tridiag.h declares, and rejects invalid arguments on the host before any HIP
call is made."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tridiag.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tridiag_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_1108_4181_amd as td

    if not os.path.exists(td.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return td.load_library()


def test_header_declares_the_solver_api():
    names = header_functions()
    for required in ("tridiag_factor", "tridiag_solve", "tridiag_solve_adjoint", "tridiag_destroy",
                     "tridiag_batch_create", "tridiag_batch_solve", "tridiag_status_string", "tridiag_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_export_list_matches_header():
    import paper_1108_4181_amd as td

    assert sorted(td.EXPORTS) == header_functions()


def test_status_strings(lib):
    import paper_1108_4181_amd as td

    lib.tridiag_status_string.restype = ctypes.c_char_p
    for code, name in td.STATUS.items():
        s = lib.tridiag_status_string(code).decode()
        assert s.startswith(name), (code, s)


def _desc(td, **kw):
    d = td._Desc()
    d.N, d.M, d.subdomains = kw.get("N", 64), kw.get("M", 16), kw.get("p", 4)
    d.fmt_A, d.fmt_B, d.fmt_C = kw.get("fA", 1), kw.get("fB", 1), kw.get("fC", 2)
    d.sweep_prec, d.adjoint, d.reserved = kw.get("prec", 0), 0, kw.get("reserved", 0)
    return d


@pytest.mark.parametrize("kw,code", [
    (dict(N=0), 1), (dict(M=0), 1), (dict(p=65), 1), (dict(p=-1), 1), (dict(fA=2), 1), (dict(fC=1), 1),
    (dict(prec=3), 1), (dict(reserved=1), 1), (dict(M=513), 7),
])
def test_factor_rejects_bad_descriptors_on_host(lib, kw, code):
    import paper_1108_4181_amd as td

    d = _desc(td, **kw)
    plan = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    st = lib.tridiag_factor(ctypes.byref(d), dummy, dummy, dummy, None, ctypes.byref(plan))
    assert st == code
    assert plan.value is None
    lib.tridiag_last_error.restype = ctypes.c_char_p
    assert lib.tridiag_last_error().decode()


def test_null_arguments_rejected(lib):
    import paper_1108_4181_amd as td

    d = _desc(td)
    plan = ctypes.c_void_p()
    assert lib.tridiag_factor(None, None, None, None, None, ctypes.byref(plan)) == 1
    assert lib.tridiag_factor(ctypes.byref(d), None, None, None, None, ctypes.byref(plan)) == 1
    assert lib.tridiag_factor(ctypes.byref(d), None, None, None, None, None) == 1
    assert lib.tridiag_solve(None, None, 0, None, 0, 1, None, None, None) == 1
    assert lib.tridiag_solve_adjoint(None, None, 0, None, 0, 1, None, None, None) == 1
    assert lib.tridiag_diag_grad(None, 0, None, 0, 0, 0, None, None) == 1
    assert lib.tridiag_destroy(None) == 0


@pytest.mark.parametrize("n,kl,ku,ldab,M,code", [
    (0, 1, 1, 3, 2, 1), (10, -1, 1, 3, 2, 1), (10, 2, 2, 4, 2, 1), (10, 3, 1, 5, 2, 1), (10, 1, 1, 3, 600, 7),
])
def test_band_conversion_rejects_bad_sizes(lib, n, kl, ku, ldab, M, code):
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    assert lib.tridiag_band_to_blocks(n, kl, ku, dummy, ldab, M, dummy, dummy, dummy, None) == code


@pytest.mark.parametrize("N,M,icol,band,code", [
    (10, 4, [0], 2, 1), (10, 4, [3, 4], 2, 1), (10, 4, [9], 2, 1), (10, 4, [4], 65, 1), (10, 4, [4], -2, 1),
    (10, 513, [4], 2, 7), (2, 4, [1], 2, 1), (10, 4, [2, 4, 6, 8, 8], 2, 1),
])
def test_schur_create_rejects_bad_arguments_on_host(lib, N, M, icol, band, code):
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    arr = (ctypes.c_int64 * len(icol))(*icol)
    out = ctypes.c_void_p()
    lib.tridiag_schur_create.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    assert lib.tridiag_schur_create(N, M, dummy, dummy, dummy, len(icol), arr, band, None, ctypes.byref(out)) == code
    assert out.value is None


def test_schur_null_handles(lib):
    assert lib.tridiag_schur_solve(None, None, 0, None, 0, 1, ctypes.c_double(0.0), 0, None, None) == 1
    assert lib.tridiag_schur_apply(None, None, 0, None, 0, 1, None) == 1
    assert lib.tridiag_schur_destroy(None) == 0


def test_default_subdomain_count_fills_the_gpu(tmp_path, monkeypatch, lib):
    """Without an autotuned entry the subdomain length is the longest of 32, 16, 8 rows that gives
    the sweeps about 512 work-groups (subdomains x 32-column tiles); the binding and the library's
    subdomains = 0 use the same rule (tridiag_default_subdomains)."""
    import paper_1108_4181_amd as td

    monkeypatch.setenv("TD_AUTOTUNE_CACHE", str(tmp_path / "none.json"))
    assert td.default_subdomains(2048, 512) == 64      # L = 32: 64 subdomains x 16 tiles
    assert td.default_subdomains(4096, 1024) == 128
    assert td.default_subdomains(1093, 256) == 68      # L = 16: 34 x 8 would be 272 work-groups
    assert td.default_subdomains(2032, 64) == 254      # L = 8
    assert td.default_subdomains(64, 8) == 8
    assert td.default_subdomains(4, 1) == 1
    assert td.default_subdomains(2048, 0) == 64        # K <= 0 means 512
    assert td.choose_subdomains(1093, 60, 256) == 68
    assert td.choose_subdomains(4, 16, 1) == 1
    p = ctypes.c_int64()
    assert lib.tridiag_default_subdomains(0, 8, ctypes.byref(p)) == 1
    assert lib.tridiag_default_subdomains(8, 8, None) == 1


def test_plan_bytes_on_host(lib):
    """The factor's footprint (checked against free device memory before anything is allocated) is
    computed on the host: it grows with N, doubles with the transposed plan, and p = 0 gives the
    footprint of the default subdomain count."""
    import paper_1108_4181_amd as td

    def nbytes(**kw):
        d = _desc(td, **kw)
        d.adjoint = kw.get("adj", 0)
        b = ctypes.c_int64()
        assert lib.tridiag_plan_bytes(ctypes.byref(d), ctypes.byref(b)) == 0
        return b.value

    base = nbytes(N=2048, M=256, p=64)
    assert base > 4 * 2048 * 256 * 256 * 8           # D^-1, alpha, U and V at least
    assert nbytes(N=4096, M=256, p=64) > 1.8 * base
    assert nbytes(N=2048, M=256, p=64, adj=1) == 2 * base
    assert nbytes(N=2048, M=256, p=0) == base         # p = 0: the default rule gives 64 here
    d = _desc(td, M=600)
    assert lib.tridiag_plan_bytes(ctypes.byref(d), ctypes.byref(ctypes.c_int64())) == 7
    assert lib.tridiag_plan_bytes(None, ctypes.byref(ctypes.c_int64())) == 1


def test_allocator_callbacks_must_come_in_pairs(lib):
    import paper_1108_4181_amd as td

    d = _desc(td)
    d.dev_alloc = td.TORCH_ALLOC
    plan = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    assert lib.tridiag_factor(ctypes.byref(d), dummy, dummy, dummy, None, ctypes.byref(plan)) == 1
    assert plan.value is None


def test_solve_batched_rejects_bad_arguments(lib):
    assert lib.tridiag_solve_batched(-1, None, None, None, None, None, None, None) == 1
    assert lib.tridiag_solve_batched(2, None, None, None, None, None, None, None) == 1
    assert lib.tridiag_solve_batched(0, None, None, None, None, None, None, None) == 0   # releases the cache

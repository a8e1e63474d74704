"""Boundary behaviour on the GPU: plan memory through torch's caching allocator (td_desc callbacks),
the footprint check that rejects a plan larger than free device memory before allocating anything
(TD_ENOMEM), the library's default subdomain count for subdomains = 0, and the one-call batched solve
(tridiag_solve_batched: captured on the first call, replayed on later ones)."""
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


def test_plan_memory_is_torch_allocated(td):
    sys = synth.varcoef_system(256, 64, seed=81)
    F = _dev(synth.rhs_columns(81, 256, 64, range(24)))
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    plan = td.Plan.from_system(sys, subdomains=8, adjoint=True)
    X = plan.solve(F)
    torch.cuda.synchronize()
    held = plan.plan_info()["device_bytes"]
    grown = torch.cuda.memory_allocated() - before
    # the plan's buffers (factor, its transposed plan, the solve workspace) plus X are torch blocks
    assert held > 0 and grown >= held + X.numel() * 8
    assert rel_err(X.cpu().numpy(), oracle.solve(sys, F.cpu().numpy())) <= 1e-12
    plan.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before == X.numel() * 8   # every plan buffer returned
    del X
    assert torch.cuda.memory_allocated() == before


def test_plan_memory_with_library_allocator(td):
    sys = synth.varcoef_system(64, 32, seed=82)
    F = _dev(synth.rhs_columns(82, 64, 32, range(5)))
    before = torch.cuda.memory_allocated()
    plan = td.Plan.from_system(sys, subdomains=4, torch_allocator=False)
    X = plan.solve(F)
    assert torch.cuda.memory_allocated() - before == X.numel() * 8
    assert rel_err(X.cpu().numpy(), oracle.solve(sys, F.cpu().numpy())) <= 1e-12
    plan.close()


def test_footprint_above_free_memory_is_rejected_before_allocating(td):
    """N = 40000 block rows of 512 x 512: the float64 factor alone would need about 500 GB.  The
    inputs are real, valid device arrays (diagonal A, B and tridiagonal C); the library compares its
    footprint with the free memory and returns TD_ENOMEM without allocating anything."""
    N, M = 40000, 512
    A = torch.ones((N, M), dtype=torch.float64, device="cuda")
    B = torch.ones((N, M), dtype=torch.float64, device="cuda")
    C = torch.zeros((N, 3, M), dtype=torch.float64, device="cuda")
    C[:, 1, :] = 4.5
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    for alloc in (True, False):
        with pytest.raises(td.TridiagError) as e:
            td.Plan(A, B, C, N, M, subdomains=1250, torch_allocator=alloc)
        assert e.value.code == 2 and "bytes" in str(e.value)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before


def test_default_subdomains_in_the_library(td):
    """subdomains = 0 in the descriptor: the library's rule for k_hint right-hand sides (the same
    function the binding's choose_subdomains falls back to)."""
    import ctypes

    sys = synth.laplace_system(1093, 16, 4.5)
    A, B, C = _dev(sys.A), _dev(sys.B), _dev(sys.C)
    lib = td.load_library()
    for k_hint, want in ((256, 68), (64, 136), (0, 34)):
        d = td._Desc(1093, 16, 0, 1, 1, 2, 0, 0, 0, k_hint, td._ALLOC_FN(), td._FREE_FN(), None)
        h = ctypes.c_void_p()
        assert lib.tridiag_factor(ctypes.byref(d), ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                  ctypes.c_void_p(C.data_ptr()), td._stream(), ctypes.byref(h)) == 0
        info = td._PlanInfo()
        assert lib.tridiag_plan_info(h, ctypes.byref(info)) == 0
        assert info.subdomains == want == td.default_subdomains(1093, k_hint)
        lib.tridiag_destroy(h)


@pytest.mark.parametrize("refine", [None, {"tol": 1e-10, "max_iter": 3}])
def test_solve_batched_captures_then_replays(td, refine):
    shapes = [(40, 64, 5, 4), (97, 64, 33, 6), (64, 128, 17, 4)]
    prec = "f32" if refine else "f64"
    plans, Fs, Xs, systems, Fh = [], [], [], [], []
    for q, (N, M, K, p) in enumerate(shapes):
        sysq = synth.varcoef_system(N, M, seed=600 + q)
        F = synth.rhs_columns(600 + q, N, M, range(K))
        plans.append(td.Plan.from_system(sysq, subdomains=p, sweep_prec=prec))
        Fs.append(_dev(F))
        Xs.append(torch.zeros_like(Fs[-1]))
        systems.append(sysq)
        Fh.append(F)
    infos, ok = td.solve_batched(plans, Fs, Xs, refine=refine, info=True)
    assert ok
    first = [x.clone() for x in Xs]
    tol = 1e-9 if refine else 1e-12
    for q in range(len(shapes)):
        assert rel_err(Xs[q].cpu().numpy(), oracle.solve(systems[q], Fh[q])) <= tol
        if refine:
            assert infos[q]["max_col_rel_residual"] <= 1e-10
    for _ in range(2):                 # replays of the captured batch
        for x in Xs:
            x.zero_()
        td.solve_batched(plans, Fs, Xs, refine=refine)
        torch.cuda.synchronize()
        for a, b in zip(first, Xs):
            assert torch.equal(a, b)
    td.release_batched()
    for p in plans:
        p.close()

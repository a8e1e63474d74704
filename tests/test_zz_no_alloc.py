"""tridiag_solve_noalloc (through the C ABI): the plain solve with its workspace in the library's fixed
device array instead of the plan's, for callers that cannot allocate.  Its result must equal the
plan's own solve (tridiag_solve) bitwise, on two calls in a row whose second input is smaller (the
array keeps the first call's contents), on float64 and float32 plans; sizes above the array are
rejected on the host; and the solve allocates nothing through torch either."""
import ctypes
import gc

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


def _noalloc(td, plan, F, X):
    n = plan.N * plan.M
    return td.load_library().tridiag_solve_noalloc(plan.h, ctypes.c_void_p(F.data_ptr()), n,
                                                   ctypes.c_void_p(X.data_ptr()), n, F.shape[0], td._stream())


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_matches_plan_solve_twice(td, prec):
    big = synth.varcoef_system(96, 64, seed=91)
    small = synth.varcoef_system(40, 48, seed=92)
    Fb = _dev(synth.rhs_columns(91, 96, 64, range(40)))
    Fs = _dev(synth.rhs_columns(92, 40, 48, range(7)))
    pb = td.Plan.from_system(big, subdomains=6, sweep_prec=prec)
    ps = td.Plan.from_system(small, subdomains=5, sweep_prec=prec)
    refb, refs = pb.solve(Fb).clone(), ps.solve(Fs).clone()
    torch.cuda.synchronize()
    Xb = torch.full_like(Fb, float("nan"))
    Xs = torch.full_like(Fs, float("nan"))
    # unreachable objects of earlier tests (a plan in a reference cycle frees its memory when the
    # collector runs) must not be collected inside the measured window
    gc.collect()
    gc.disable()
    try:
        before = torch.cuda.memory_allocated()
        assert _noalloc(td, pb, Fb, Xb) == 0           # first call: the larger system
        assert _noalloc(td, ps, Fs, Xs) == 0           # second call: smaller, other plan, same array
        torch.cuda.synchronize()
        after = torch.cuda.memory_allocated()
    finally:
        gc.enable()
    assert after == before
    assert torch.equal(Xb, refb)
    assert torch.equal(Xs, refs)
    # and a smaller call on the same plan after the larger one
    Xb2 = torch.full_like(Fb[:9], float("nan"))
    assert _noalloc(td, pb, Fb[:9].contiguous(), Xb2) == 0
    torch.cuda.synchronize()
    assert torch.equal(Xb2, pb.solve(Fb[:9].contiguous()))
    if prec == "f64":
        assert rel_err(Xs.cpu().numpy(), oracle.solve(small, Fs.cpu().numpy())) <= 1e-12
    pb.close()
    ps.close()


def test_noalloc_rejects_workspace_above_the_array(td):
    sys = synth.laplace_system(256, 256, 4.5)          # W alone: 256 * 256 * 256 * 8 = 128 MiB
    plan = td.Plan.from_system(sys, subdomains=8)
    F = torch.zeros((256, 256 * 256), dtype=torch.float64, device="cuda")
    X = torch.empty_like(F)
    assert _noalloc(td, plan, F, X) == 1
    assert b"scratch" in td.load_library().tridiag_last_error()
    plan.close()


def test_noalloc_scalar_plan(td):
    """The scalar plan (block size 1, every row an interface row): the no-allocation solve places the
    top levels' partial sums and top-row values in the fixed array; equal to the plan's own solve."""
    sys = synth.varcoef_system(3000, 1, seed=93)
    F = _dev(synth.rhs_columns(93, 3000, 1, range(9)))
    plan = td.Plan.from_system(sys, subdomains=3000)
    ref = plan.solve(F).clone()
    X = torch.full_like(F, float("nan"))
    assert _noalloc(td, plan, F, X) == 0
    torch.cuda.synchronize()
    assert torch.equal(X, ref)
    plan.close()

"""Adjoint (transposed) solves and the torch.autograd.Function built on them.

* Lambda = P^{-T} G against the oracle on a nonsymmetric system (float64, <= 1e-12);
* the adjoint identity <P^{-1} F, G> = <F, P^{-T} G>;
* gradients of L = 0.5 ||X - X_t||^2 w.r.t. F and the diagonal shift sigma from backward()
  against the oracle's adjoint formula and against central finite differences (h = 1e-6,
  32 random sigma entries, float64, relative error <= 1e-6), at the differentiation workload's
  size (N=1024, M=256, K=256, 32 subdomains);
* the float32 path with refinement agrees with the float64 gradient to <= 1e-8.
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


def test_adjoint_identity_device(td):
    sys = synth.varcoef_system(96, 48, seed=61)
    F = synth.rhs_columns(61, 96, 48, range(7))
    G = synth.rhs_columns(62, 96, 48, range(7))
    plan = td.Plan.from_system(sys, subdomains=6, adjoint=True)
    X = plan.solve(_dev(F)).cpu().numpy()
    Lam = plan.solve_adjoint(_dev(G)).cpu().numpy()
    lhs, rhs = float(np.sum(X * G)), float(np.sum(F * Lam))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert rel_err(Lam, oracle.solve_adjoint(sys, G)) <= 1e-12


def test_adjoint_without_transpose_factor(td):
    sys = synth.varcoef_system(16, 16, seed=63)
    plan = td.Plan.from_system(sys, subdomains=2)
    with pytest.raises(td.TridiagError) as e:
        plan.solve_adjoint(_dev(synth.rhs_columns(63, 16, 16, range(1))))
    assert e.value.code == 5


def test_diag_grad_kernel(td):
    Lam = synth.rhs_columns(64, 8, 16, range(5))
    X = synth.rhs_columns(65, 8, 16, range(5))
    got = td.diag_grad(_dev(Lam), _dev(X)).cpu().numpy()
    assert np.allclose(got, -(Lam * X).sum(axis=0), rtol=1e-14, atol=0)


def _shift_inputs(name):
    w = synth.WORKLOADS[name]
    N, M, K = w["N"], w["M"], w["K"]
    sigma = synth.shift_sigma(N, M, w["seed"])
    base = synth.shift_system(np.zeros((N, M)))
    F = synth.rhs_columns(w["seed"], N, M, range(K))
    Xt = synth.rhs_columns(w["seed"], N, M, range(K), stream=synth.STREAM_XT)
    return w, sigma, base, F, Xt


def _loss_grad(td, sigma, base, F, Xt, p, prec="f64", refine=None):
    sig = _dev(sigma).requires_grad_(True)
    Ft = _dev(F).requires_grad_(True)
    X = td.shifted_solve(Ft, sig, _dev(base.C), _dev(base.A), _dev(base.B), subdomains=p, sweep_prec=prec,
                         refine=refine)
    L = 0.5 * ((X - _dev(Xt)) ** 2).sum()
    L.backward()
    return X.detach().cpu().numpy(), sig.grad.cpu().numpy(), Ft.grad.cpu().numpy()


@pytest.fixture(scope="module")
def grad64(td):
    w, sigma, base, F, Xt = _shift_inputs("adjoint_n1024_m256_k256")
    X, gs, gF = _loss_grad(td, sigma, base, F, Xt, w["p"])
    return w, sigma, base, F, Xt, X, gs, gF


def test_gradient_matches_oracle_adjoint(td, grad64):
    w, sigma, base, F, Xt, X, gs, gF = grad64
    sys = synth.shift_system(sigma)
    Xo = oracle.solve(sys, F)
    assert rel_err(X, Xo) <= 1e-12
    Lam = oracle.solve_adjoint(sys, Xo - Xt)
    assert rel_err(gF, Lam) <= 1e-12
    assert rel_err(gs, oracle.diag_shift_grad(Lam, Xo, sys.N, sys.M)) <= 1e-12


def test_gradient_finite_differences(td, grad64):
    w, sigma, base, F, Xt, X, gs, gF = grad64
    N, M = sigma.shape
    rng = np.random.default_rng([4, 7])
    picks = rng.choice(N * M, 32, replace=False)
    h = 1e-6
    Fd, Xtd = _dev(F), _dev(Xt)
    A, B = _dev(base.A), _dev(base.B)
    worst = 0.0
    for e in picks:
        j, i = divmod(int(e), M)
        Xs = []
        for sgn in (1.0, -1.0):
            C = base.C.copy()
            C[:, 1, :] += sigma
            C[j, 1, i] += sgn * h
            plan = td.Plan(A, B, _dev(C), N, M, subdomains=w["p"])
            Xs.append(plan.solve(Fd))
            plan.close()
        # L+ - L- = 0.5 sum (X+ - X-) o (X+ + X- - 2 Xt): no cancellation of two large L values
        dL = 0.5 * float(((Xs[0] - Xs[1]) * (Xs[0] + Xs[1] - 2 * Xtd)).sum())
        fd = dL / (2 * h)
        worst = max(worst, abs(fd - gs[j, i]) / max(abs(gs[j, i]), 1e-30))
    assert worst <= 1e-6, worst


def test_float32_gradient_refined(td, grad64):
    w, sigma, base, F, Xt, X, gs, gF = grad64
    _, gs32, gF32 = _loss_grad(td, sigma, base, F, Xt, w["p"], prec="f32", refine={"tol": 1e-12, "max_iter": 10})
    assert rel_err(gs32, gs) <= 1e-8
    assert rel_err(gF32, gF) <= 1e-8


def test_float32_gradient_unrefined(td, grad64):
    """Float32 sweeps without refinement (forward and adjoint solves each carry float32 rounding of
    the factor): gradients within 1e-4 of the float64 adjoint (finite differences at h = 1e-6 are
    meaningless at float32 resolution, so the float64 gradient is the reference)."""
    w, sigma, base, F, Xt, X, gs, gF = grad64
    X32, gs32, gF32 = _loss_grad(td, sigma, base, F, Xt, w["p"], prec="f32", refine=None)
    assert rel_err(X32, X) <= 1e-5
    assert rel_err(gs32, gs) <= 1e-4
    assert rel_err(gF32, gF) <= 1e-4


def test_shifted_solver_reuses_its_plan(td):
    """ShiftedSolver factors once per distinct sigma: two gradient steps at one sigma reuse the plan
    (same gradients as a one-shot solve), a changed sigma refactors."""
    N, M, K = 64, 32, 6
    sigma = synth.shift_sigma(N, M, 41)
    base = synth.shift_system(np.zeros((N, M)))
    F = synth.rhs_columns(41, N, M, range(K))
    Xt = synth.rhs_columns(42, N, M, range(K))
    solver = td.ShiftedSolver(_dev(base.C), _dev(base.A), _dev(base.B), subdomains=4)
    grads = []
    for step in range(3):
        sig = _dev(sigma if step < 2 else sigma * 1.5).requires_grad_(True)
        Ft = _dev(F).requires_grad_(True)
        X = solver(Ft, sig)
        (0.5 * ((X - _dev(Xt)) ** 2).sum()).backward()
        grads.append(sig.grad.cpu().numpy())
        assert solver.factors == (1 if step < 2 else 2)
    assert np.array_equal(grads[0], grads[1])
    _, gs_ref, _ = _loss_grad(td, sigma, base, F, Xt, 4)
    assert rel_err(grads[0], gs_ref) <= 1e-12
    sys2 = synth.shift_system(sigma * 1.5)
    Xo = oracle.solve(sys2, F)
    Lam = oracle.solve_adjoint(sys2, Xo - Xt)
    assert rel_err(grads[2], oracle.diag_shift_grad(Lam, Xo, N, M)) <= 1e-12


def test_adjoint_more_interior_rows_than_one_launch(td):
    """The transposed plan takes the forward block inverses transposed, in launches of at most 65535
    blocks: N = 66000 block rows of 16 in 64 subdomains (65936 interior rows), against the oracle."""
    N, M, K = 66000, 16, 2
    sys = synth.varcoef_system(N, M, seed=66)
    G = synth.rhs_columns(66, N, M, range(K))
    plan = td.Plan.from_system(sys, subdomains=64, adjoint=True)
    Lam = plan.solve_adjoint(_dev(G)).cpu().numpy()
    assert rel_err(Lam, oracle.solve_adjoint(sys, G)) < 1e-12
    plan.close()

"""Batched solve of uneven systems (a HIP graph of one launch per stage, or one persistent launch
with counted dependencies) against the CPU oracle: float32 sweeps, float64 reduced systems and
refinement to a max column relative residual of 1e-10; error vs the float64 oracle <= 1e-9.
Replays of the graph give bitwise the same result as the first run.  Every test runs in both
launch forms."""
import os

import numpy as np
import pytest

import oracle
import synth
from dense_ref import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = [  # N, M, K, p
    (40, 64, 5, 4), (97, 64, 33, 6), (128, 128, 64, 8), (200, 64, 17, 10), (64, 256, 40, 4), (150, 128, 3, 15),
]


@pytest.fixture(autouse=True, params=["staged", "persistent"])
def batch_mode(request):
    old = os.environ.get("TD_BATCH_MODE")
    os.environ["TD_BATCH_MODE"] = request.param
    yield request.param
    if old is None:
        del os.environ["TD_BATCH_MODE"]
    else:
        os.environ["TD_BATCH_MODE"] = old


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1108_4181_amd as m

    m.load_library()
    return m


def _build(td):
    plans, Fs, Xs, systems, Fh = [], [], [], [], []
    for q, (N, M, K, p) in enumerate(SHAPES):
        sys = synth.laplace_system(N, M, 4.5) if q % 2 == 0 else synth.varcoef_system(N, M, seed=300 + q)
        F = synth.rhs_columns(300 + q, N, M, range(K))
        plans.append(td.Plan.from_system(sys, subdomains=p, sweep_prec="f32"))
        Fs.append(torch.as_tensor(F, device="cuda"))
        Xs.append(torch.zeros((K, N * M), dtype=torch.float64, device="cuda"))
        systems.append(sys)
        Fh.append(F)
    return plans, Fs, Xs, systems, Fh


def test_batched_matches_oracle_and_replays(td):
    plans, Fs, Xs, systems, Fh = _build(td)
    batch = td.Batch(plans, Fs, Xs, passes=4, tol=1e-10)
    batch.solve()
    infos, ok = batch.info()
    assert ok, infos
    first = [x.clone() for x in Xs]
    for q, (sys, F) in enumerate(zip(systems, Fh)):
        X = Xs[q].cpu().numpy()
        R = F - oracle.apply(sys, X)
        res = float(np.max(np.linalg.norm(R, axis=1) / np.linalg.norm(F, axis=1)))
        assert res <= 1e-10 and infos[q]["max_col_rel_residual"] <= 1e-10, (q, res, infos[q])
        assert rel_err(X, oracle.solve(sys, F)) <= 1e-9
    for _ in range(2):
        for x in Xs:
            x.zero_()
        batch.solve()
        _, ok = batch.info()
        assert ok
        for a, b in zip(first, Xs):
            assert torch.equal(a, b)
    batch.close()


def test_batched_float64_and_mixed_plans(td):
    """float64 plans in the persistent launch: one pass reaches float64 accuracy; float64 and
    float32 plans can share one batch."""
    plans, Fs, Xs, systems, Fh = [], [], [], [], []
    for q, (N, M, K, p) in enumerate(SHAPES):
        sys = synth.varcoef_system(N, M, seed=400 + q)
        F = synth.rhs_columns(400 + q, N, M, range(K))
        plans.append(td.Plan.from_system(sys, subdomains=p, sweep_prec="f64" if q % 2 == 0 else "f32"))
        Fs.append(torch.as_tensor(F, device="cuda"))
        Xs.append(torch.zeros((K, N * M), dtype=torch.float64, device="cuda"))
        systems.append(sys)
        Fh.append(F)
    batch = td.Batch(plans, Fs, Xs, passes=3, tol=1e-10)
    batch.solve()
    infos, ok = batch.info()
    assert ok, infos
    for q, (sys, F) in enumerate(zip(systems, Fh)):
        X = Xs[q].cpu().numpy()
        ref = oracle.solve(sys, F)
        if q % 2 == 0:
            assert infos[q]["iterations"] == 0 and rel_err(X, ref) <= 1e-12
        else:
            assert rel_err(X, ref) <= 1e-9
    batch.close()


def test_batched_single_pass_without_check(td):
    N, M, K, p = 128, 128, 24, 8
    sys = synth.varcoef_system(N, M, seed=500)
    F = synth.rhs_columns(500, N, M, range(K))
    plan = td.Plan.from_system(sys, subdomains=p)
    Fd = torch.as_tensor(F, device="cuda")
    X = torch.zeros_like(Fd)
    batch = td.Batch([plan], [Fd], [X], passes=3, tol=-1.0)
    batch.solve()
    infos, ok = batch.info()
    assert ok and infos[0]["max_col_rel_residual"] == -1.0
    assert rel_err(X.cpu().numpy(), oracle.solve(sys, F)) <= 1e-12
    batch.close()


def test_batched_rejects_bf16_plans(td):
    sys = synth.laplace_system(32, 64, 4.5)
    plan = td.Plan.from_system(sys, subdomains=2, sweep_prec="bf16")
    F = torch.zeros((2, 32 * 64), dtype=torch.float64, device="cuda")
    with pytest.raises(td.TridiagError) as e:
        td.Batch([plan], [F], [torch.zeros_like(F)])
    assert e.value.code == 7


def _stencil_residual(sysq, X, F):
    """max over columns of ||F - P X|| / ||F|| for diagonal A, B and tridiagonal C, in plain torch
    float64 on the device (written from the definition of P, independent of the library)."""
    N, M = sysq.N, sysq.M
    K = X.shape[0]
    x = X.view(K, N, M)
    a = torch.as_tensor(sysq.A, device=X.device)
    b = torch.as_tensor(sysq.B, device=X.device)
    c = torch.as_tensor(sysq.C, device=X.device)
    px = c[:, 1, :] * x
    px[:, :, 1:] += c[:, 0, 1:] * x[:, :, :-1]
    px[:, :, :-1] += c[:, 2, :-1] * x[:, :, 1:]
    px[:, 1:, :] -= a[1:] * x[:, :-1, :]
    px[:, :-1, :] -= b[:-1] * x[:, 1:, :]
    r = F.view(K, N, M) - px
    return float((r.reshape(K, -1).norm(dim=1) / F.norm(dim=1)).max())


def test_batched_largest_systems(td):
    """The eight systems of the 64-system batched workload with the most sweep work (all M = 256;
    N up to 3600, K up to 478) in one batch, float32 sweeps with float64 refinement, default
    subdomain counts: every column's residual <= 1e-10 (plain torch stencil), and samples of
    columns 0, K/2 and K-1 within 1e-9 of the oracle (tests/golden/batched_64_largest.json)."""
    import json

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batched_64_largest.json")
    with open(path) as f:
        gold = json.load(f)
    plans, Fs, Xs, systems = [], [], [], []
    for ent in gold["systems"]:
        N, M, K, seed = ent["N"], ent["M"], ent["K"], ent["seed"]
        sysq = synth.laplace_system(N, M, 4.5)
        plans.append(td.Plan.from_system(sysq, subdomains=td.choose_subdomains(N, M, K, "f32"), sweep_prec="f32"))
        Fs.append(synth.rhs_torch(seed, N, M, K, "cuda"))
        Xs.append(torch.zeros_like(Fs[-1]))
        systems.append(sysq)
    batch = td.Batch(plans, Fs, Xs, passes=3, tol=1e-10)
    batch.solve()
    infos, ok = batch.info()
    assert ok, infos
    worst = 0.0
    for q, ent in enumerate(gold["systems"]):
        assert infos[q]["max_col_rel_residual"] <= 1e-10
        assert _stencil_residual(systems[q], Xs[q], Fs[q]) <= 1e-10
        for smp in ent["samples"]:
            idx = torch.as_tensor(smp["index"], dtype=torch.int64, device="cuda")
            got = Xs[q][smp["column"]].index_select(0, idx).cpu().numpy()
            ref = np.array([float(v) for v in smp["value"]])
            worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    assert worst <= 1e-9, worst
    batch.close()
    for p in plans:
        p.close()
    del plans, Fs, Xs
    torch.cuda.empty_cache()

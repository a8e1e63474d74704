"""The autotuner (tridiag_autotune over subdomain lengths, tridiag_autotune_tiles over lengths and
launch shapes, timed on the device) and the binding's cache: the search returns one of the
candidates, writes its entry keyed by (architecture, M, K bucket, precision), and choose_subdomains
and plans built with the default subdomain count then use that length (and its launch shapes);
without an entry the library's default rule applies.  Every launch shape gives the same solution
(the same products in the same order), checked bit for bit against the default shapes and against
the oracle."""
import numpy as np
import json
import os

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1108_4181_amd as m

    m.load_library()
    return m


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_autotune_writes_and_uses_cache(td, tmp_path, monkeypatch, prec):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("TD_AUTOTUNE_CACHE", str(cache))
    M, K, N = 64, 40, 1000
    assert td.choose_subdomains(N, M, K, prec) == td.default_subdomains(N, K)
    cands = (8, 16, 32)
    res = td.autotune(M, K, prec, probe_N=256, candidates=cands, tiles=False)
    assert res["L"] in cands
    assert set(res["ms_per_solve"]) == {str(c) for c in cands}
    assert all(v > 0.0 for v in res["ms_per_solve"].values())
    with open(cache) as f:
        entry = json.load(f)[f"gfx950|M{M}|K{td._kbucket(K)}|{prec}"]
    assert entry["L"] == res["L"]
    assert td.choose_subdomains(N, M, K, prec) == N // res["L"]
    # the tuned length is used by a plan built with the default subdomain count
    plan = td.Plan(torch.ones((N, M), dtype=torch.float64, device="cuda"),
                   torch.ones((N, M), dtype=torch.float64, device="cuda"),
                   _laplace_C(N, M), N, M, sweep_prec=prec, k_hint=K)
    assert plan.plan_info()["subdomains"] == N // res["L"]
    plan.close()


def _laplace_C(N, M):
    C = torch.empty((N, 3, M), dtype=torch.float64, device="cuda")
    C[:, 0, :] = -1.0
    C[:, 1, :] = 4.5
    C[:, 2, :] = -1.0
    return C


@pytest.mark.parametrize("prec,M", [("f64", 64), ("f64", 256), ("f32", 256), ("bf16", 128)])
def test_autotune_tiles_writes_and_applies(td, tmp_path, monkeypatch, prec, M):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("TD_AUTOTUNE_CACHE", str(cache))
    K, N = 40, 512
    cands = (16, 32)
    res = td.autotune(M, K, prec, probe_N=128, candidates=cands)
    assert res["L"] in cands and res["ms_per_solve"] > 0.0
    assert set(res["tiles"]) == set(td.TILE_FIELDS)
    with open(cache) as f:
        entry = json.load(f)[f"gfx950|M{M}|K{td._kbucket(K)}|{prec}"]
    assert entry["tiles"] == res["tiles"]
    plan = td.Plan(torch.ones((N, M), dtype=torch.float64, device="cuda"),
                   torch.ones((N, M), dtype=torch.float64, device="cuda"),
                   _laplace_C(N, M), N, M, sweep_prec=prec, k_hint=K)
    assert plan.plan_info()["subdomains"] == N // res["L"]
    assert plan.get_tiles() == res["tiles"]
    plan.close()


@pytest.mark.parametrize("prec,M,K", [("f64", 256, 70), ("f64", 512, 40), ("f64", 64, 33), ("f32", 256, 100),
                                      ("f32", 512, 70), ("bf16", 128, 70)])
def test_every_launch_shape_gives_the_same_solution(td, prec, M, K):
    """Each alternative column count and wave count of the sweeps and of the superposition, alone and
    combined (the launchers ignore the ones a block size does not allow), solves the system: float64
    plans agree with the default shapes to 1e-13 (bit for bit but for the summation order of the
    half-panel superposition above block size 256, which adds the interface halves in an order that
    alternates by row) and with the oracle to 1e-12; refined low-precision plans reach 1e-10."""
    import oracle
    import synth
    from dense_ref import rel_err

    N, p = 24, 4
    sysw = synth.varcoef_system(N, M, seed=900 + M + K)
    F = synth.rhs_columns(900 + M, N, M, range(K))
    Fd = torch.as_tensor(np.ascontiguousarray(F), dtype=torch.float64, device="cuda")
    ref_o = oracle.solve(sysw, F)
    plan = td.Plan.from_system(sysw, subdomains=p, sweep_prec=prec, tiles=None)
    refine = None if prec == "f64" else {"tol": 1e-10, "max_iter": 10}
    ref, _ = plan.solve(Fd, refine=refine, info=True)
    cols = (8, 16, 32) if prec == "f64" else (16, 32, 64)
    waves = (1, 2, 3, 4, 5, 6, 7, 8)
    shapes = [dict(sweep_cols=c) for c in cols] + [dict(sup_cols=c) for c in cols]
    shapes += [dict(sweep_waves=w) for w in waves] + [dict(sup_waves=w) for w in waves]
    shapes += [dict(sweep_cols=cols[0], sweep_waves=2, sup_cols=cols[-1], sup_waves=4)]
    for t in shapes:
        plan.set_tiles(**t)
        assert plan.get_tiles() == {k: t.get(k, 0) for k in td.TILE_FIELDS}
        X, info = plan.solve(Fd, refine=refine, info=True)
        X2 = plan.solve(Fd, refine=refine)          # the captured graph of this shape
        if prec == "f64":
            assert rel_err(X.cpu().numpy(), ref.cpu().numpy()) <= 1e-13, t
            assert rel_err(X.cpu().numpy(), ref_o) <= 1e-12, t
            assert torch.equal(X2, X), t
        else:
            assert info["max_col_rel_residual"] <= 1e-10, t
            assert rel_err(X.cpu().numpy(), ref_o) <= 1e-9, t
    plan.set_tiles()
    assert plan.get_tiles() == {k: 0 for k in td.TILE_FIELDS}
    plan.close()

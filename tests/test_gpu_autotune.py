"""The subdomain-length autotuner (tridiag_autotune, timed on the device) and the binding's cache:
the search returns one of the candidates with a time for each, writes its entry keyed by
(architecture, M, K bucket, precision), and choose_subdomains then uses that length; without an
entry it falls back to the library's default rule."""
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
    res = td.autotune(M, K, prec, probe_N=256, candidates=cands)
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

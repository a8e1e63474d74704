"""Band matrices through their block-tridiagonal form (tridiag_band_to_blocks + a float64 plan with
dense triangular couplings) against scipy's banded LU solver on the CPU (float64, relative error
<= 1e-12), including n not a multiple of the block size, a block size above the bandwidth, one
empty side (kl = 0) and the transposed solve."""
import numpy as np
import pytest
import scipy.linalg

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1108_4181_amd as m

    m.load_library()
    return m


def band_matrix(n, kl, ku, seed):
    """General band storage (LAPACK / scipy layout, (kl+ku+1) x n) of a diagonally dominant matrix."""
    ab = synth.uniform_range(seed, 11, 0, (kl + ku + 1) * n, -1.0, 1.0).reshape(kl + ku + 1, n)
    ab[ku, :] = (kl + ku + 1) * 1.5 + np.abs(ab[ku, :])
    for d in range(kl + ku + 1):   # entries outside the matrix are unused; zero them
        off = ku - d               # column j holds a(j - off, j)
        for j in range(n):
            i = j - off
            if i < 0 or i >= n:
                ab[d, j] = 0.0
    return ab


def rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


@pytest.mark.parametrize("n,kl,ku,M,p,K", [
    (1000, 7, 5, 0, 0, 9), (999, 3, 8, 8, 16, 4), (257, 0, 4, 4, 8, 3), (64, 6, 6, 16, 2, 5), (5, 2, 1, 4, 1, 2),
])
def test_band_matches_scipy(td, n, kl, ku, M, p, K):
    ab = band_matrix(n, kl, ku, seed=900 + n)
    F = synth.rhs_columns(900 + n, n, 1, range(K))          # (K, n)
    ref = scipy.linalg.solve_banded((kl, ku), ab, F.T).T
    solver = td.BandSolver(torch.as_tensor(np.ascontiguousarray(ab.T), device="cuda"), kl, ku, M=M, subdomains=p)
    X = solver.solve(torch.as_tensor(F, device="cuda")).cpu().numpy()
    assert rel(X, ref) <= 1e-12


def test_band_transposed(td):
    n, kl, ku = 300, 4, 2
    ab = band_matrix(n, kl, ku, seed=951)
    G = synth.rhs_columns(951, n, 1, range(3))
    dense = np.zeros((n, n))
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            dense[i, j] = ab[ku + i - j, j]
    ref = np.linalg.solve(dense.T, G.T).T
    solver = td.BandSolver(torch.as_tensor(np.ascontiguousarray(ab.T), device="cuda"), kl, ku, subdomains=6,
                           adjoint=True)
    Lam = solver.solve_adjoint(torch.as_tensor(G, device="cuda")).cpu().numpy()
    assert rel(Lam, ref) <= 1e-12

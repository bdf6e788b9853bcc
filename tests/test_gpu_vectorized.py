"""GPU parity of the vectorized solve with general commutativity operators (fmap_solve_vectorized) against the
float64 oracle: the register row solve (n = kx ky <= 64) and the tiled one (64 < n <= 319), square and
rectangular maps, non-symmetric operators; diagonal operators against fmap_solve; invalid lambda and
unsupported sizes."""
import numpy as np
import pytest

from oracle import vectorized as vz
import oracle
from paper_2604_10377_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5  # relative Frobenius error of C, float32 arithmetic against float64


@pytest.fixture(scope="module")
def F():
    from paper_2604_10377_amd import fmap
    return fmap


@pytest.fixture(scope="module")
def dev():
    import torch
    return torch.device("cuda:0")


def T(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def rel_fro(x, r):
    return float(np.linalg.norm(x - r) / np.linalg.norm(r))


# (P, kx, ky, d, lam, skew): n = kx ky spans the register solve's widths (25, 56, 64) and the tiled instances
# (81 and 120: 4 tile rows; 196: 7; 256, 300, 306, 315 and 319: 10), with d close to kx in one case (A A^T less
# well conditioned); kx or ky above 32 (35 x 9, 3 x 100) forms H without the LDS staging; the 1 x 1 map and
# one-sided maps (kx = 1 or ky = 1)
CASES = [(3, 5, 5, 32, 0.5, 0.3), (2, 7, 8, 40, 1.0, 0.3), (2, 8, 8, 64, 2.0, 0.3), (2, 9, 9, 64, 0.5, 0.3),
         (2, 4, 30, 40, 1.0, 0.3), (2, 14, 14, 96, 0.5, 0.3), (2, 16, 16, 128, 1.0, 0.3),
         (1, 17, 18, 128, 0.5, 0.3), (2, 29, 11, 64, 1.0, 0.3), (2, 12, 10, 14, 0.2, 0.2),
         (2, 35, 9, 64, 0.5, 0.3), (1, 3, 100, 128, 0.5, 0.3),
         (1, 1, 1, 8, 0.5, 0.3), (2, 1, 40, 16, 1.0, 0.3), (2, 40, 1, 64, 1.0, 0.3)]


@pytest.mark.parametrize("P,kx,ky,d,lam,skew", CASES)
def test_vectorized_solve_matches_oracle(F, dev, P, kx, ky, d, lam, skew):
    A, B, D1, D2, lamv = synth.workload_vectorized(P, kx, d, ky=ky, lam=lam, skew=skew, tag=81)
    C, info = F.fmap_solve_vectorized(T(A, dev), T(B, dev), T(D1, dev), T(D2, dev), T(lamv, dev))
    C, info = C.cpu().numpy(), info.cpu().numpy()
    assert (info == 0).all(), info
    for p in range(P):
        ref = vz.solve(A[p], B[p], D1[p], D2[p], float(lamv[p]))
        assert rel_fro(C[p], ref) <= TOL, (p, rel_fro(C[p], ref))


@pytest.mark.parametrize("k,d", [(6, 48), (12, 96), (17, 128)])
def test_diagonal_operators_equal_row_wise_solve(F, dev, k, d):
    """Eigenvalue operators: the same map as fmap_solve with the Laplacian mask (and as the row-wise oracle)."""
    import torch
    P = 2
    A, B, _, _, lamv = synth.workload_vectorized(P, k, d, lam=0.7, tag=82)
    rng = np.random.default_rng(5)
    ex = np.sort(rng.uniform(0, 2, (P, k)), axis=1).astype(np.float32)
    ey = np.sort(rng.uniform(0, 2, (P, k)), axis=1).astype(np.float32)
    D1 = np.stack([np.diag(e) for e in ex]).astype(np.float32)
    D2 = np.stack([np.diag(e) for e in ey]).astype(np.float32)
    C, info = F.fmap_solve_vectorized(T(A, dev), T(B, dev), T(D1, dev), T(D2, dev), T(lamv, dev))
    Crow = F.fmap_solve(T(A, dev), T(B, dev), T(ex, dev), T(ey, dev), T(lamv, dev), 0, 0.5)[0]
    torch.cuda.synchronize()
    C, Crow = C.cpu().numpy(), Crow.cpu().numpy()
    assert (info.cpu().numpy() == 0).all()
    for p in range(P):
        ref, _ = oracle.solve(A[p], B[p], oracle.mask(ex[p], ey[p], 0), float(lamv[p]))
        assert rel_fro(C[p], ref) <= TOL
        assert rel_fro(C[p], Crow[p]) <= 2 * TOL


def test_invalid_lambda_and_unsupported_size(F, dev):
    A, B, D1, D2, lamv = synth.workload_vectorized(3, 10, 64, lam=0.5, tag=83)
    lamv = lamv.copy()
    lamv[1] = -1.0
    C, info = F.fmap_solve_vectorized(T(A, dev), T(B, dev), T(D1, dev), T(D2, dev), T(lamv, dev))
    C, info = C.cpu().numpy(), info.cpu().numpy()
    assert info[1] == -1 and np.isnan(C[1]).all()
    for p in (0, 2):
        assert info[p] == 0
        assert rel_fro(C[p], vz.solve(A[p], B[p], D1[p], D2[p], float(lamv[p]))) <= TOL
    A2, B2, D12, D22, l2 = synth.workload_vectorized(1, 18, 64, lam=0.5, tag=84)  # n = 324 > 319
    with pytest.raises(RuntimeError):
        F.fmap_solve_vectorized(T(A2, dev), T(B2, dev), T(D12, dev), T(D22, dev), T(l2, dev))


def test_full_bench_batch_sampled(F, dev):
    """The bench's batch (256 pairs, k = 16, d = 256) in the bench's launch configuration, pairs sampled."""
    A, B, D1, D2, lamv = synth.workload_vectorized()
    C, info = F.fmap_solve_vectorized(T(A, dev), T(B, dev), T(D1, dev), T(D2, dev), T(lamv, dev))
    C, info = C.cpu().numpy(), info.cpu().numpy()
    assert (info == 0).all()
    for p in (0, 97, 255):
        assert rel_fro(C[p], vz.solve(A[p], B[p], D1[p], D2[p], float(lamv[p]))) <= TOL

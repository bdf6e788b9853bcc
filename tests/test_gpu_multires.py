"""GPU parity of the maps at several spectral resolutions and of the projection with the projector given
directly, against the oracle (relative Frobenius error <= 1e-5; info bit-exact)."""
import numpy as np
import pytest

import oracle
from paper_2604_10377_amd import synth
from tests.conftest import rel_fro
from tests.test_gpu_parity import _spectral, T, N

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def F(dev):
    from paper_2604_10377_amd import fmap
    return fmap


# the register row solve (k_x' <= 64), the tiled one, square and rectangular resolutions, the full one
RES_CASES = [(3, 64, 64, 160, [(30, 30), (50, 50), (20, 40), (64, 64), (1, 1), (64, 8)]),
             (2, 200, 200, 420, [(50, 50), (120, 120), (200, 200), (80, 150), (150, 64)]),
             (2, 40, 70, 150, [(40, 70), (10, 70), (40, 5)])]


@pytest.mark.parametrize("mask", [0, 1])
@pytest.mark.parametrize("P,kx,ky,d,res", RES_CASES)
def test_solve_resolutions(F, dev, mask, P, kx, ky, d, res):
    A, B, ex, ey, lam = _spectral(31, P, kx, ky, d)
    print("resolutions", P, kx, ky, d, res, "mask", mask, flush=True)
    out = F.fmap_solve_resolutions(T(A, dev), T(B, dev), T(ex, dev), T(ey, dev), T(lam, dev), mask, 0.5, res)
    for p in range(P):
        for (C, info), r in zip(out, res):
            if mask == 1 and max(ex[p, :r[0]].max(), ey[p, :r[1]].max()) <= 0:
                # truncated spectra {mu_0 = 0}: the resolvent normaliser is not positive (info -2, NaN rows)
                assert (N(info)[p] == -2).all() and np.isnan(N(C)[p]).all(), (p, r)
                continue
            (Cr, ir), = oracle.solve_resolutions(A[p], B[p], ex[p], ey[p], float(lam[p]), mask, 0.5, [r[0]], [r[1]])
            assert np.array_equal(N(info)[p], ir), (p, r)
            assert rel_fro(N(C)[p], Cr) <= TOL, (p, r, rel_fro(N(C)[p], Cr))


def test_solve_resolutions_headline_projection(F, dev):
    """One projection at k = 200 of headline-like pairs (n = 5000, d = 256), maps at five resolutions."""
    b = synth.make_batch("multires-k200", 13, 4, 5000, 200, 256, mask=synth.MASK_LAPLACIAN)
    P = b.pairs
    AB = F.fmap_project(T(b.phi, dev), T(b.mass, dev), T(b.feat, dev))
    res = [(30, 30), (50, 50), (80, 80), (120, 120), (200, 200)]
    out = F.fmap_solve_resolutions(AB[:P], AB[P:], T(b.evals_x, dev), T(b.evals_y, dev), T(b.lam, dev), b.mask,
                                   b.gamma, res)
    for p in (0, P - 1):
        A = oracle.project(b.phi[p], b.mass[p], b.feat[p])
        B = oracle.project(b.phi[P + p], b.mass[P + p], b.feat[P + p])
        refs = oracle.solve_resolutions(A, B, b.evals_x[p], b.evals_y[p], float(b.lam[p]), b.mask, b.gamma,
                                        [r[0] for r in res], [r[1] for r in res])
        for (C, _), (Cr, _), r in zip(out, refs, res):
            assert rel_fro(N(C)[p], Cr) <= TOL, (p, r)


def test_solve_resolutions_argument_errors(F, dev):
    A, B, ex, ey, lam = _spectral(32, 2, 20, 20, 48)
    args = [T(A, dev), T(B, dev), T(ex, dev), T(ey, dev), T(lam, dev), 0, 0.5]
    for bad in ([(21, 5)], [(0, 3)], [(5, 21)]):
        with pytest.raises(F.FmapError):
            F.fmap_solve_resolutions(*args, bad)


@pytest.mark.parametrize("b,n,k,d", [(2, 5000, 50, 256), (3, 1234, 30, 128), (1, 2052, 200, 384), (2, 999, 17, 33)])
def test_project_pinv(F, dev, b, n, k, d):
    """A = P^T F and dF = P dA with P = (Phi^+)^T given directly (float32)."""
    rng = np.random.default_rng(33)
    P = (rng.standard_normal((b, n, k)) / np.sqrt(n)).astype(np.float32)
    feat = rng.standard_normal((b, n, d)).astype(np.float32)
    dA = rng.standard_normal((b, k, d)).astype(np.float32)
    A = N(F.fmap_project_pinv(T(P, dev), T(feat, dev)))
    dF = N(F.fmap_project_pinv_backward(T(P, dev), T(dA, dev)))
    for s in range(b):
        assert rel_fro(A[s], oracle.project_pinv(P[s], feat[s])) <= TOL
        assert rel_fro(dF[s], oracle.project_pinv_backward(P[s], dA[s])) <= TOL


def test_project_pinv_moore_penrose_basis(F, dev):
    """Eq. (1) literally: the Moore-Penrose pseudo-inverse of a (non-orthonormal) basis; F = Phi X gives X."""
    rng = np.random.default_rng(34)
    n, k, d = 3000, 40, 64
    Phi = rng.standard_normal((n, k))
    X = rng.standard_normal((k, d))
    P = np.linalg.pinv(Phi).T.astype(np.float32)[None]
    feat = (Phi @ X).astype(np.float32)[None]
    A = N(F.fmap_project_pinv(T(P, dev), T(feat, dev)))[0]
    assert rel_fro(A, oracle.project_pinv(P[0], feat[0])) <= TOL
    assert rel_fro(A, X) <= 1e-4  # float32 inputs: X up to the rounding of P and F

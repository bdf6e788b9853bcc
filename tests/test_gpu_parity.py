"""GPU parity: every HIP entry point against the FP64 oracle on the same seeded inputs.

Tolerance: relative Frobenius error <= 1e-5 for every float32 array result
(C, factors, dA, dB, dF), per item, on well-conditioned inputs (d >= 2k for
random spectral data, so cond(A A^T) stays below ~40 and float32 rounding of
the products and of the factorisation stays near 1e-6).  The scalar dlambda
is a sum of k^2 cancelling terms; its error is bounded by 1e-5 times the sum
of the terms' magnitudes.  Integer results (info) are bit-exact.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2604_10377_amd import synth
from tests.conftest import rel_fro

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def F(dev):
    from paper_2604_10377_amd import fmap
    return fmap


def T(x, dev, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def N(t):
    return t.detach().cpu().numpy()


def _shapes(seed, b, n, k, d, bf16=False):
    rng = np.random.default_rng(seed)
    mass = (rng.uniform(0.5, 1.5, (b, n)) / n).astype(np.float32)
    phi = rng.standard_normal((b, n, k)).astype(np.float32)
    feat = rng.standard_normal((b, n, d)).astype(np.float32)
    if bf16:
        phi = synth.bf16_bits_to_f32(synth.to_bf16_bits(phi)).reshape(phi.shape)
        feat = synth.bf16_bits_to_f32(synth.to_bf16_bits(feat)).reshape(feat.shape)
    return phi, mass, feat


# ----------------------------------------------------------------------------- projection

# the last group takes the LDS-pipelined kernels (n % 4 == 0, k <= 64): tail stages, every
# remainder width of k mod 16, partial and multiple 256-column blocks
LDS_CASES = [(2, 4004, 30, 128), (3, 2048, 17, 200), (2, 640, 52, 256), (1, 1000, 64, 512), (2, 4000, 49, 256),
             (1, 516, 16, 8), (2, 1028, 35, 260), (1, 8192, 50, 256)]
# float32 operands split for the bf16 matrix cores (k even <= 64, n % 4 == 0, d % 4 == 0): most cases
# above, plus the smallest k with a partial second column block and a narrow block at k = 62
SPLIT_CASES = [(2, 1028, 4, 260), (1, 2052, 62, 36)]
# k > 64 (k % 4 == 0): the basis is taken in 64-row slices; partial last slices and column blocks
SLICED_CASES = [(2, 4004, 80, 256), (1, 2052, 300, 516), (3, 1024, 128, 64), (1, 8192, 68, 260)]


@pytest.mark.parametrize("b,n,k,d", [(1, 1, 1, 1), (2, 37, 5, 7), (3, 1234, 30, 128), (2, 5000, 50, 256),
                                     (1, 4097, 64, 300), (2, 999, 65, 33), (1, 20011, 120, 256)] + LDS_CASES + SPLIT_CASES
                         + SLICED_CASES)
def test_project_forward(F, dev, b, n, k, d):
    import torch
    phi, mass, feat = _shapes(1, b, n, k, d)
    A = N(F.fmap_project(T(phi, dev), T(mass, dev), T(feat, dev)))
    torch.cuda.synchronize()
    for s in range(b):
        ref = oracle.project(phi[s], mass[s], feat[s])
        assert rel_fro(A[s], ref) <= TOL, (s, rel_fro(A[s], ref))


@pytest.mark.parametrize("b,n,k,d", [(2, 777, 30, 128), (1, 5000, 50, 256)])
def test_project_forward_bf16_inputs(F, dev, b, n, k, d):
    """bf16 basis/features: compared with the oracle fed the same bf16-rounded values."""
    import torch
    phi, mass, feat = _shapes(2, b, n, k, d, bf16=True)
    A = N(F.fmap_project(T(phi, dev, torch.bfloat16), T(mass, dev), T(feat, dev, torch.bfloat16)))
    for s in range(b):
        assert rel_fro(A[s], oracle.project(phi[s], mass[s], feat[s])) <= TOL


# bf16 matrix-core forward (k % 8 == 0, k <= 256, d % 8 == 0, n % 4 == 0): every row-slab
# width (k <= 64, <= 128, <= 256), partial row and column blocks, a 4-vertex tail stage,
# the smallest k, and the mixed-precision workload's shape.  basis x mass is split into
# two bf16 parts (product error <= 2^-16 relative), so the float32 bar applies.
BF16_MFMA_CASES = [(2, 4000, 200, 384), (1, 2048, 128, 256), (2, 1024, 64, 520), (1, 3000, 8, 16),
                   (3, 4004, 96, 136), (2, 132, 256, 64), (1, 50000, 200, 384)]


@pytest.mark.parametrize("b,n,k,d", BF16_MFMA_CASES)
def test_project_forward_bf16_matrix_cores(F, dev, b, n, k, d):
    import torch
    print("bf16 mfma projection", b, n, k, d, flush=True)
    phi, mass, feat = _shapes(6, b, n, k, d, bf16=True)
    A = N(F.fmap_project(T(phi, dev, torch.bfloat16), T(mass, dev), T(feat, dev, torch.bfloat16)))
    for s in range(b):
        err = rel_fro(A[s], oracle.project(phi[s], mass[s], feat[s]))
        assert err <= TOL, (s, err)


# bf16 matrix-core backward (k % 8 == 0, k <= 256): dA is split into two bf16 parts, so the
# float32 bar applies; partial column blocks, ragged n, smallest and largest k.
@pytest.mark.parametrize("b,n,k,d", [(2, 4000, 200, 384), (1, 1000, 8, 20), (3, 777, 256, 130), (2, 3001, 64, 128),
                                     (1, 50000, 200, 384)])
def test_project_backward_bf16_matrix_cores(F, dev, b, n, k, d):
    import torch
    print("bf16 mfma projection backward", b, n, k, d, flush=True)
    phi, mass, _ = _shapes(7, b, n, k, d, bf16=True)
    dA = np.random.default_rng(8).standard_normal((b, k, d)).astype(np.float32)
    dF = N(F.fmap_project_backward(T(phi, dev, torch.bfloat16), T(mass, dev), T(dA, dev)))
    for s in range(b):
        err = rel_fro(dF[s], oracle.project_backward(phi[s], mass[s], dA[s]))
        assert err <= TOL, (s, err)


# float32 backward with 64 < k <= 319, k even (64-column blocks, every K step's dA^T parts in LDS): partial
# column blocks, partial vertex tiles, d % 4 != 0 (element stores), three to ten K steps of 32 (k = 120 and
# k = 150 are the uneven workload's large groups: four and five K steps)
BWDK_CASES = [(2, 1028, 80, 260), (1, 2052, 300, 516), (1, 999, 130, 33), (2, 4004, 318, 64), (1, 600, 66, 8),
              (2, 3001, 120, 256), (1, 20000, 120, 256), (1, 2500, 150, 200), (2, 1500, 96, 128)]


@pytest.mark.parametrize("b,n,k,d", [(1, 1, 1, 1), (2, 37, 5, 7), (3, 1234, 30, 128), (2, 5000, 50, 256),
                                     (1, 4097, 64, 300), (2, 999, 65, 33)] + LDS_CASES + SPLIT_CASES + BWDK_CASES)
def test_project_backward(F, dev, b, n, k, d):
    phi, mass, _ = _shapes(3, b, n, k, d)
    dA = np.random.default_rng(4).standard_normal((b, k, d)).astype(np.float32)
    dF = N(F.fmap_project_backward(T(phi, dev), T(mass, dev), T(dA, dev)))
    for s in range(b):
        assert rel_fro(dF[s], oracle.project_backward(phi[s], mass[s], dA[s])) <= TOL


# ----------------------------------------------------------------------------- solve

def _spectral(seed, P, kx, ky, d):
    rng = synth.rng_for(555, seed, kx, ky)
    A = rng.standard_normal((P, kx, d)).astype(np.float32)
    B = rng.standard_normal((P, ky, d)).astype(np.float32)
    ex = np.stack([synth.eigenvalues_linear(rng, kx) for _ in range(P)]).astype(np.float32)
    ey = np.stack([synth.eigenvalues_linear(rng, ky) for _ in range(P)]).astype(np.float32)
    lam = (10.0 ** rng.uniform(-3, 0, P)).astype(np.float32)
    return A, B, ex, ey, lam


def _oracle_solve(A, B, ex, ey, lam, mask, gamma, dC=None):
    out = []
    for p in range(A.shape[0]):
        D = oracle.mask(ex[p], ey[p], mask, gamma)
        C, info, L = oracle.solve(A[p], B[p], D, float(lam[p]), return_factors=True)
        r = dict(C=C, info=info, L=L, D=D)
        if dC is not None:
            r["dA"], r["dB"], r["dl"] = oracle.solve_backward(A[p], B[p], C, D, float(lam[p]), dC[p])
            # error scale of the scalar dlambda = -sum_ij V_ij D_ij C_ij: a float32 sum of k^2 terms
            # is accurate relative to sum |terms|, not to |sum| (the terms cancel)
            V = np.stack([scipy.linalg.cho_solve((L[i], True), dC[p][i]) for i in range(L.shape[0])])
            r["dl_scale"] = float(np.sum(np.abs(V * D * C)))
        out.append(r)
    return out


def _unpack_lower_colmajor(packed, m):
    L = np.zeros((m, m))
    idx = 0
    for c in range(m):
        for r in range(c, m):
            L[r, c] = packed[idx]
            idx += 1
    return L


# k_x picks the register row length (the next multiple of 8, or 52 for 49..52): both sides of each boundary
SOLVE_CASES = [(3, 1, 1, 4), (5, 5, 5, 16), (4, 30, 30, 128), (3, 50, 50, 256), (2, 64, 64, 256),
               (3, 17, 33, 80), (2, 40, 23, 96), (7, 32, 32, 64), (2, 52, 52, 128), (2, 53, 41, 128)]


@pytest.mark.parametrize("mask", [0, 1])
@pytest.mark.parametrize("P,kx,ky,d", SOLVE_CASES)
def test_solve_forward(F, dev, mask, P, kx, ky, d):
    if mask == 1 and kx == 1 and ky == 1:
        pytest.skip("resolvent normaliser of a single zero eigenvalue is not positive")
    A, B, ex, ey, lam = _spectral(1, P, kx, ky, d)
    C, fac, info, _ = F.fmap_solve(T(A, dev), T(B, dev), T(ex, dev), T(ey, dev), T(lam, dev), mask, 0.5)
    C, fac, info = N(C), N(fac), N(info)
    ref = _oracle_solve(A, B, ex, ey, lam, mask, 0.5)
    for p in range(P):
        assert (info[p] == 0).all() and (ref[p]["info"] == 0).all()
        assert rel_fro(C[p], ref[p]["C"]) <= TOL, (p, rel_fro(C[p], ref[p]["C"]))
        m = kx * (kx + 1) // 2
        for i in (0, ky // 2, ky - 1):
            Lg = _unpack_lower_colmajor(fac[p, i * m:(i + 1) * m], kx)
            assert rel_fro(Lg, ref[p]["L"][i]) <= TOL


@pytest.mark.parametrize("mask", [0, 1])
@pytest.mark.parametrize("stored", [True, False])
@pytest.mark.parametrize("P,kx,ky,d", SOLVE_CASES)
def test_solve_backward(F, dev, mask, stored, P, kx, ky, d):
    if mask == 1 and kx == 1 and ky == 1:
        pytest.skip("resolvent normaliser of a single zero eigenvalue is not positive")
    A, B, ex, ey, lam = _spectral(2, P, kx, ky, d)
    dC = np.random.default_rng(5).standard_normal((P, ky, kx)).astype(np.float32)
    tA, tB, tex, tey, tl = (T(x, dev) for x in (A, B, ex, ey, lam))
    C, fac, info, _ = F.fmap_solve(tA, tB, tex, tey, tl, mask, 0.5, store_factors=stored)
    dA, dB, dl = F.fmap_solve_backward(T(dC, dev), tA, tB, C, tex, tey, tl, mask, 0.5, fac, want_dlam=True)
    dA, dB, dl = N(dA), N(dB), N(dl)
    # the oracle recomputes its own C from the same inputs; it never consumes GPU results
    ref = _oracle_solve(A, B, ex, ey, lam, mask, 0.5, dC)
    for p in range(P):
        assert rel_fro(dA[p], ref[p]["dA"]) <= TOL, (p, rel_fro(dA[p], ref[p]["dA"]))
        assert rel_fro(dB[p], ref[p]["dB"]) <= TOL, (p, rel_fro(dB[p], ref[p]["dB"]))
        assert abs(dl[p] - ref[p]["dl"]) <= TOL * ref[p]["dl_scale"], (p, dl[p], ref[p]["dl"], ref[p]["dl_scale"])


# Tiled row solve (k_x > 64): tile-boundary sizes, the workspace-tile variant (k_x >= 224), rectangular maps.
# Inputs keep cond(A A^T) near 30 (d = 2k); the float32 bar of 1e-5 holds at every k (measured C <= 1.4e-6,
# gradients <= 1.9e-6 at k = 319).
LARGE_CASES = [(2, 65, 65, 160, TOL), (2, 96, 96, 200, TOL), (2, 127, 127, 256, TOL), (1, 128, 128, 256, TOL),
               (1, 150, 150, 300, TOL), (1, 200, 200, 400, TOL), (1, 223, 223, 450, TOL),
               (1, 224, 224, 450, TOL), (1, 300, 300, 600, TOL), (1, 319, 319, 640, TOL),
               (2, 100, 40, 200, TOL), (2, 30, 100, 128, TOL)]


@pytest.mark.parametrize("mask", [0, 1])
@pytest.mark.parametrize("P,kx,ky,d,tol", LARGE_CASES)
def test_solve_large_k(F, dev, mask, P, kx, ky, d, tol):
    A, B, ex, ey, lam = _spectral(11, P, kx, ky, d)
    dC = np.random.default_rng(6).standard_normal((P, ky, kx)).astype(np.float32)
    tA, tB, tex, tey, tl = (T(x, dev) for x in (A, B, ex, ey, lam))
    C, fac, info, _ = F.fmap_solve(tA, tB, tex, tey, tl, mask, 0.5)
    Cr = N(C)
    ref = _oracle_solve(A, B, ex, ey, lam, mask, 0.5, dC)
    for p in range(P):
        assert (N(info)[p] == 0).all()
        assert rel_fro(Cr[p], ref[p]["C"]) <= tol, (p, rel_fro(Cr[p], ref[p]["C"]))
    m = kx * (kx + 1) // 2
    facn = N(fac)
    for i in (0, ky - 1):
        Lg = _unpack_lower_colmajor(facn[0, i * m:(i + 1) * m], kx)
        assert rel_fro(Lg, ref[0]["L"][i]) <= tol
    for stored in (True, False):
        dA, dB, dl = F.fmap_solve_backward(T(dC, dev), tA, tB, C, tex, tey, tl, mask, 0.5,
                                           fac if stored else None, want_dlam=True)
        dA, dB, dl = N(dA), N(dB), N(dl)
        for p in range(P):
            assert rel_fro(dA[p], ref[p]["dA"]) <= tol, (stored, p, rel_fro(dA[p], ref[p]["dA"]))
            assert rel_fro(dB[p], ref[p]["dB"]) <= tol, (stored, p, rel_fro(dB[p], ref[p]["dB"]))
            assert abs(dl[p] - ref[p]["dl"]) <= tol * ref[p]["dl_scale"]


def test_solve_large_k_info_convention(F, dev):
    """Zero pivot inside a later block column of the tiled path: info = j+1, NaN row."""
    P, k, d = 2, 150, 300
    A, B, ex, ey, lam = _spectral(12, P, k, k, d)
    A[0, 100] = 0.0
    lam[0] = 0.0
    lam[1] = -2.0
    C, _, info, _ = F.fmap_solve(T(A, dev), T(B, dev), T(ex, dev), T(ey, dev), T(lam, dev), 0, 0.5)
    C, info = N(C), N(info)
    assert (info[0] == 101).all() and np.isnan(C[0]).all()
    assert (info[1] == -1).all() and np.isnan(C[1]).all()


def test_solve_info_convention(F, dev):
    """-1 for a bad lambda, j+1 for an exactly zero pivot, -2 for a zero resolvent normaliser; NaN rows."""
    import torch
    P, k, d = 4, 12, 40
    A, B, ex, ey, lam = _spectral(3, P, k, k, d)
    lam[0] = -1.0
    lam[1] = np.nan
    A[2, 5] = 0.0          # zero row 5 of A ...
    lam[2] = 0.0           # ... with lambda = 0: every row system has an exactly zero pivot 6
    ey[3, 4] = ex[3, 7]    # pair 3: row 4's mask entry at column 7 vanishes; zero row 7 makes that pivot 0
    A[3, 7] = 0.0
    C, _, info, _ = F.fmap_solve(T(A, dev), T(B, dev), T(ex, dev), T(ey, dev), T(lam, dev), 0, 0.5)
    C, info = N(C), N(info)
    assert (info[0] == -1).all() and np.isnan(C[0]).all()
    assert (info[1] == -1).all() and np.isnan(C[1]).all()
    assert (info[2] == 6).all() and np.isnan(C[2]).all()
    ref3 = _oracle_solve(A[3:], B[3:], ex[3:], ey[3:], lam[3:], 0, 0.5)[0]
    np.testing.assert_array_equal(info[3], ref3["info"])
    assert info[3, 4] == 8 and np.isnan(C[3, 4]).all()
    ok = ref3["info"] == 0
    assert rel_fro(C[3][ok], ref3["C"][ok]) <= TOL
    # resolvent with all-zero eigenvalues
    z = np.zeros((1, k), np.float32)
    C, _, info, _ = F.fmap_solve(T(A[:1], dev), T(B[:1], dev), T(z, dev), T(z, dev),
                                 T(np.ones(1, np.float32), dev), 1, 0.5)
    assert (N(info) == -2).all() and np.isnan(N(C)).all()
    torch.cuda.synchronize()


@pytest.mark.parametrize("kx", [50, 150])
def test_solve_backward_stored_info_convention(F, dev, kx):
    """Reverse mode with stored factors: a non-positive pivot (column 5) in one system's factor reports
    info = 6 for that row system alone, an invalid lambda reports -1 for every row of its pair, and the
    failed systems' solutions are NaN (the register path k_x <= 64 and the streaming path above)."""
    import torch
    P, ky, d = 2, 20, 2 * kx
    A, B, ex, ey, lam = _spectral(4, P, kx, ky, d)
    tA, tB, tex, tey, tl = (T(x, dev) for x in (A, B, ex, ey, lam))
    C, fac, info, _ = F.fmap_solve(tA, tB, tex, tey, tl, 0, 0.5, store_factors=True)
    assert (N(info) == 0).all()
    tri = kx * (kx + 1) // 2
    fac = fac.clone()
    fac[0, 3 * tri + 5 * kx - (5 * 4) // 2] = -1.0  # diagonal entry of column 5, row system 3 of pair 0
    lam_bad = tl.clone()
    lam_bad[1] = -1.0
    ib = torch.full((P, ky), 12345, dtype=torch.int32, device=dev)
    dC = np.random.default_rng(6).standard_normal((P, ky, kx)).astype(np.float32)
    dA, dB, _ = F.fmap_solve_backward(T(dC, dev), tA, tB, C, tex, tey, lam_bad, 0, 0.5, fac, info=ib)
    expect = np.zeros((P, ky), np.int32)
    expect[0, 3] = 6
    expect[1, :] = -1
    np.testing.assert_array_equal(N(ib), expect)
    dB = N(dB)
    others = np.arange(ky) != 3
    assert np.isnan(dB[0, 3]).all() and np.isfinite(dB[0, others]).all()
    assert np.isnan(N(dA)[1]).all() and np.isnan(dB[1]).all()
    torch.cuda.synchronize()


# ----------------------------------------------------------------------------- whole pipeline

def _pipeline_gpu(F, b, dev, bwd="stored"):
    import torch
    feat = T(b.feat, dev).requires_grad_(True)
    C, info = F.functional_map(feat, T(b.phi, dev), T(b.mass, dev), T(b.evals, dev), T(b.lam, dev), b.mask,
                               b.gamma, bwd=bwd)
    C.backward(T(b.dC, dev))
    torch.cuda.synchronize()
    return N(C), N(info), N(feat.grad)


def _pipeline_oracle_pair(b, p):
    P = b.pairs
    A, B, D, C, info = oracle.forward_pair(b.phi[p], b.mass[p], b.feat[p], b.phi[P + p], b.mass[P + p],
                                           b.feat[P + p], b.evals[p], b.evals[P + p], float(b.lam[p]), b.mask, b.gamma)
    dA, dB, _ = oracle.solve_backward(A, B, C, D, float(b.lam[p]), b.dC[p])
    return C, info, oracle.project_backward(b.phi[p], b.mass[p], dA), oracle.project_backward(b.phi[P + p],
                                                                                            b.mass[P + p], dB)


@pytest.mark.parametrize("bwd", ["stored", "recompute"])
def test_pipeline_headline_workload_full_size(F, dev, bwd):
    """32 pairs, n=5000, k=50, d=256, resolvent mask: C and dF of sampled pairs vs the oracle."""
    b = synth.workload_headline()
    C, info, dF = _pipeline_gpu(F, b, dev, bwd)
    assert (info == 0).all()
    P = b.pairs
    for p in (0, 1, 2, 3, 17, P - 1):
        Cr, ir, dFx, dFy = _pipeline_oracle_pair(b, p)
        assert rel_fro(C[p], Cr) <= TOL, (p, rel_fro(C[p], Cr))
        assert rel_fro(dF[p], dFx) <= TOL, (p, rel_fro(dF[p], dFx))
        assert rel_fro(dF[P + p], dFy) <= TOL, (p, rel_fro(dF[P + p], dFy))


def test_pipeline_headline_shape_regulariser_weighted(F, dev):
    """Headline shape (32 pairs, n=5000, k=50, d=256, resolvent mask) with lambda from 1 to 4, where lambda
    times the mean mask entry is 1-5% of the mean diagonal of A A^T (at lambda = 1e-3 it is ~1e-5 of it,
    and C is nearly the lambda = 0 solution):
    C and dF of sampled pairs against the oracle, and the regulariser visibly moves the oracle's C."""
    b = synth.make_batch("headline-shape-lambda1", 12, 32, 5000, 50, 256, mask=synth.MASK_RESOLVENT, gamma=0.5,
                         lam=np.geomspace(1.0, 4.0, 32))
    C, info, dF = _pipeline_gpu(F, b, dev, "stored")
    assert (info == 0).all()
    P = b.pairs
    for p in (0, 13, P - 1):
        Cr, ir, dFx, dFy = _pipeline_oracle_pair(b, p)
        assert rel_fro(C[p], Cr) <= TOL, (p, rel_fro(C[p], Cr))
        assert rel_fro(dF[p], dFx) <= TOL, (p, rel_fro(dF[p], dFx))
        assert rel_fro(dF[P + p], dFy) <= TOL, (p, rel_fro(dF[P + p], dFy))
    A, B, D, Cr, _ = oracle.forward_pair(b.phi[0], b.mass[0], b.feat[0], b.phi[P], b.mass[P], b.feat[P], b.evals[0],
                                         b.evals[P], float(b.lam[0]), b.mask, b.gamma)
    C0, _ = oracle.solve(A, B, D, 0.0)
    assert rel_fro(Cr, C0) >= 1e-2  # the mask term shapes the solution


def test_pipeline_large_workload_full_size(F, dev):
    """Large-basis workload at full size: n=100000, k=300, d=512, resolvent mask, factor recomputation in the
    backward (two pairs: the kernels' split counts and tile ranges depend on n, k and d, not on the number
    of pairs); C and dF of pair 1 against the oracle."""
    b = synth.workload_large(pairs=2)
    print("large workload", b.pairs, b.n, b.k, b.d, flush=True)
    C, info, dF = _pipeline_gpu(F, b, dev, "recompute")
    assert (info == 0).all()
    P, p = b.pairs, 1
    Cr, ir, dFx, dFy = _pipeline_oracle_pair(b, p)
    errs = (rel_fro(C[p], Cr), rel_fro(dF[p], dFx), rel_fro(dF[P + p], dFy))
    print("large pair", p, "errors C, dF_x, dF_y", errs, flush=True)
    assert max(errs) <= TOL, errs


def test_pipeline_plain_workload_full_size(F, dev):
    """1 pair, n=5000, k=30, d=128, Laplacian mask, forward."""
    import torch
    b = synth.workload_plain()
    P = b.pairs
    AB = F.fmap_project(T(b.phi, dev), T(b.mass, dev), T(b.feat, dev))
    C, _, info, _ = F.fmap_solve(AB[:P], AB[P:], T(b.evals_x, dev), T(b.evals_y, dev), T(b.lam, dev), b.mask)
    torch.cuda.synchronize()
    A, B, D, Cr, ir = oracle.forward_pair(b.phi[0], b.mass[0], b.feat[0], b.phi[1], b.mass[1], b.feat[1],
                                          b.evals[0], b.evals[1], float(b.lam[0]), b.mask, b.gamma)
    assert (N(info) == 0).all()
    assert rel_fro(N(C)[0], Cr) <= TOL


def test_pipeline_ragged_small_batch(F, dev):
    """n not a multiple of any tile, several pairs, both backward modes agree with the oracle."""
    b = synth.make_batch("t", 77, 3, 1531, 37, 100, mask=synth.MASK_RESOLVENT)
    for bwd in ("stored", "recompute"):
        C, info, dF = _pipeline_gpu(F, b, dev, bwd)
        for p in range(3):
            Cr, _, dFx, dFy = _pipeline_oracle_pair(b, p)
            assert rel_fro(C[p], Cr) <= TOL
            assert rel_fro(dF[p], dFx) <= TOL and rel_fro(dF[3 + p], dFy) <= TOL


def test_autograd_against_oracle_finite_differences(F, dev):
    """Headline workload, pairs 0-3 (reduced n): GPU gradient wrt features vs FP64 central differences."""
    b = synth.workload_headline(pairs=4, n=800)
    C, info, dF = _pipeline_gpu(F, b, dev)
    P = b.pairs
    for p in range(P):
        args = [b.phi[p], b.mass[p], b.feat[p].astype(np.float64), b.phi[P + p], b.mass[P + p],
                b.feat[P + p].astype(np.float64), b.evals[p], b.evals[P + p], float(b.lam[p]), b.mask, b.gamma]
        rng = np.random.default_rng(100 + p)
        ux, uy = rng.standard_normal(b.feat[p].shape), rng.standard_normal(b.feat[P + p].shape)
        h = 1e-4
        def L_of(t):
            a = list(args)
            a[2] = args[2] + t * ux
            a[5] = args[5] + t * uy
            return float(np.sum(b.dC[p] * oracle.forward_pair(*a)[3]))
        fd = (L_of(h) - L_of(-h)) / (2 * h)
        an = float(np.sum(dF[p] * ux) + np.sum(dF[P + p] * uy))
        # u ~ N(0, I): <e, u> ~ N(0, |e|^2) for a gradient error e, so the scale is |dF|, not |<dF, u>|;
        # a gradient within 1e-5 relative passes with a 5-sigma margin
        scale = float(np.sqrt(np.sum(dF[p] ** 2) + np.sum(dF[P + p] ** 2)))
        assert abs(fd - an) <= 5e-5 * scale, (p, fd, an, scale)
        _, _, dFx, dFy = _pipeline_oracle_pair(b, p)
        assert rel_fro(dF[p], dFx) <= TOL and rel_fro(dF[P + p], dFy) <= TOL


def test_repeat_calls_are_deterministic(F, dev):
    import torch
    b = synth.workload_headline(pairs=4, n=3000)
    r1 = _pipeline_gpu(F, b, dev)
    r2 = _pipeline_gpu(F, b, dev)
    for x, y in zip(r1, r2):
        np.testing.assert_array_equal(x, y)
    torch.cuda.synchronize()


# ----------------------------------------------------------------------------- refinement / conditioning

def _conditioned(seed, P, k, d, sigma_ratio):
    """A with singular values geometric from 1 down to 1/sigma_ratio (cond(A A^T) = sigma_ratio^2)."""
    rng = np.random.default_rng(seed)
    A = np.empty((P, k, d), np.float32)
    for p in range(P):
        U = synth.random_orthogonal(rng, k)
        V = synth.random_orthogonal(rng, d)[:k]
        s = np.geomspace(1.0, 1.0 / sigma_ratio, k)
        A[p] = (U * s[None, :]) @ V
    B = rng.standard_normal((P, k, d)).astype(np.float32) * 0.1
    ex = np.stack([synth.eigenvalues_linear(rng, k) for _ in range(P)]).astype(np.float32)
    ey = np.stack([synth.eigenvalues_linear(rng, k) for _ in range(P)]).astype(np.float32)
    return A, B, ex, ey


# small k: the estimate's last column group reaches past the factor into the allocation's padding;
# 64 / 65 / 129: register-slot boundaries of the solves; 256: the largest order the estimate supports
@pytest.mark.parametrize("k,d,ratio", [(50, 128, 30.0), (50, 128, 300.0), (120, 256, 100.0), (200, 400, 100.0),
                                       (3, 8, 10.0), (7, 16, 30.0), (9, 20, 30.0), (64, 130, 30.0),
                                       (65, 140, 30.0), (129, 260, 30.0), (256, 520, 30.0)])
def test_condition_estimate(F, dev, k, d, ratio):
    """1-norm estimate of cond(A A^T) against the exact value (Hager's estimate is a lower bound, within ~x3)."""
    P = 2
    A, B, ex, ey = _conditioned(21, P, k, d, ratio)
    lam = np.full(P, 1e-3, np.float32)
    _, _, _, cond = F.fmap_solve(T(A, dev), T(B, dev), T(ex, dev), T(ey, dev), T(lam, dev), 0, 0.5, want_cond=True)
    cond = N(cond)
    for p in range(P):
        Kx = A[p].astype(np.float64) @ A[p].astype(np.float64).T
        exact = np.linalg.norm(Kx, 1) * np.linalg.norm(np.linalg.inv(Kx), 1)
        assert exact / 10 <= cond[p] <= exact * 1.05, (p, cond[p], exact)


@pytest.mark.parametrize("k,d,ratio,lam", [(50, 128, 300.0, 1e-6), (64, 160, 1000.0, 1e-7), (150, 300, 300.0, 1e-6),
                                           (200, 400, 300.0, 1e-6)])
def test_refinement_reduces_error(F, dev, k, d, ratio, lam):
    P = 2
    A, B, ex, ey = _conditioned(22, P, k, d, ratio)
    lam = np.full(P, lam, np.float32)
    args = [T(A, dev), T(B, dev), T(ex, dev), T(ey, dev), T(lam, dev), 0, 0.5]
    C0 = N(F.fmap_solve(*args)[0])
    C1 = N(F.fmap_solve(*args, refine_steps=1)[0])
    C2 = N(F.fmap_solve(*args, refine_steps=2)[0])
    ref = _oracle_solve(A, B, ex, ey, lam, 0, 0.5)
    for p in range(P):
        e0, e1, e2 = (rel_fro(C[p], ref[p]["C"]) for C in (C0, C1, C2))
        assert e1 <= 1.1 * e0 and e2 <= 1.1 * e1 + 1e-7, (p, e0, e1, e2)
        assert e2 <= 1e-5, (p, e0, e1, e2)


# k = 40: register row solve, estimate first; k = 150: tiled row solve, the estimate beside it on a second
# stream and the flagged pairs solved again (pair 1 well conditioned, so only pairs 0 and 2 are redone)
@pytest.mark.parametrize("k,d", [(40, 96), (150, 320)])
def test_fp64_normal_matrix_branch(F, dev, k, d):
    """Pairs whose estimate exceeds the threshold factorise the rounded float64 product; the result stays
    within tolerance after refinement and the estimate reports the ill-conditioning."""
    P = 3
    A, B, ex, ey = _conditioned(23, P, k, d, 3000.0)   # cond(A A^T) ~ 9e6
    A1, B1, _, _ = _conditioned(24, 1, k, d, 3.0)
    A[1], B[1] = A1[0], B1[0]
    lam = np.full(P, 1e-4, np.float32)
    args = [T(A, dev), T(B, dev), T(ex, dev), T(ey, dev), T(lam, dev), 0, 0.5]
    C, _, info, cond = F.fmap_solve(*args, refine_steps=2, cond_fp64_threshold=1e6, want_cond=True)
    ref = _oracle_solve(A, B, ex, ey, lam, 0, 0.5)
    cond = N(cond)
    assert cond[0] > 1e6 and cond[2] > 1e6 and cond[1] < 1e3, cond
    assert (N(info) == 0).all()
    for p in range(P):
        assert rel_fro(N(C)[p], ref[p]["C"]) <= 1e-5, (p, rel_fro(N(C)[p], ref[p]["C"]))


BF16_PATH_TOL = 2e-3  # stated bar of the bf16-projection path (C and dF against the oracle on the same bf16 inputs)


@pytest.mark.parametrize("pairs,n", [(2, 6000), (4, 50000)])
def test_mixed_precision_pipeline(F, dev, pairs, n):
    """bf16 projections, float32 row solves with one float64-residual refinement step and the float64
    normal matrix above a condition estimate of 1e6, backward through the bf16 projection, at the mixed
    workload's k, d and spectra (n=50000 is its full size; n=6000 a reduced one).  Per pair, C and dF
    against the oracle fed the same bf16-rounded inputs (the path's own error), and against the oracle fed
    the unrounded float32 inputs (the path's error including the bf16 rounding of basis and features)."""
    import torch
    b = synth.workload_mixed(pairs=pairs, n=n)
    P = b.pairs
    phi = torch.from_numpy(b.phi_bf16.view(np.int16)).to(dev).view(torch.bfloat16)
    feat = torch.from_numpy(b.feat_bf16.view(np.int16)).to(dev).view(torch.bfloat16)
    mass = T(b.mass, dev)
    AB = F.fmap_project(phi, mass, feat)
    C, fac, info, cond = F.fmap_solve(AB[:P], AB[P:], T(b.evals_x, dev), T(b.evals_y, dev), T(b.lam, dev), b.mask,
                                      b.gamma, refine_steps=1, cond_fp64_threshold=1e6, want_cond=True)
    dAB = torch.empty_like(AB)
    F.fmap_solve_backward(T(b.dC, dev), AB[:P], AB[P:], C, T(b.evals_x, dev), T(b.evals_y, dev), T(b.lam, dev),
                          b.mask, b.gamma, fac, dA=dAB[:P], dB=dAB[P:])
    dF = N(F.fmap_project_backward(phi, mass, dAB))
    C, info = N(C), N(info)
    for p in sorted({0, P - 1}):
        for label, ph, fe in (("same bf16 inputs", b.phi_consumed(), b.feat_consumed()),
                              ("unrounded inputs", b.phi, b.feat)):
            A, B, D, Cr, ir = oracle.forward_pair(ph[p], b.mass[p], fe[p], ph[P + p], b.mass[P + p], fe[P + p],
                                                  b.evals_x[p], b.evals_y[p], float(b.lam[p]), b.mask, b.gamma)
            dA, dB, _ = oracle.solve_backward(A, B, Cr, D, float(b.lam[p]), b.dC[p])
            errs = (rel_fro(C[p], Cr), rel_fro(dF[p], oracle.project_backward(ph[p], b.mass[p], dA)),
                    rel_fro(dF[P + p], oracle.project_backward(ph[P + p], b.mass[P + p], dB)))
            print("mixed pair", p, label, "errors C, dF_x, dF_y:", errs, "cond", float(N(cond)[p]), flush=True)
            assert np.array_equal(info[p], ir)
            assert max(errs) <= BF16_PATH_TOL, (p, label, errs)
            if label == "same bf16 inputs":
                assert errs[0] <= 1e-4  # the refinement step leaves the projection's float32 sums as the error

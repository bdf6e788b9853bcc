"""Pins for the vectorized (k^2 x k^2) solve oracle, independent of its code.

Each pin reaches the oracle's normal equations by a different route: the row-wise oracle (diagonal operators
reduce the problem to Eqs. (4)-(7) with the Laplacian mask), the gradient of the objective written in matrix
form, library least squares on the stacked problem, the lambda = 0 closed form and the scalar case.  The
operators are non-symmetric in every pin that can tell D from D^T, so a transposed operator, a wrong sign of a
cross term, a dropped term or a wrong vectorization order fails at least one of them.
"""
import numpy as np
import pytest

import oracle
from oracle import vectorized as vz


def _inputs(seed, kx, ky, d, scale=0.3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((kx, d))
    B = rng.standard_normal((ky, d))
    D1 = np.diag(np.sort(rng.uniform(0, 2, kx))) + scale * rng.standard_normal((kx, kx))
    D2 = np.diag(np.sort(rng.uniform(0, 2, ky))) + scale * rng.standard_normal((ky, ky))
    return A, B, D1, D2


@pytest.mark.parametrize("kx,ky,d,lam", [(3, 3, 8, 0.7), (5, 4, 12, 0.05), (4, 6, 10, 2.0), (8, 8, 20, 1e-3)])
def test_diagonal_operators_reduce_to_row_wise_solve(kx, ky, d, lam):
    """Eigenvalue operators: the row systems of Eqs. (4)-(7) with D_ij = (mu_y(i) - mu_x(j))^2."""
    rng = np.random.default_rng(kx * 100 + ky)
    A, B = rng.standard_normal((kx, d)), rng.standard_normal((ky, d))
    mx, my = np.sort(rng.uniform(0, 3, kx)), np.sort(rng.uniform(0, 3, ky))
    C = vz.solve(A, B, np.diag(mx), np.diag(my), lam)
    D = oracle.mask(mx, my, 0)
    Crow, info = oracle.solve(A, B, D, lam)
    assert (info == 0).all()
    assert np.abs(C - Crow).max() <= 1e-10 * max(1.0, np.abs(Crow).max())


@pytest.mark.parametrize("kx,ky,d,lam", [(3, 3, 8, 0.7), (5, 4, 12, 0.05), (4, 6, 10, 2.0), (7, 5, 6, 0.3)])
def test_gradient_vanishes_at_solution(kx, ky, d, lam):
    """The objective's gradient, 2 (CA - B) A^T + 2 lambda (E D1^T - D2^T E) with E = C D1 - D2 C, is zero."""
    A, B, D1, D2 = _inputs(3, kx, ky, d)
    C = vz.solve(A, B, D1, D2, lam)
    G = vz.gradient(A, B, D1, D2, lam, C)
    scale = np.abs(B @ A.T).max()
    assert np.abs(G).max() <= 1e-10 * scale
    # and it is a minimum: any perturbation raises the objective
    f0 = vz.objective(A, B, D1, D2, lam, C)
    rng = np.random.default_rng(4)
    for _ in range(5):
        assert vz.objective(A, B, D1, D2, lam, C + 1e-3 * rng.standard_normal(C.shape)) > f0


@pytest.mark.parametrize("kx,ky,d,lam", [(3, 3, 8, 0.7), (5, 4, 3, 0.05), (6, 4, 10, 2.0)])
def test_normal_equations_match_library_least_squares(kx, ky, d, lam):
    """The stacked least-squares problem solved by the library (no normal equations), including d < kx."""
    A, B, D1, D2 = _inputs(5, kx, ky, d)
    C = vz.solve(A, B, D1, D2, lam)
    C2 = vz.solve_lstsq(A, B, D1, D2, lam)
    assert np.abs(C - C2).max() <= 1e-9 * max(1.0, np.abs(C2).max())


def test_lambda_zero_is_plain_least_squares():
    """Without the regulariser the map is B A^T (A A^T)^{-1}, whatever the operators."""
    A, B, D1, D2 = _inputs(6, 5, 4, 16)
    C = vz.solve(A, B, D1, D2, 0.0)
    Cls = B @ A.T @ np.linalg.inv(A @ A.T)
    assert np.abs(C - Cls).max() <= 1e-11 * np.abs(Cls).max()


def test_scalar_case_closed_form():
    """kx = ky = 1: c = (B . A) / (A . A + lambda (d1 - d2)^2)."""
    rng = np.random.default_rng(7)
    A, B = rng.standard_normal((1, 9)), rng.standard_normal((1, 9))
    d1, d2, lam = 1.7, -0.4, 0.9
    c = vz.solve(A, B, np.array([[d1]]), np.array([[d2]]), lam)[0, 0]
    assert c == pytest.approx(float(B @ A.T) / (float(A @ A.T) + lam * (d1 - d2) ** 2), rel=1e-13)


def test_system_matrix_entries_from_index_form():
    """H[(i,j),(p,q)] = delta_ip (AA^T)_jq + lambda (delta_ip (D1 D1^T)_jq - D2_ip D1_jq - D2_pi D1_qj
    + delta_jq (D2^T D2)_ip), written out from the objective's second derivatives, loop by loop."""
    kx, ky = 3, 4
    A, B, D1, D2 = _inputs(8, kx, ky, 7)
    lam = 0.6
    H, g = vz.system(A, B, D1, D2, lam)
    K = A @ A.T
    for i in range(ky):
        for j in range(kx):
            assert g[i * kx + j] == pytest.approx(float(B[i] @ A[j]), rel=1e-13, abs=1e-13)
            for p in range(ky):
                for q in range(kx):
                    dip, djq = float(i == p), float(j == q)
                    v = dip * K[j, q] + lam * (dip * float(D1[j] @ D1[q]) - D2[i, p] * D1[j, q] - D2[p, i] * D1[q, j]
                                               + djq * float(D2[:, i] @ D2[:, p]))
                    assert H[i * kx + j, p * kx + q] == pytest.approx(v, rel=1e-12, abs=1e-12)

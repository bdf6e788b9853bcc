"""Double-precision CPU oracle for the vectorized functional-map solve with general (non-diagonal)
commutativity operators: the k^2 x k^2 formulation that Sec. 3.1 contrasts with the row-wise solve, and that
the paper's conclusion names for non-orthogonal bases.

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline leg may import this module; the
GPU library and its Python binding never do.  It shares no code with the GPU path.

Problem (Eq. (2) with the Frobenius norm, the operators kept as general matrices):
    C = argmin ||C A - B||_F^2 + lambda ||C D1 - D2 C||_F^2,
with A [kx][d], B [ky][d], D1 [kx][kx] (source operator), D2 [ky][ky] (target operator), C [ky][kx].  In an
orthonormal eigenbasis D1 and D2 are the diagonal eigenvalue matrices and the problem splits into the row
systems of Eqs. (4)-(7) with the Laplacian mask (mu_y(i) - mu_x(j))^2; in a non-orthogonal basis they are
full, and every entry of C couples to every other one.

Vectorization: c = vec_r(C), c[i kx + j] = C[i][j] (row-major).  With that ordering
    vec_r(C M) = (I_ky kron M^T) c,     vec_r(M C) = (M kron I_kx) c,
so the objective is ||(I kron A^T) c - vec_r(B)||^2 + lambda ||(I kron D1^T - D2 kron I) c||^2 and the
normal equations are H c = g with
    H = I kron (A A^T) + lambda (I kron D1^T - D2 kron I)^T (I kron D1^T - D2 kron I),
    g = vec_r(B A^T).
H is symmetric positive definite when A A^T is.

Functions:
  system       H and g, built from Kronecker products exactly as written above
  solve        C from H c = g (numpy's LU solve in float64)
  solve_lstsq  C from the stacked least-squares problem (library least squares, no normal equations),
               used as an independent pin of `system` / `solve`

Pins (tests/test_oracle_pins_vectorized.py): diagonal operators reproduce the row-wise oracle with the
Laplacian mask; `solve` equals `solve_lstsq`; the gradient of the objective, written in matrix form, vanishes
at the solution and the objective rises under perturbation; lambda = 0 gives the plain least-squares map
B A^T (A A^T)^{-1}; the scalar case kx = ky = 1 has a closed form; every entry of H matches the index form
of the objective's second derivatives.
"""
from __future__ import annotations

import numpy as np


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _operator(D1, D2):
    """The matrix of C -> vec_r(C D1 - D2 C) acting on c = vec_r(C)."""
    kx, ky = D1.shape[0], D2.shape[0]
    return np.kron(np.eye(ky), D1.T) - np.kron(D2, np.eye(kx))


def system(A, B, D1, D2, lam: float):
    """(H [n][n], g [n]) of the normal equations, n = ky kx, c[i kx + j] = C[i][j]."""
    A, B, D1, D2 = _f64(A), _f64(B), _f64(D1), _f64(D2)
    kx, ky = A.shape[0], B.shape[0]
    assert D1.shape == (kx, kx) and D2.shape == (ky, ky) and B.shape[1] == A.shape[1]
    T = _operator(D1, D2)
    H = np.kron(np.eye(ky), A @ A.T) + float(lam) * (T.T @ T)
    g = (B @ A.T).reshape(-1)
    return H, g


def solve(A, B, D1, D2, lam: float) -> np.ndarray:
    """C [ky][kx] from the normal equations H c = g."""
    H, g = system(A, B, D1, D2, lam)
    kx, ky = np.shape(A)[0], np.shape(B)[0]
    return np.linalg.solve(H, g).reshape(ky, kx)


def solve_lstsq(A, B, D1, D2, lam: float) -> np.ndarray:
    """C [ky][kx] from the stacked least-squares problem [I kron A^T; sqrt(lambda) T] c ~ [vec_r(B); 0]."""
    A, B, D1, D2 = _f64(A), _f64(B), _f64(D1), _f64(D2)
    kx, ky, d = A.shape[0], B.shape[0], A.shape[1]
    top = np.kron(np.eye(ky), A.T)          # rows (i, e): sum_j C[i][j] A[j][e]
    rhs_top = B.reshape(-1)                 # (i, e) -> B[i][e]
    M = np.vstack([top, np.sqrt(float(lam)) * _operator(D1, D2)])
    rhs = np.concatenate([rhs_top, np.zeros(ky * kx)])
    c, *_ = np.linalg.lstsq(M, rhs, rcond=None)
    return c.reshape(ky, kx)


def objective(A, B, D1, D2, lam: float, C) -> float:
    A, B, D1, D2, C = _f64(A), _f64(B), _f64(D1), _f64(D2), _f64(C)
    return float(np.sum((C @ A - B) ** 2) + float(lam) * np.sum((C @ D1 - D2 @ C) ** 2))


def gradient(A, B, D1, D2, lam: float, C) -> np.ndarray:
    """Gradient of `objective` with respect to C, written in matrix form (not from H)."""
    A, B, D1, D2, C = _f64(A), _f64(B), _f64(D1), _f64(D2), _f64(C)
    E = C @ D1 - D2 @ C
    return 2.0 * (C @ A - B) @ A.T + 2.0 * float(lam) * (E @ D1.T - D2.T @ E)

"""Double-precision CPU oracle for the regularised functional-map solve.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library and its Python
binding never do.  It shares no code with the GPU path.

The arithmetic lives in ``fmap_oracle.c`` (plain C, OpenMP, no BLAS/LAPACK);
this module builds it with gcc and wraps it with ctypes.  Inputs of any float
dtype are promoted to float64 before the call.

Functions and the passages they follow (Sec. 3.1 of the paper):
  project            Eq. (1), pseudo-inverse read in the mass inner product
  project_backward   adjoint of Eq. (1)
  mask               Eq. (3) / the mask defined after Eq. (4); resolvent mask
  solve              Eqs. (4)-(7), row-decoupled normal equations, Cholesky
  solve_backward     reverse mode of `solve` (derived)
  pipeline_batch     the whole forward + backward pass over a batch of pairs
  project_pinv       Eq. (1) with the projector given directly: A = P^T F for
                     P = (Phi^+)^T, and its adjoint dF = P dA
  solve_resolutions  maps at several spectral resolutions from one projection:
                     resolution (k_x', k_y') is the solve restricted to the
                     first k_x' source and k_y' target eigenpairs

Pins: every function is checked in ``tests/test_oracle_pins.py`` against closed
forms, invariants, a Kronecker brute force, library least squares, hand-worked
fixtures in ``tests/golden`` and central finite differences.

Two further oracles, in plain numpy float64, live in submodules:
  oracle.overlap     confusion counts and overlap metrics, balanced accuracy
                     (Sec. 3.3); pins in tests/test_oracle_pins_overlap.py
  oracle.gradfeat    DiffusionNet spatial-gradient features, variants A and B,
                     and their reverse mode (Sec. 3.2); pins in
                     tests/test_oracle_pins_gradfeat.py
  oracle.vectorized  the vectorized k^2 x k^2 solve with general (non-diagonal)
                     commutativity operators (Sec. 3.1, the formulation the
                     conclusion names for non-orthogonal bases); pins in
                     tests/test_oracle_pins_vectorized.py
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmap_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MASK_LAPLACIAN = 0
MASK_RESOLVENT = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile fmap_oracle.c into liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, dp, ip = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_project.argtypes = [i64, i64, i64, dp, dp, dp, dp]
        lib.oracle_project_backward.argtypes = [i64, i64, i64, dp, dp, dp, dp]
        lib.oracle_mask.argtypes = [i64, i64, dp, dp, ctypes.c_int, ctypes.c_double, dp]
        lib.oracle_mask.restype = ctypes.c_int
        lib.oracle_solve.argtypes = [i64, i64, i64, dp, dp, dp, ctypes.c_double, dp, ip, dp]
        lib.oracle_solve_backward.argtypes = [i64, i64, i64, dp, dp, dp, dp, ctypes.c_double, dp, dp, dp, dp, ip]
        lib.oracle_pipeline_batch.argtypes = [i64, i64, i64, i64, dp, dp, dp, dp, dp, ctypes.c_int,
                                              ctypes.c_double, dp, dp, dp]
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def project(phi, mass, feat) -> np.ndarray:
    """A = Phi^T diag(M) F for one shape: phi [n,k], mass [n], feat [n,d] -> [k,d]."""
    phi, mass, feat = _f64(phi), _f64(mass), _f64(feat)
    n, k = phi.shape
    d = feat.shape[1]
    assert mass.shape == (n,) and feat.shape[0] == n
    A = np.empty((k, d))
    _load().oracle_project(n, k, d, _p(phi), _p(mass), _p(feat), _p(A))
    return A


def project_backward(phi, mass, dA) -> np.ndarray:
    """dF = diag(M) Phi dA for one shape: dA [k,d] -> [n,d]."""
    phi, mass, dA = _f64(phi), _f64(mass), _f64(dA)
    n, k = phi.shape
    d = dA.shape[1]
    assert dA.shape[0] == k and mass.shape == (n,)
    dF = np.empty((n, d))
    _load().oracle_project_backward(n, k, d, _p(phi), _p(mass), _p(dA), _p(dF))
    return dF


def mask(evals_x, evals_y, kind: int, gamma: float = 0.5) -> np.ndarray:
    """Penalty mask D [ky,kx]; raises ValueError when the resolvent normaliser is not positive."""
    ex, ey = _f64(evals_x), _f64(evals_y)
    D = np.empty((ey.shape[0], ex.shape[0]))
    rc = _load().oracle_mask(ex.shape[0], ey.shape[0], _p(ex), _p(ey), int(kind), float(gamma), _p(D))
    if rc != 0:
        raise ValueError("resolvent normaliser max(mu) is not positive")
    return D


def solve(A, B, D, lam: float, return_factors: bool = False):
    """C [ky,kx] and info [ky] (and the ky Cholesky factors if asked)."""
    A, B, D = _f64(A), _f64(B), _f64(D)
    kx, d = A.shape
    ky = B.shape[0]
    assert B.shape[1] == d and D.shape == (ky, kx)
    C = np.empty((ky, kx))
    info = np.empty(ky, np.int32)
    L = np.empty((ky, kx, kx)) if return_factors else None
    _load().oracle_solve(kx, ky, d, _p(A), _p(B), _p(D), float(lam), _p(C),
                         info.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         _p(L) if L is not None else None)
    return (C, info, L) if return_factors else (C, info)


def solve_backward(A, B, C, D, lam: float, dC):
    """(dA [kx,d], dB [ky,d], dlambda) for upstream gradient dC [ky,kx]."""
    A, B, C, D, dC = _f64(A), _f64(B), _f64(C), _f64(D), _f64(dC)
    kx, d = A.shape
    ky = B.shape[0]
    dA = np.empty((kx, d))
    dB = np.empty((ky, d))
    dl = ctypes.c_double(0.0)
    _load().oracle_solve_backward(kx, ky, d, _p(A), _p(B), _p(C), _p(D), float(lam), _p(dC), _p(dA), _p(dB),
                                  ctypes.byref(dl), None)
    return dA, dB, dl.value


def pipeline_batch(phi, mass, feat, evals, lam, mask_kind: int, gamma: float, dC):
    """Forward + backward over P equal pairs: returns C [P,k,k], dF [2P,n,d]."""
    phi, mass, feat, evals, lam, dC = map(_f64, (phi, mass, feat, evals, lam, dC))
    P2, n, k = phi.shape
    P = P2 // 2
    d = feat.shape[2]
    C = np.empty((P, k, k))
    dF = np.empty((P2, n, d))
    _load().oracle_pipeline_batch(P, n, k, d, _p(phi), _p(mass), _p(feat), _p(evals), _p(lam), int(mask_kind),
                                  float(gamma), _p(dC), _p(C), _p(dF))
    return C, dF


def forward_pair(phi_x, mass_x, feat_x, phi_y, mass_y, feat_y, ex, ey, lam, mask_kind, gamma):
    """Forward pass of one pair: A, B, D, C, info."""
    A = project(phi_x, mass_x, feat_x)
    B = project(phi_y, mass_y, feat_y)
    D = mask(ex, ey, mask_kind, gamma)
    C, info = solve(A, B, D, lam)
    return A, B, D, C, info


def solve_resolutions(A, B, evals_x, evals_y, lam: float, mask_kind: int, gamma: float, kxs, kys):
    """Maps at several spectral resolutions from one pair of spectral descriptors: for each r, the solve of
    Eqs. (4)-(7) on the first kxs[r] rows of A, the first kys[r] rows of B and the eigenvalues truncated
    alike (the mask, and the resolvent's normaliser, are those of the truncated spectra).  Returns a list
    of (C_r [kys[r], kxs[r]], info_r)."""
    out = []
    for kx, ky in zip(kxs, kys):
        D = mask(np.asarray(evals_x)[:kx], np.asarray(evals_y)[:ky], mask_kind, gamma)
        out.append(solve(np.asarray(A)[:kx], np.asarray(B)[:ky], D, lam))
    return out


def project_pinv(pinv_t, feat) -> np.ndarray:
    """A = P^T F for one shape with the projector given directly, P = (Phi^+)^T [n,k], feat [n,d] -> [k,d]."""
    P, F = _f64(pinv_t), _f64(feat)
    assert P.shape[0] == F.shape[0]
    return P.T @ F


def project_pinv_backward(pinv_t, dA) -> np.ndarray:
    """dF = P dA for one shape: P [n,k], dA [k,d] -> [n,d]."""
    return _f64(pinv_t) @ _f64(dA)

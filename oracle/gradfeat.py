"""Double-precision CPU oracle for DiffusionNet's spatial-gradient features (Sec. 3.2).

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline leg
may import this module; the GPU library and its Python binding never do.  It
shares no code with the GPU path.

At one vertex the D channels carry complex gradients z = x + i y (x, y in R^D:
the two components of D tangent vectors).  With a learned complex matrix
A = A_re + i A_im (D x D, (A z)_c = sum_j A_cj z_j) the features are

    g = x * (A z)_re + y * (A z)_im          (elementwise; the paper's Eq. for g)

and the two implementations the paper documents differ in (A z)_im only:

    (A z)_re = A_re x - A_im y               (both variants)
    (A z)_im = A_re y + A_im x               variant "A" (the complex product)
    (A z)_im = A_re x + A_im y               variant "B"

so that g_i = sum_j v_i^T [[a, -b], [b, a]] v_j (variant A) or
sum_j v_i^T [[a, -b], [a, b]] v_j (variant B), with a = A_re[i, j],
b = A_im[i, j] and v_j = (x_j, y_j).

Functions:
  gradient_features           g [V, D] from z [V, D, 2] (last axis: x, y)
  gradient_features_backward  reverse mode: dz [V, D, 2], dA_re, dA_im [D, D]
                              for an upstream gradient dg [V, D] (derived here by
                              the chain rule; the paper states no gradients)
"""
from __future__ import annotations

import numpy as np

VARIANTS = ("A", "B")


def _parts(z):
    z = np.asarray(z, dtype=np.float64)
    assert z.shape[-1] == 2, z.shape
    return z[..., 0], z[..., 1]


def transformed(z, A_re, A_im, variant: str):
    """((A z)_re, (A z)_im) per vertex, [V, D] each."""
    assert variant in VARIANTS
    x, y = _parts(z)
    Ar = np.asarray(A_re, dtype=np.float64)
    Ai = np.asarray(A_im, dtype=np.float64)
    re = x @ Ar.T - y @ Ai.T
    im = (y @ Ar.T + x @ Ai.T) if variant == "A" else (x @ Ar.T + y @ Ai.T)
    return re, im


def gradient_features(z, A_re, A_im, variant: str) -> np.ndarray:
    """g [V, D] for z [V, D, 2], A_re, A_im [D, D]."""
    x, y = _parts(z)
    re, im = transformed(z, A_re, A_im, variant)
    return x * re + y * im


def gradient_features_backward(z, A_re, A_im, variant: str, dg):
    """(dz [V, D, 2], dA_re [D, D], dA_im [D, D]) for the upstream gradient dg [V, D].

    With u = dg * x (the gradient reaching (A z)_re) and w = dg * y (reaching (A z)_im):
      variant A:  dx = dg * re + u A_re + w A_im,   dy = dg * im - u A_im + w A_re,
                  dA_re = u^T x + w^T y,            dA_im = -u^T y + w^T x;
      variant B:  dx = dg * re + u A_re + w A_re,   dy = dg * im - u A_im + w A_im,
                  dA_re = u^T x + w^T x,            dA_im = -u^T y + w^T y.
    """
    x, y = _parts(z)
    Ar = np.asarray(A_re, dtype=np.float64)
    Ai = np.asarray(A_im, dtype=np.float64)
    dg = np.asarray(dg, dtype=np.float64)
    re, im = transformed(z, Ar, Ai, variant)
    u = dg * x
    w = dg * y
    if variant == "A":
        dx = dg * re + u @ Ar + w @ Ai
        dy = dg * im - u @ Ai + w @ Ar
        dAr = u.T @ x + w.T @ y
        dAi = -u.T @ y + w.T @ x
    else:
        dx = dg * re + u @ Ar + w @ Ar
        dy = dg * im - u @ Ai + w @ Ai
        dAr = u.T @ x + w.T @ x
        dAi = -u.T @ y + w.T @ y
    return np.stack([dx, dy], axis=-1), dAr, dAi

"""Pins for the spatial-gradient feature oracle (Sec. 3.2), independent of its code.

Variant A is the complex expression the paper starts from, Re(conj(z) * (A z))
(checked with numpy complex arithmetic), and it is invariant under a rotation
of each vertex's tangent plane; both variants equal the paper's per-channel
2x2 block sums (checked by explicit loops), and special weights give closed
forms.  The derived backward is pinned by central finite differences.
"""
import numpy as np
import pytest

from oracle import gradfeat as gf


def _inputs(seed, V, D):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((V, D, 2))
    Ar = rng.standard_normal((D, D)) / np.sqrt(D)
    Ai = rng.standard_normal((D, D)) / np.sqrt(D)
    return z, Ar, Ai


def test_variant_a_is_the_complex_form():
    z, Ar, Ai = _inputs(1, 17, 9)
    zc = z[..., 0] + 1j * z[..., 1]
    Ac = Ar + 1j * Ai
    ref = np.real(np.conj(zc) * (zc @ Ac.T))
    np.testing.assert_allclose(gf.gradient_features(z, Ar, Ai, "A"), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("variant,block", [("A", lambda a, b: np.array([[a, -b], [b, a]])),
                                           ("B", lambda a, b: np.array([[a, -b], [a, b]]))])
def test_block_sums(variant, block):
    """g_i = sum_j v_i^T M(a_ij, b_ij) v_j with the variant's 2x2 block (explicit loops)."""
    z, Ar, Ai = _inputs(2, 3, 5)
    V, D, _ = z.shape
    ref = np.zeros((V, D))
    for v in range(V):
        for i in range(D):
            for j in range(D):
                ref[v, i] += z[v, i] @ block(Ar[i, j], Ai[i, j]) @ z[v, j]
    np.testing.assert_allclose(gf.gradient_features(z, Ar, Ai, variant), ref, rtol=0, atol=1e-12)


def test_rotation_of_the_tangent_plane():
    """Rotating every tangent vector of a vertex by that vertex's angle leaves variant A unchanged (a
    rotation is multiplication by a unit complex number); variant B is not invariant."""
    z, Ar, Ai = _inputs(3, 11, 6)
    th = np.random.default_rng(4).uniform(0, 2 * np.pi, (11, 1))
    c, s = np.cos(th), np.sin(th)
    zr = np.stack([c * z[..., 0] - s * z[..., 1], s * z[..., 0] + c * z[..., 1]], axis=-1)
    np.testing.assert_allclose(gf.gradient_features(zr, Ar, Ai, "A"), gf.gradient_features(z, Ar, Ai, "A"),
                               rtol=0, atol=1e-12)
    assert np.abs(gf.gradient_features(zr, Ar, Ai, "B") - gf.gradient_features(z, Ar, Ai, "B")).max() > 1e-3


def test_identity_weights():
    """A_re = I, A_im = 0: variant A gives |v_i|^2 = x^2 + y^2, variant B gives x^2 + x y."""
    z, _, _ = _inputs(5, 7, 4)
    I, Z = np.eye(4), np.zeros((4, 4))
    x, y = z[..., 0], z[..., 1]
    np.testing.assert_allclose(gf.gradient_features(z, I, Z, "A"), x * x + y * y, atol=1e-14)
    np.testing.assert_allclose(gf.gradient_features(z, I, Z, "B"), x * x + x * y, atol=1e-14)
    # A_re = 0, A_im = I: variant A gives x (-y) + y x = 0, variant B gives -x y + y y
    np.testing.assert_allclose(gf.gradient_features(z, Z, I, "A"), 0.0, atol=1e-14)
    np.testing.assert_allclose(gf.gradient_features(z, Z, I, "B"), -x * y + y * y, atol=1e-14)


@pytest.mark.parametrize("variant", gf.VARIANTS)
def test_backward_finite_differences(variant):
    """<dg, g(z + h u) - g(z - h u)> / 2h against the analytic directional derivative (z, A_re, A_im)."""
    z, Ar, Ai = _inputs(6, 9, 5)
    rng = np.random.default_rng(7)
    dg = rng.standard_normal((9, 5))
    dz, dAr, dAi = gf.gradient_features_backward(z, Ar, Ai, variant, dg)
    uz, ur, ui = rng.standard_normal(z.shape), rng.standard_normal(Ar.shape), rng.standard_normal(Ai.shape)
    h = 1e-6
    L = lambda t: float(np.sum(dg * gf.gradient_features(z + t * uz, Ar + t * ur, Ai + t * ui, variant)))
    fd = (L(h) - L(-h)) / (2 * h)
    an = float(np.sum(dz * uz) + np.sum(dAr * ur) + np.sum(dAi * ui))
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)
    # each argument alone (a wrong term in one of them cannot cancel against another)
    for k, (u, g) in enumerate(((uz, dz), (ur, dAr), (ui, dAi))):
        args = [z, Ar, Ai]
        Lk = lambda t: float(np.sum(dg * gf.gradient_features(*[a + t * u if i == k else a
                                                                  for i, a in enumerate(args)], variant)))
        assert abs((Lk(h) - Lk(-h)) / (2 * h) - float(np.sum(g * u))) <= 1e-7 * max(1.0, abs(float(np.sum(g * u))))

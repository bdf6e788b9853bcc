"""Seeded synthetic inputs for the functional-map solve.

Shared by the tests, the benchmark and the smoke check.  This module only
*draws* inputs (bases, masses, eigenvalues, features, upstream gradients);
it computes nothing the solver computes: no projection onto a basis, no mask,
no normal equations, no solve.  Correlated features are made by *synthesis*
(basis times coefficients), never by projecting.

Every array is built in float64 and rounded once, to float32 (and for the
mixed-precision workload additionally to bfloat16, round-to-nearest-even),
and both the GPU path and the oracle consume the rounded values.

Streams are numpy PCG64 keyed by SeedSequence(260410377, spawn_key=(tag,...)),
so a (workload, pair, shape) triple always gets the same draw regardless of
the order in which items are generated.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

ROOT_SEED = 260410377

# Mask kinds (values match the C ABI).
MASK_LAPLACIAN = 0
MASK_RESOLVENT = 1


def rng_for(*key: int) -> np.random.Generator:
    """Independent PCG64 stream for an integer key tuple."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=tuple(int(x) for x in key))))


# ----------------------------------------------------------------------------
# Per-shape spectral data
# ----------------------------------------------------------------------------

def lumped_mass(rng: np.random.Generator, n: int) -> np.ndarray:
    """Per-vertex lumped mass, M_ii ~ U[0.5, 1.5] / n (float64)."""
    return rng.uniform(0.5, 1.5, size=n) / n


def mass_orthonormal_basis(rng: np.random.Generator, mass: np.ndarray, k: int) -> np.ndarray:
    """An n x k basis with Phi^T diag(mass) Phi = I (float64).

    Gaussian n x k matrix, QR of diag(sqrt(mass)) X with the signs fixed so
    that diag(R) > 0, then Phi = diag(1/sqrt(mass)) Q.
    """
    n = mass.shape[0]
    x = rng.standard_normal((n, k))
    sq = np.sqrt(mass)
    q, r = np.linalg.qr(sq[:, None] * x, mode="reduced")
    sgn = np.sign(np.diag(r))
    sgn[sgn == 0] = 1.0
    q = q * sgn[None, :]
    return q / sq[:, None]


def eigenvalues_linear(rng: np.random.Generator, k: int) -> np.ndarray:
    """mu_0 = 0, mu_j = 0.05 j (1 + 0.1 N(0,1)), clamped >= 1e-6, sorted increasing."""
    j = np.arange(1, k, dtype=np.float64)
    mu = 0.05 * j * (1.0 + 0.1 * rng.standard_normal(k - 1))
    mu = np.maximum(mu, 1e-6)
    return np.sort(np.concatenate([[0.0], mu]))


def eigenvalues_log(rng: np.random.Generator, k: int, decades: float = 3.0) -> np.ndarray:
    """mu_0 = 0, mu_j = 0.05 * 10^(decades (j-1)/(k-2)) (1 + 0.1 N(0,1)), sorted.

    Spread mu_max / mu_1 of about 10^decades, to stress the conditioning of the
    row systems.
    """
    j = np.arange(1, k, dtype=np.float64)
    expo = decades * (j - 1.0) / max(k - 2, 1)
    mu = 0.05 * np.power(10.0, expo) * (1.0 + 0.1 * rng.standard_normal(k - 1))
    mu = np.maximum(mu, 1e-6)
    return np.sort(np.concatenate([[0.0], mu]))


def random_orthogonal(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-like d x d orthogonal matrix (QR of a Gaussian, signs fixed)."""
    q, r = np.linalg.qr(rng.standard_normal((d, d)))
    sgn = np.sign(np.diag(r))
    sgn[sgn == 0] = 1.0
    return q * sgn[None, :]


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16), round-to-nearest-even, NaN kept quiet."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint32)
    nan = np.isnan(x)
    r = np.where(nan, ((u >> 16) | 0x40).astype(np.uint32), r)
    return r.astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns (uint16) -> float32 values (exact)."""
    return (np.ascontiguousarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


# ----------------------------------------------------------------------------
# Batches of shape pairs
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class PairBatch:
    """A batch of shape pairs with equal n, k, d (float32 arrays, row-major).

    phi:   [2P, n, k]   x shapes first (0..P-1), then y shapes (P..2P-1)
    mass:  [2P, n]
    feat:  [2P, n, d]
    evals: [2P, k]
    lam:   [P]
    dC:    [P, k, k]    upstream gradient dL/dC (None for forward-only workloads)
    phi_bf16 / feat_bf16: bfloat16 bit patterns when the projection consumes bf16
    """

    name: str
    pairs: int
    n: int
    k: int
    d: int
    mask: int
    gamma: float
    phi: np.ndarray
    mass: np.ndarray
    feat: np.ndarray
    evals: np.ndarray
    lam: np.ndarray
    dC: Optional[np.ndarray] = None
    phi_bf16: Optional[np.ndarray] = None
    feat_bf16: Optional[np.ndarray] = None

    @property
    def evals_x(self) -> np.ndarray:
        return self.evals[: self.pairs]

    @property
    def evals_y(self) -> np.ndarray:
        return self.evals[self.pairs:]

    def phi_consumed(self) -> np.ndarray:
        """The basis values the projection actually reads (bf16-rounded if bf16)."""
        return self.phi if self.phi_bf16 is None else bf16_bits_to_f32(self.phi_bf16)

    def feat_consumed(self) -> np.ndarray:
        return self.feat if self.feat_bf16 is None else bf16_bits_to_f32(self.feat_bf16)


def _shape(tag: int, pair: int, side: int, n: int, k: int, eig: str):
    rng = rng_for(tag, pair, side, 0)
    mass = lumped_mass(rng, n)
    phi = mass_orthonormal_basis(rng, mass, k)
    mu = eigenvalues_linear(rng, k) if eig == "linear" else eigenvalues_log(rng, k)
    return mass, phi, mu


def make_batch(name: str, tag: int, pairs: int, n: int, k: int, d: int, *, mask: int, gamma: float = 0.5,
               lam: float | np.ndarray = 1e-3, features: str = "correlated", eig: str = "linear",
               noise: float = 0.05, with_grad: bool = True, bf16: bool = False) -> PairBatch:
    """Generate a batch of P shape pairs.

    features="independent": F_x, F_y ~ N(0,1) i.i.d.
    features="correlated":  coefficients X ~ N(0, 1/k) per pair (k x d), a d x d
        orthogonal R shared by the batch; F_x = Phi_x X + noise E_x,
        F_y = Phi_y (X R) + noise E_y with E ~ N(0,1).  The synthesised part has
        unit-variance entries, so features look N(0,1) per vertex while the
        spectral descriptors of the two shapes are related by R up to noise.
    """
    P = pairs
    phi = np.empty((2 * P, n, k), np.float32)
    mass = np.empty((2 * P, n), np.float32)
    feat = np.empty((2 * P, n, d), np.float32)
    evals = np.empty((2 * P, k), np.float32)
    rot = random_orthogonal(rng_for(tag, 10_000, 0, 1), d) if features == "correlated" else None
    for p in range(P):
        mx, px, ex = _shape(tag, p, 0, n, k, eig)
        my, py, ey = _shape(tag, p, 1, n, k, eig)
        rf = rng_for(tag, p, 2, 2)
        if features == "independent":
            fx = rf.standard_normal((n, d))
            fy = rf.standard_normal((n, d))
        else:
            coef = rf.standard_normal((k, d)) / np.sqrt(k)
            fx = px @ coef + noise * rf.standard_normal((n, d))
            fy = py @ (coef @ rot) + noise * rf.standard_normal((n, d))
        phi[p], phi[P + p] = px, py
        mass[p], mass[P + p] = mx, my
        feat[p], feat[P + p] = fx, fy
        evals[p], evals[P + p] = ex, ey
    lam_arr = np.broadcast_to(np.asarray(lam, np.float64), (P,)).astype(np.float32).copy()
    dC = rng_for(tag, 20_000, 0, 3).standard_normal((P, k, k)).astype(np.float32) if with_grad else None
    out = PairBatch(name, P, n, k, d, mask, float(gamma), phi, mass, feat, evals, lam_arr, dC)
    if bf16:
        out.phi_bf16 = to_bf16_bits(phi)
        out.feat_bf16 = to_bf16_bits(feat)
    return out


# ----------------------------------------------------------------------------
# The five benchmark workloads (sizes of the paper's settings; see DESIGN)
# ----------------------------------------------------------------------------

def workload_plain(scale: float = 1.0) -> PairBatch:
    """1 pair, n=5000, k=30, d=128, independent N(0,1) features, Laplacian mask, lambda=1e-3."""
    return make_batch("plain-fwd-k30", 1, 1, int(5000 * scale), 30, 128, mask=MASK_LAPLACIAN,
                      features="independent", with_grad=False)


def workload_headline(pairs: int = 32, n: int = 5000) -> PairBatch:
    """32 pairs, n=5000, k=50, d=256, correlated features, resolvent mask gamma=0.5, lambda=1e-3."""
    return make_batch("batched-k50-d256", 2, pairs, n, 50, 256, mask=MASK_RESOLVENT, gamma=0.5)


def workload_mixed(pairs: int = 16, n: int = 50000) -> PairBatch:
    """16 pairs, n=50000, k=200, d=384, log-spread eigenvalues, Laplacian mask, bf16 projection inputs."""
    return make_batch("mixed-k200-d384", 4, pairs, n, 200, 384, mask=MASK_LAPLACIAN, eig="log", bf16=True)


def workload_large(pairs: int = 8, n: int = 100000) -> PairBatch:
    """8 pairs, n=100000, k=300, d=512, resolvent mask gamma=0.5, lambda=1e-3."""
    return make_batch("large-k300-d512", 5, pairs, n, 300, 512, mask=MASK_RESOLVENT, gamma=0.5)


@dataclasses.dataclass
class RaggedPair:
    n_x: int
    n_y: int
    k: int
    lam: float
    phi_x: np.ndarray
    phi_y: np.ndarray
    mass_x: np.ndarray
    mass_y: np.ndarray
    feat_x: np.ndarray
    feat_y: np.ndarray
    evals_x: np.ndarray
    evals_y: np.ndarray
    dC: np.ndarray


def workload_ragged(pairs: int = 64, d: int = 256, n_lo: int = 2000, n_hi: int = 20000,
                    ks=(30, 50, 80, 120)) -> list:
    """Uneven batch: n ~ U{n_lo..n_hi} per shape, k from `ks` per pair, lambda = 10^U[-4,-2].

    Features are correlated as in make_batch (one shared d x d rotation), Laplacian mask.
    """
    tag = 3
    rot = random_orthogonal(rng_for(tag, 10_000, 0, 1), d)
    out = []
    for p in range(pairs):
        rp = rng_for(tag, p, 9, 9)
        nx = int(rp.integers(n_lo, n_hi + 1))
        ny = int(rp.integers(n_lo, n_hi + 1))
        k = int(rp.choice(np.asarray(ks)))
        lam = float(10.0 ** rp.uniform(-4.0, -2.0))
        mx, px, ex = _shape(tag, p, 0, nx, k, "linear")
        my, py, ey = _shape(tag, p, 1, ny, k, "linear")
        rf = rng_for(tag, p, 2, 2)
        coef = rf.standard_normal((k, d)) / np.sqrt(k)
        fx = px @ coef + 0.05 * rf.standard_normal((nx, d))
        fy = py @ (coef @ rot) + 0.05 * rf.standard_normal((ny, d))
        dC = rf.standard_normal((k, k))
        f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
        out.append(RaggedPair(nx, ny, k, np.float32(lam).item(), f32(px), f32(py), f32(mx), f32(my),
                              f32(fx), f32(fy), f32(ex), f32(ey), f32(dC)))
    return out


def small_problem(seed: int, k: int, d: int, *, kx: Optional[int] = None, lam: float = 1e-2,
                  mask: int = MASK_LAPLACIAN):
    """Spectral-domain test problem (A, B, evals) drawn directly, float64.

    A [kx, d], B [k, d], evals_x [kx], evals_y [k].  For solver tests that do
    not need a projection.
    """
    kx = k if kx is None else kx
    rng = rng_for(777, seed, k, d)
    A = rng.standard_normal((kx, d))
    B = rng.standard_normal((k, d))
    ex = eigenvalues_linear(rng, kx)
    ey = eigenvalues_linear(rng, k)
    return A, B, ex, ey, lam, mask


@dataclasses.dataclass
class OverlapBatch:
    """Scores and ground-truth overlap labels of S shapes, concatenated (shape s owns
    [offsets[s], offsets[s+1]))."""
    scores: np.ndarray   # [total] float32
    truth: np.ndarray    # [total] uint8
    offsets: np.ndarray  # [S + 1] int64
    ratios: np.ndarray   # [S] overlap ratio r the labels were drawn with


def workload_overlap(shapes: int = 1024, n_lo: int = 2000, n_hi: int = 20000, tag: int = 6) -> OverlapBatch:
    """Overlap predictions of a partial-matching evaluation batch.

    Per shape: n ~ U{n_lo..n_hi} vertices, overlap ratio r ~ U[0, 1], exactly round(r n) vertices
    labelled overlapping (in a random order), and a noisy predictor's score
    sigmoid(a (2 t - 1) + N(0, 1)) with a per-shape skill a ~ U[0, 3] (a = 0: a coin flip).
    """
    ns, ts, ss, rs = [], [], [], []
    for s in range(shapes):
        rng = rng_for(tag, s, 0, 0)
        n = int(rng.integers(n_lo, n_hi + 1))
        r = float(rng.uniform(0.0, 1.0))
        t = np.zeros(n, np.uint8)
        t[: int(round(r * n))] = 1
        rng.shuffle(t)
        a = rng.uniform(0.0, 3.0)
        score = 1.0 / (1.0 + np.exp(-(a * (2.0 * t - 1.0) + rng.standard_normal(n))))
        ns.append(n)
        ts.append(t)
        ss.append(score.astype(np.float32))
        rs.append(r)
    off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    return OverlapBatch(np.concatenate(ss) if ss else np.zeros(0, np.float32),
                        np.concatenate(ts) if ts else np.zeros(0, np.uint8), off, np.asarray(rs))


def workload_gradfeat(vertices: int = 160_000, channels: int = 128, tag: int = 7):
    """Inputs of DiffusionNet's spatial-gradient features: per-vertex complex gradients z [V, D, 2] ~ N(0, 1)
    (x, y interleaved per channel) and weights A_re, A_im [D, D] ~ U(-1/sqrt(D), 1/sqrt(D)) (the default
    initialisation of a bias-free linear layer).  The default V is the headline batch's vertex count
    (32 shapes of 5000 vertices), D = 128 the usual DiffusionNet width."""
    rng = rng_for(tag, vertices, channels, 0)
    z = rng.standard_normal((vertices, channels, 2)).astype(np.float32)
    s = 1.0 / np.sqrt(channels)
    A_re = rng.uniform(-s, s, (channels, channels)).astype(np.float32)
    A_im = rng.uniform(-s, s, (channels, channels)).astype(np.float32)
    return z, A_re, A_im


def operator_nonorthogonal(rng: np.random.Generator, k: int, skew: float = 0.1) -> np.ndarray:
    """A Laplacian-like operator expressed in a non-orthogonal basis: Q diag(mu) Q^{-1} with mu the sorted
    eigenvalue draw of `eigenvalues_linear` and Q = I + skew N (N ~ N(0, 1/k)), i.e. real positive spectrum,
    non-symmetric matrix, nearly diagonal for small skew."""
    mu = eigenvalues_linear(rng, k)
    Q = np.eye(k) + skew * rng.standard_normal((k, k)) / np.sqrt(k)
    return (Q * mu) @ np.linalg.inv(Q)


def workload_vectorized(pairs: int = 256, k: int = 16, d: int = 256, *, ky: Optional[int] = None, lam: float = 0.1,
                        skew: float = 0.1, tag: int = 8):
    """Inputs of the vectorized solve with general operators: A [P, kx, d] ~ N(0, 1/d) and B = C0 A + 0.05 E
    with C0 ~ N(0, 1/kx) (a synthesized map plus noise), operators from `operator_nonorthogonal` for both sides,
    lambda [P] = lam.  Float32, rounded once."""
    kx = k
    ky = k if ky is None else ky
    A = np.empty((pairs, kx, d), np.float32)
    B = np.empty((pairs, ky, d), np.float32)
    D1 = np.empty((pairs, kx, kx), np.float32)
    D2 = np.empty((pairs, ky, ky), np.float32)
    for p in range(pairs):
        rng = rng_for(tag, pairs, kx, ky, d, p)
        a = rng.standard_normal((kx, d)) / np.sqrt(d)
        c0 = rng.standard_normal((ky, kx)) / np.sqrt(kx)
        A[p] = a
        B[p] = c0 @ a + 0.05 * rng.standard_normal((ky, d)) / np.sqrt(d)
        D1[p] = operator_nonorthogonal(rng, kx, skew)
        D2[p] = operator_nonorthogonal(rng, ky, skew)
    return A, B, D1, D2, np.full(pairs, lam, np.float32)

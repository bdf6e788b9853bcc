"""GPU parity of the overlap metrics (Sec. 3.3) against the oracle.

Counts are integers: bit-exact.  The metrics are computed on both sides in
float64 from the same counts with the same operations and rounded once to
float32, so they are compared for equality too.  Shapes of every size class:
empty, a single vertex, shorter than one 256-vertex row, rows crossing shape
boundaries, and the evaluation-batch workload (1024 shapes, 2000-20000
vertices each).
"""
import numpy as np
import pytest

from oracle import overlap as ov
from paper_2604_10377_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F(dev):
    from paper_2604_10377_amd import fmap
    return fmap


def _run(F, dev, scores, truth, off, thr):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    counts, mets = F.fmap_overlap_metrics(t(scores), t(truth), t(off), thr)
    torch.cuda.synchronize()
    return counts.cpu().numpy(), mets.cpu().numpy()


def _check(F, dev, scores, truth, off, thr=0.5):
    c, m = _run(F, dev, scores, truth, off, thr)
    rc, rm = ov.overlap_batch(scores, truth, off, thr)
    np.testing.assert_array_equal(c, rc)
    np.testing.assert_array_equal(m, rm.astype(np.float32))


@pytest.mark.parametrize("lens", [[0], [1], [5, 0, 300, 1, 0, 257, 255, 256, 1000], [70000], [3] * 500,
                                  [0, 0, 0, 12345, 0]])
def test_overlap_small_and_boundary_shapes(F, dev, lens):
    rng = np.random.default_rng(len(lens))
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    n = int(off[-1])
    scores = rng.random(n).astype(np.float32)
    scores[::7] = 0.5   # exactly at the threshold: negative
    scores[::11] = np.nan  # NaN: negative
    truth = rng.integers(0, 2, n).astype(np.uint8)
    print("overlap shapes", lens[:10], "total", n, flush=True)
    _check(F, dev, scores, truth, off)


def test_overlap_degenerate_predictors(F, dev):
    """Zeros, Ones and coin-flip predictors over shapes of every overlap ratio: balanced accuracy 0.5
    for Zeros and Ones (exactly), counts and metrics equal to the oracle's."""
    b = synth.workload_overlap(shapes=64, n_lo=500, n_hi=3000)
    for name, sc in (("zeros", np.zeros_like(b.scores)), ("ones", np.ones_like(b.scores)),
                     ("coin", np.random.default_rng(3).random(b.scores.shape[0]).astype(np.float32))):
        c, m = _run(F, dev, sc, b.truth, b.offsets, 0.5)
        rc, rm = ov.overlap_batch(sc, b.truth, b.offsets, 0.5)
        np.testing.assert_array_equal(c, rc)
        np.testing.assert_array_equal(m, rm.astype(np.float32))
        if name != "coin":
            has_both = (c[:, 0] + c[:, 2] > 0) & (c[:, 1] + c[:, 3] > 0)
            assert (m[has_both, 6] == 0.5).all(), name


def test_overlap_evaluation_batch_full_size(F, dev):
    """1024 shapes of 2000-20000 vertices (about 11M vertices), thresholds 0.5 and 0.3."""
    b = synth.workload_overlap()
    for thr in (0.5, 0.3):
        _check(F, dev, b.scores, b.truth, b.offsets, thr)


def test_overlap_repeat_calls_identical(F, dev):
    b = synth.workload_overlap(shapes=100)
    r1 = _run(F, dev, b.scores, b.truth, b.offsets, 0.5)
    r2 = _run(F, dev, b.scores, b.truth, b.offsets, 0.5)
    np.testing.assert_array_equal(r1[0], r2[0])
    np.testing.assert_array_equal(r1[1], r2[1])

"""Pins for the overlap-metric oracle (Sec. 3.3), independent of its code.

The paper fixes the expected confusion counts of three degenerate predictors
(Zeros, Ones, Random) as functions of the overlap ratio r, and states that
balanced accuracy is 0.5 for all three at every r.  Those closed forms, a
hand-worked fixture, brute-force counting and label symmetries pin the
counting and every metric formula: a wrong denominator, a metric built from
the wrong counts or a non-strict threshold fails at least one of them.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import overlap as ov

GOLD = os.path.join(os.path.dirname(__file__), "golden")
IDX = {name: i for i, name in enumerate(ov.METRIC_NAMES)}


def _labels(N, r, seed):
    """Ground truth with exactly round(r N) overlapping vertices, in a seeded random order."""
    npos = int(round(r * N))
    gt = np.zeros(N, np.uint8)
    gt[:npos] = 1
    np.random.default_rng(seed).shuffle(gt)
    return gt, npos


def test_golden_ten_vertices():
    g = json.load(open(os.path.join(GOLD, "overlap_10.json")))
    counts = ov.confusion_counts(np.array(g["scores"], np.float32), np.array(g["truth"]), 0.5)
    assert list(counts) == g["counts"]
    m = ov.metrics_from_counts(*counts)
    for name, frac in g["metrics"].items():
        assert m[IDX[name]] == pytest.approx(float(Fraction(frac)), abs=1e-15), name


@pytest.mark.parametrize("r", [0.05, 0.3, 0.5, 0.8, 0.97])
def test_degenerate_predictors_closed_forms(r):
    """Zeros, Ones and an exactly balanced Random predictor (half of each class positive): the counts
    of Sec. 3.3 and the metrics they imply; balanced accuracy is 0.5 for all three."""
    N = 2000
    gt, P = _labels(N, r, 1)
    Q = N - P
    zeros = np.zeros(N, np.float32)
    ones = np.ones(N, np.float32)
    half = np.zeros(N, np.float32)  # every second vertex of each class predicted positive
    half[np.flatnonzero(gt)[::2]] = 1.0
    half[np.flatnonzero(gt == 0)[::2]] = 1.0
    cz, co, ch = (ov.confusion_counts(s, gt, 0.5) for s in (zeros, ones, half))
    assert cz == (0, 0, P, Q)
    assert co == (P, Q, 0, 0)
    tp_h, fp_h = (P + 1) // 2, (Q + 1) // 2
    assert ch == (tp_h, fp_h, P - tp_h, Q - fp_h)
    mz, mo, mh = (ov.metrics_from_counts(*c) for c in (cz, co, ch))
    rr = P / N
    # Zeros: accuracy 1 - r, nothing predicted: precision, recall, IoU, F1 = 0, specificity 1
    np.testing.assert_allclose(mz, [1 - rr, 0, 0, 1, 0, 0, 0.5], atol=1e-15)
    # Ones: accuracy = precision = IoU = r, recall 1, specificity 0, F1 = 2r / (1 + r)
    np.testing.assert_allclose(mo, [rr, rr, 1, 0, rr, 2 * rr / (1 + rr), 0.5], atol=1e-15)
    # balanced Random (exact halves when the class sizes are even)
    if P % 2 == 0 and Q % 2 == 0:
        np.testing.assert_allclose(mh, [0.5, rr, 0.5, 0.5, rr / (1 + rr), 2 * rr / (2 * rr + 1), 0.5], atol=1e-15)
    assert abs(mh[IDX["balanced_accuracy"]] - 0.5) <= 1.0 / min(P, Q)


def test_random_predictor_balanced_accuracy_in_expectation():
    """Each vertex positive with probability 1/2: balanced accuracy concentrates at 0.5 (within 5 sigma)
    while accuracy, IoU and F1 follow r."""
    N = 200_000
    for r in (0.1, 0.6):
        gt, P = _labels(N, r, 2)
        s = np.random.default_rng(3).random(N).astype(np.float32)
        m = ov.metrics_from_counts(*ov.confusion_counts(s, gt, 0.5))
        sigma = 0.5 * np.sqrt(0.25 / P + 0.25 / (N - P))
        assert abs(m[IDX["balanced_accuracy"]] - 0.5) <= 5 * sigma
        assert abs(m[IDX["precision"]] - r) <= 5 * np.sqrt(r * (1 - r) / (N / 2))


def test_counts_match_brute_force_loop():
    rng = np.random.default_rng(4)
    for N in (0, 1, 7, 100):
        s = rng.random(N).astype(np.float32)
        s[::5] = 0.5  # exactly at the threshold: negative
        gt = rng.integers(0, 2, N)
        c = [0, 0, 0, 0]
        for v in range(N):
            pos = float(s[v]) > 0.5
            c[(0 if gt[v] else 1) if pos else (2 if gt[v] else 3)] += 1
        assert ov.confusion_counts(s, gt, 0.5) == tuple(c)


def test_label_symmetries():
    """Swapping prediction and truth swaps FP and FN and keeps IoU and F1; complementing both labels swaps
    TP with TN and FP with FN and keeps accuracy and balanced accuracy."""
    rng = np.random.default_rng(5)
    N = 5000
    pred = rng.integers(0, 2, N)
    gt = rng.integers(0, 2, N)
    tp, fp, fn, tn = ov.confusion_counts(pred.astype(np.float32), gt, 0.5)
    assert tp + fp + fn + tn == N
    assert ov.confusion_counts(gt.astype(np.float32), pred, 0.5) == (tp, fn, fp, tn)
    assert ov.confusion_counts((1 - pred).astype(np.float32), 1 - gt, 0.5) == (tn, fn, fp, tp)
    m = ov.metrics_from_counts(tp, fp, fn, tn)
    ms = ov.metrics_from_counts(tp, fn, fp, tn)
    mc = ov.metrics_from_counts(tn, fn, fp, tp)
    for name in ("iou", "f1", "accuracy"):
        assert m[IDX[name]] == pytest.approx(ms[IDX[name]], abs=1e-15)
    for name in ("accuracy", "balanced_accuracy"):
        assert m[IDX[name]] == pytest.approx(mc[IDX[name]], abs=1e-15)


def test_single_class_and_empty_shapes():
    """Ground truth with one class only: balanced accuracy is that class's recall; empty shape: all 0."""
    m = ov.metrics_from_counts(0, 3, 0, 7)  # no overlapping vertex: specificity 7/10
    assert m[IDX["balanced_accuracy"]] == pytest.approx(0.7, abs=1e-15)
    m = ov.metrics_from_counts(4, 0, 1, 0)  # every vertex overlapping: recall 4/5
    assert m[IDX["balanced_accuracy"]] == pytest.approx(0.8, abs=1e-15)
    assert (ov.metrics_from_counts(0, 0, 0, 0) == 0).all()


def test_batch_equals_per_shape():
    rng = np.random.default_rng(6)
    lens = [0, 13, 1, 400, 0, 77]
    off = np.concatenate([[0], np.cumsum(lens)])
    s = rng.random(off[-1]).astype(np.float32)
    gt = rng.integers(0, 2, off[-1]).astype(np.uint8)
    counts, mets = ov.overlap_batch(s, gt, off, 0.3)
    for i in range(len(lens)):
        c = ov.confusion_counts(s[off[i]:off[i + 1]], gt[off[i]:off[i + 1]], 0.3)
        assert tuple(counts[i]) == c
        np.testing.assert_array_equal(mets[i], ov.metrics_from_counts(*c))

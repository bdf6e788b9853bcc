"""Double-precision CPU oracle for the overlap-prediction metrics (Sec. 3.3).

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline leg
may import this module; the GPU library and its Python binding never do.  It
shares no code with the GPU path.

A predictor labels each vertex of a shape as overlapping (positive) or not;
the ground truth labels the truly overlapping vertices.  Sec. 3.3 works with
the confusion counts TP, FP, FN, TN of one shape and the metrics built from
them; balanced accuracy is the mean of sensitivity TP / (TP + FN) and
specificity TN / (TN + FP).

Readings (the paper does not fix them):
  * a vertex is predicted positive when its score is strictly greater than the
    threshold (both in float32; a NaN score is negative);
  * a ratio whose denominator is zero (e.g. precision of the Zeros predictor)
    is 0;
  * balanced accuracy averages the class recalls that are defined: a shape
    whose ground truth holds one class only gets that class's recall, an
    empty shape gets 0.
Metrics are computed in float64 from the exact integer counts.

Functions:
  confusion_counts   TP, FP, FN, TN of one shape (plain counting)
  metrics_from_counts  accuracy, precision, recall (sensitivity), specificity,
                       IoU, F1 and balanced accuracy
  overlap_batch      counts and metrics of every shape of a concatenated batch
"""
from __future__ import annotations

import numpy as np

METRIC_NAMES = ("accuracy", "precision", "recall", "specificity", "iou", "f1", "balanced_accuracy")


def predicted_positive(scores, threshold: float) -> np.ndarray:
    """Positive iff score > threshold, compared in float32."""
    s = np.asarray(scores, dtype=np.float32)
    return s > np.float32(threshold)


def confusion_counts(scores, truth, threshold: float = 0.5):
    """(TP, FP, FN, TN) of one shape: scores [N] float, truth [N] (nonzero = overlapping)."""
    pos = predicted_positive(scores, threshold)
    gt = np.asarray(truth) != 0
    assert pos.shape == gt.shape
    tp = int(np.count_nonzero(pos & gt))
    fp = int(np.count_nonzero(pos & ~gt))
    fn = int(np.count_nonzero(~pos & gt))
    tn = int(np.count_nonzero(~pos & ~gt))
    return tp, fp, fn, tn


def _ratio(num: int, den: int) -> float:
    return float(num) / float(den) if den != 0 else 0.0


def metrics_from_counts(tp: int, fp: int, fn: int, tn: int) -> np.ndarray:
    """The seven metrics in METRIC_NAMES order, float64."""
    n = tp + fp + fn + tn
    acc = _ratio(tp + tn, n)
    prec = _ratio(tp, tp + fp)
    sens = _ratio(tp, tp + fn)
    spec = _ratio(tn, tn + fp)
    iou = _ratio(tp, tp + fp + fn)
    f1 = _ratio(2 * tp, 2 * tp + fp + fn)
    defined = [r for r, den in ((sens, tp + fn), (spec, tn + fp)) if den != 0]
    bal = sum(defined) / len(defined) if defined else 0.0
    return np.array([acc, prec, sens, spec, iou, f1, bal], dtype=np.float64)


def overlap_batch(scores, truth, offsets, threshold: float = 0.5):
    """Shapes s = 0..S-1 occupy [offsets[s], offsets[s+1]) of the concatenated arrays.

    Returns counts [S, 4] int64 (TP, FP, FN, TN) and metrics [S, 7] float64."""
    offsets = np.asarray(offsets, dtype=np.int64)
    S = offsets.shape[0] - 1
    counts = np.zeros((S, 4), np.int64)
    mets = np.zeros((S, 7), np.float64)
    for s in range(S):
        a, b = int(offsets[s]), int(offsets[s + 1])
        counts[s] = confusion_counts(scores[a:b], truth[a:b], threshold)
        mets[s] = metrics_from_counts(*(int(x) for x in counts[s]))
    return counts, mets

"""Segmentation accuracy measures of the paper's evaluation (Sec. V.A, Eqs. 1-3).

TEST INFRASTRUCTURE ONLY.

recall    R = TP / (TP + FN)          (Eq. 1)
precision P = TP / (TP + FP)          (Eq. 2)
F1        = 2 P R / (P + R)           (Eq. 3)
An undefined ratio (zero denominator) is reported as NaN.
"""
from __future__ import annotations

import numpy as np


def confusion(pred, truth):
    pred = np.asarray(pred, dtype=bool).ravel()
    truth = np.asarray(truth, dtype=bool).ravel()
    tp = int(np.count_nonzero(pred & truth))
    fp = int(np.count_nonzero(pred & ~truth))
    tn = int(np.count_nonzero(~pred & ~truth))
    fn = int(np.count_nonzero(~pred & truth))
    return tp, fp, tn, fn


def _ratio(num, den):
    return float(num) / float(den) if den else float("nan")


def recall(pred, truth) -> float:
    tp, fp, tn, fn = confusion(pred, truth)
    return _ratio(tp, tp + fn)


def precision(pred, truth) -> float:
    tp, fp, tn, fn = confusion(pred, truth)
    return _ratio(tp, tp + fp)


def f1_score(pred, truth) -> float:
    P = precision(pred, truth)
    R = recall(pred, truth)
    if np.isnan(P) or np.isnan(R) or P + R == 0:
        return float("nan")
    return 2.0 * P * R / (P + R)

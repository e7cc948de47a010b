"""Segmentation quality of device masks against a reference mask (Sec. V.A, Eqs. 1-3).

recall R = TP/(TP+FN) (Eq. 1), precision P = TP/(TP+FP) (Eq. 2), F1 = 2PR/(P+R) (Eq. 3). The
counts come from the library's gmm_mask_confusion kernel on bit-packed device masks; only the
three ratios are formed on the host. An undefined ratio is NaN.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

from . import _abi


@dataclass(frozen=True)
class Confusion:
    tp: int
    fp: int
    tn: int
    fn: int

    @property
    def recall(self) -> float:
        d = self.tp + self.fn
        return self.tp / d if d else math.nan

    @property
    def precision(self) -> float:
        d = self.tp + self.fp
        return self.tp / d if d else math.nan

    @property
    def f1(self) -> float:
        p, r = self.precision, self.recall
        if math.isnan(p) or math.isnan(r) or p + r == 0:
            return math.nan
        return 2 * p * r / (p + r)


def pack_mask(bits):
    """Bool device tensor (any shape, row-major pixel order) -> bit-packed int64 words."""
    import torch
    flat = bits.reshape(-1).to(torch.int64)
    n = flat.numel()
    pad = (-n) % 64
    if pad:
        flat = torch.cat([flat, torch.zeros(pad, dtype=torch.int64, device=flat.device)])
    shifts = torch.arange(64, dtype=torch.int64, device=flat.device)
    # distinct powers of two: the int64 sum is exact (bit 63 wraps to the sign bit)
    return (flat.view(-1, 64) << shifts).sum(dim=1)


def confusion(pred_words, truth_words, npix: int, counts=None, stream=None) -> Confusion:
    """TP/FP/TN/FN of two bit-packed device masks (synchronises to read the counts)."""
    import torch
    if counts is None:
        counts = torch.empty(4, dtype=torch.int64, device=pred_words.device)
    _abi.gmm_mask_confusion(pred_words, truth_words, npix, counts, stream)
    tp, fp, tn, fn = (int(v) for v in counts.cpu().tolist())
    return Confusion(tp, fp, tn, fn)

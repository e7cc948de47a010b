"""Oracle of the colour/depth foreground fusion rule (paper Sec. III.C, List 1).

TEST INFRASTRUCTURE ONLY.

Per pixel the rule keeps a fused bit I and an integer counter cpt (both persistent across
frames; both start at 0 here). With r, d the colour and depth foreground bits:
  * r == d: I takes the common value and the counter resets;
  * r != d and cpt == +3: I takes the colour bit, counter reset;
  * r != d and cpt == -3: I takes the depth bit, counter reset;
  * otherwise the counter moves by +1 when I equals the colour bit and by -1 when it does not,
    and I is kept.
The saturation checks come before the counter moves (the listing's order), and the listing's
lower- and upper-case names of the same images are read as the same variables. The fused
output of the frame is the new I.
"""
from __future__ import annotations

import numpy as np


def fuse_step(r, d, I, cpt):
    """One transition of the rule, vectorised. Returns (I_new, cpt_new)."""
    r = np.asarray(r).astype(np.int64)
    d = np.asarray(d).astype(np.int64)
    I = np.asarray(I).astype(np.int64)
    cpt = np.asarray(cpt).astype(np.int64)
    agree = r == d
    sat_pos = ~agree & (cpt == 3)
    sat_neg = ~agree & (cpt == -3)
    moving = ~agree & ~sat_pos & ~sat_neg
    I_new = np.where(agree, d, np.where(sat_pos, r, np.where(sat_neg, d, I)))
    cpt_new = np.where(moving, np.where(I == r, cpt + 1, cpt - 1), 0)
    return I_new, cpt_new


class FusionOracle:
    """Fusion state of n pixels."""

    def __init__(self, n: int):
        self.I = np.zeros(n, dtype=np.int64)
        self.cpt = np.zeros(n, dtype=np.int64)

    def step(self, fg_rgb, fg_depth) -> np.ndarray:
        self.I, self.cpt = fuse_step(fg_rgb, fg_depth, self.I, self.cpt)
        return self.I.astype(bool)

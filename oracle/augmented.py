"""FP64 oracle of the augmentation variant: one four-channel mixture over R, G, B and depth.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the product path.

Sec. III.B of the paper describes, and rejects, adding depth to the colour model as a fourth
channel beside the three colour bytes (its Fig. 2); the method keeps the two modalities in
separate mixtures instead. This module models that rejected variant for the ablation: the
per-pixel step of ``mixture`` with C = 4, fed x = (R, G, B, D8).

Readings (the paper gives no detail of the variant):
  * depth enters as an intensity byte, D8 = min(255, floor(depth_mm / 16)): a 16 mm quantum,
    0..4080 mm, the working range of a Kinect v1 depth map;
  * one isotropic variance per component over all four channels, with the colour model's
    sigma0 and variance floor (depth is just one more byte);
  * a depth hole (0) with the hole policy on leaves the pixel's state untouched and classifies
    it background, as in the depth-only model.
"""
from __future__ import annotations

import numpy as np

from .mixture import MixParams, MixtureOracle, StepInfo


def depth_byte(depth) -> np.ndarray:
    """Depth in millimetres (integers) to the fourth intensity byte."""
    d = np.asarray(depth, dtype=np.int64)
    return np.minimum(d // 16, 255)


class AugmentedOracle:
    """Four-channel mixture state of n pixels (axis 0 of every array is the rank)."""

    def __init__(self, params: MixParams, n: int, storage=None):
        self.p = params
        self.n = n
        self.model = MixtureOracle(params, 4, n, storage)

    def get_state(self):
        return self.model.get_state()

    def set_state(self, mu, var, w):
        self.model.set_state(mu, var, w)

    def step(self, rgb, depth) -> StepInfo:
        rgb = np.asarray(rgb, dtype=np.float64).reshape(self.n, 3)
        d = np.asarray(depth).reshape(self.n)
        x = np.concatenate([rgb, depth_byte(d).astype(np.float64)[:, None]], axis=1)
        hole = (d == 0) if self.p.hole_skip else np.zeros(self.n, dtype=bool)
        return self.model.step(x, hole=hole)

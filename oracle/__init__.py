"""FP64 CPU oracle of the RGB-D mixture-of-Gaussians segmentation (test infrastructure).

This package is TEST INFRASTRUCTURE, not part of the product. Only the test suite, the
smoke check of ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.
The GPU path never calls into it and shares no code with it.

Contents (each module cites the passage of the paper it follows):
  mixture  - vectorised per-pixel mixture update and classification (Sec. III.A), float64
  scalar   - an independent pure-Python per-pixel version of the same step (tiny inputs)
  augmented - the four-channel R, G, B, depth mixture the paper rejects (Sec. III.B), ablation
  fusion   - the List 1 fusion of the colour and depth foreground masks (Sec. III.C)
  metrics  - recall, precision and F1 (Sec. V.A, Eqs. 1-3)

Where the paper is silent it defers to Stauffer and Grimson (its reference [6]); the
readings taken for every silent or garbled point are listed in the design notes and
repeated at the top of ``mixture``.
"""
from .mixture import MixParams, MixtureOracle, StepInfo, round_to_storage
from .scalar import ScalarMixture
from .augmented import AugmentedOracle, depth_byte
from .fusion import fuse_step, FusionOracle
from .metrics import recall, precision, f1_score, confusion

__all__ = [
    "MixParams", "MixtureOracle", "StepInfo", "round_to_storage", "ScalarMixture", "AugmentedOracle", "depth_byte",
    "fuse_step", "FusionOracle", "recall", "precision", "f1_score", "confusion",
]

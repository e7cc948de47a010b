"""Pure-Python, one-pixel-at-a-time oracle of the mixture step (paper Sec. III.A).

TEST INFRASTRUCTURE ONLY. An independently written second implementation of the step that
``mixture`` vectorises, used on tiny frames so the two can be checked against each other.
It follows the same readings (listed in ``mixture``'s docstring), written as plain loops over
a list of components rather than as array operations.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

from .mixture import MixParams


class ScalarMixture:
    """One pixel of one modality. ``comps[r] = [mean list, variance, weight]`` in rank order."""

    def __init__(self, params: MixParams, C: int):
        self.p = params
        self.C = C
        self.comps: List[list] = [[[0.0] * C, float(params.sigma0) ** 2, 0.0] for _ in range(params.M)]

    def state(self) -> Tuple[list, list, list]:
        return ([list(c[0]) for c in self.comps], [c[1] for c in self.comps], [c[2] for c in self.comps])

    def step(self, x: Sequence[float], hole=None) -> bool:
        p = self.p
        a = float(p.alpha)
        xs = [float(v) for v in x]
        if hole is None:
            hole = p.hole_skip and self.C == 1 and xs[0] == 0.0
        if hole:
            return False

        # which component explains x: the first live one, in rank order, inside k sigma
        match = None
        for r, (mean, var, weight) in enumerate(self.comps):
            if weight <= 0.0:
                continue
            dist2 = 0.0
            for xc, mc in zip(xs, mean):
                dist2 += (xc - mc) * (xc - mc)
            if dist2 < (p.k * p.k) * var:
                match = r
                break

        # rate of the mean and variance update
        rate = a
        if match is not None and p.rho == "density":
            var_j = self.comps[match][1]
            density = math.exp(-dist2 / (2.0 * var_j)) / math.pow(2.0 * math.pi * var_j, self.C / 2.0)
            rate = a * density

        updated = []
        for r, (mean, var, weight) in enumerate(self.comps):
            weight = (1.0 - a) * weight + (a if r == match else 0.0)
            if r == match:
                mean = [(1.0 - rate) * mc + rate * xc for mc, xc in zip(mean, xs)]
                res = 0.0
                for xc, mc in zip(xs, mean):
                    res += (xc - mc) * (xc - mc)
                var = max(p.var_min, (1.0 - rate) * var + rate * res)
            updated.append([list(mean), var, weight])
        if match is None:
            updated[-1] = [list(xs), float(p.sigma0) ** 2, p.w_init]
            changed = len(updated) - 1
        else:
            changed = match

        total = 0.0
        for c in updated:
            total += c[2]
        for c in updated:
            c[2] = c[2] / total

        # Python's sort is stable: equal keys keep their previous rank order
        tagged = [(c, r == changed) for r, c in enumerate(updated)]
        tagged.sort(key=lambda t: -(t[0][2] / math.sqrt(t[0][1])))
        self.comps = [t[0] for t in tagged]
        q = [t[1] for t in tagged].index(True)

        B = p.M
        running = 0.0
        for b, c in enumerate(self.comps, start=1):
            running += c[2]
            if running > p.T:
                B = b
                break
        return match is None or q >= B

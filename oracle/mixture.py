"""Vectorised FP64 oracle of the per-pixel mixture-of-Gaussians background model.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the product path.

What it computes (paper Sec. III.A, with the update rules of Stauffer and Grimson, the
paper's reference [6], where the paper defers to them). Per pixel, per frame, for one
modality with C channels (C=3 colour, C=1 depth) and M components kept in rank order:

  0. initial state: every component empty (w = 0, mu = 0, var = sigma0^2)
  1. input x (integers converted exactly to float64). With the hole policy on, a depth value
     of 0 leaves the pixel's state untouched and classifies it as background
  2. match: walk the ranks in stored order; rank r matches when it is live (w > 0) and
     ||x - mu_r||^2 < k^2 var_r (strict). The first match j wins
  3. weights: w_r <- (1 - alpha) w_r + alpha [r = j]
  4. matched: mu_j <- (1 - alpha) mu_j + alpha x;
              var_j <- max(var_min, (1 - alpha) var_j + alpha ||x - mu_j(new)||^2)
     no match: the last rank is replaced: mu = x, var = sigma0^2, w = w_init
  5. renormalise: w <- w / sum(w)
  6. stable sort by w / sqrt(var), descending (equal keys keep their previous order)
  7. B = min{ b >= 1 : w_0 + ... + w_{b-1} > T } (at most M); the pixel is foreground when
     nothing matched or when the updated component's new rank is >= B

Readings taken where the paper is silent or garbled (each pinned by a test where a pin exists):
  * the mean and variance learning rate equals alpha;
  * colour uses one isotropic variance per component and the plain squared distance over the
    three channels; the variance update uses the undivided squared norm;
  * ranks are tested in decreasing w/sigma order and the first match wins;
  * the replaced component on no match is the last-ranked one (an empty slot when one exists);
  * a new component enters with weight w_init after the decay, then all are renormalised;
  * the variance update uses the new mean; variances are floored at var_min;
  * classification happens after the update and the re-sort, with a strict "> T";
  * the match test is strict (a distance exactly k sigma does not match);
  * depth 0 is a missing reading (optional, the hole policy).

Variant (an ablation, ``MixParams.rho = "density"``): the mean and variance rate is
Stauffer and Grimson's rho = alpha * eta(x | mu_j, var_j I), the C-variate isotropic Gaussian
density of x under the matched component before its update,
eta = (2 pi var_j)^(-C/2) exp(-||x - mu_j||^2 / (2 var_j)).

Besides the result, every step records how close each discrete decision came to flipping
(``StepInfo``), so a finite-precision implementation can be compared pixel by pixel with
its legitimately ambiguous decisions excused.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass(frozen=True)
class MixParams:
    M: int
    alpha: float
    k: float
    T: float
    sigma0: float
    var_min: float
    w_init: float
    hole_skip: bool = False   # depth only: value 0 means "no reading"
    rho: str = "alpha"        # "alpha" or "density" (rate of the mean and variance updates)


@dataclass
class StepInfo:
    fg: np.ndarray             # bool (n,) foreground
    matched: np.ndarray        # bool (n,)
    j: np.ndarray              # int (n,) matched rank before the step, -1 if none
    q: np.ndarray              # int (n,) rank after the sort of the matched / new component
    B: np.ndarray              # int (n,) number of background components
    hole: np.ndarray           # bool (n,) pixel skipped as a hole
    match_margin: np.ndarray   # (n,) min over tested live ranks of |sqrt(d2) - k sigma| / sigma
    weight_margin: np.ndarray  # (n,) |cumulative weight before rank q - T| (matched, q >= 1)
    key_gap: np.ndarray        # (n,) min relative gap between adjacent live keys after the sort


def _bf16_round(v: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (8 significant bits), ties to even."""
    v = np.asarray(v, dtype=np.float64)
    out = v.copy()
    fin = np.isfinite(v) & (v != 0)
    m, e = np.frexp(v[fin])                      # v = m * 2^e, 0.5 <= |m| < 1
    # quantum: 2^(e-8) for normal values, 2^-133 below the smallest normal (2^-126)
    qexp = np.maximum(e - 8, -133)
    scaled = np.ldexp(v[fin], -qexp)             # exact (power-of-two scaling)
    out[fin] = np.ldexp(np.rint(scaled), qexp)   # rint: ties to even
    big = np.abs(out) >= 2.0 ** 128
    out[big] = np.copysign(np.inf, out[big])
    return out


def round_to_storage(v: np.ndarray, storage: Optional[str]) -> np.ndarray:
    """Emulate storing float64 values in a narrower format (round to nearest, ties to even)."""
    if storage is None or storage == "f64":
        return v
    if storage == "f32":
        return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)
    if storage == "f16":
        return np.asarray(v, dtype=np.float64).astype(np.float16).astype(np.float64)
    if storage == "bf16":
        return _bf16_round(v)
    raise ValueError(storage)


class MixtureOracle:
    """Mixture state of n pixels of one modality; axis 0 of every array is the rank."""

    def __init__(self, params: MixParams, C: int, n: int, storage: Optional[str] = None):
        if not 1 <= params.M:
            raise ValueError("M must be >= 1")
        self.p = params
        self.C = C
        self.n = n
        self.storage = storage
        self.mu = np.zeros((params.M, C, n))
        self.var = np.full((params.M, n), float(params.sigma0) ** 2)
        self.w = np.zeros((params.M, n))

    # -- state access ---------------------------------------------------------------------
    def get_state(self):
        return self.mu.copy(), self.var.copy(), self.w.copy()

    def set_state(self, mu, var, w):
        self.mu = np.array(mu, dtype=np.float64).reshape(self.p.M, self.C, self.n)
        self.var = np.array(var, dtype=np.float64).reshape(self.p.M, self.n)
        self.w = np.array(w, dtype=np.float64).reshape(self.p.M, self.n)

    # -- one frame --------------------------------------------------------------------------
    def step(self, x, hole=None) -> StepInfo:
        """Advance one frame. ``hole`` (bool (n,)) marks pixels to skip; by default, with the
        hole policy on, a one-channel value of 0."""
        p, M, C, n = self.p, self.p.M, self.C, self.n
        a = float(p.alpha)
        x = np.asarray(x, dtype=np.float64).reshape(n, C).T          # (C, n)
        mu, var, w = self.mu, self.var, self.w

        if hole is not None:
            hole = np.asarray(hole, dtype=bool).reshape(n)
        elif p.hole_skip and C == 1:
            hole = x[0] == 0.0
        else:
            hole = np.zeros(n, dtype=bool)

        # 2. match, ranks in stored order, first hit wins; record the margins tested
        k2 = p.k * p.k
        j = np.full(n, -1, dtype=np.int64)
        match_margin = np.full(n, np.inf)
        d2_all = np.zeros((M, n))
        for r in range(M):
            live = w[r] > 0.0
            d2 = ((x - mu[r]) ** 2).sum(axis=0)
            d2_all[r] = d2
            hit = live & (d2 < k2 * var[r])
            tested = live & (j < 0)
            sd = np.sqrt(var[r])
            m = np.abs(np.sqrt(d2) - p.k * sd) / sd
            match_margin = np.where(tested, np.minimum(match_margin, m), match_margin)
            j = np.where((j < 0) & hit, r, j)
        matched = j >= 0

        # 3. weight decay, with the matched component reinforced
        onehot = np.arange(M)[:, None] == j[None, :]                 # (M, n)
        w_new = (1.0 - a) * w + a * onehot

        # 4. matched component: mean first, then variance about the new mean, at rate rho
        if p.rho == "alpha":
            rho = np.full(n, a)
        elif p.rho == "density":
            jj = np.maximum(j, 0)[None, :]
            d2j = np.take_along_axis(d2_all, jj, axis=0)[0]
            vj = np.take_along_axis(var, jj, axis=0)[0]
            rho = a * np.exp(-0.5 * d2j / vj) / (2.0 * np.pi * vj) ** (C / 2.0)
        else:
            raise ValueError(p.rho)
        mu_upd = (1.0 - rho) * mu + rho * x[None, :, :]
        resid2 = ((x[None, :, :] - mu_upd) ** 2).sum(axis=1)
        var_upd = np.maximum(p.var_min, (1.0 - rho) * var + rho * resid2)
        mu_new = np.where(onehot[:, None, :], mu_upd, mu)
        var_new = np.where(onehot, var_upd, var)
        #    no match: the last rank is replaced by a new component centred on x
        nm = ~matched
        mu_new[M - 1][:, nm] = x[:, nm]
        var_new[M - 1, nm] = float(p.sigma0) ** 2
        w_new[M - 1, nm] = p.w_init

        # 5. renormalise
        S = w_new.sum(axis=0)
        w_new = w_new / S

        # 6. stable sort by w / sigma, descending
        key = w_new / np.sqrt(var_new)
        order = np.argsort(-key, axis=0, kind="stable")
        mu_s = np.take_along_axis(mu_new, order[:, None, :], axis=0)
        var_s = np.take_along_axis(var_new, order, axis=0)
        w_s = np.take_along_axis(w_new, order, axis=0)
        key_s = np.take_along_axis(key, order, axis=0)
        changed = np.where(matched, j, M - 1)
        q = np.argmax(order == changed[None, :], axis=0)

        # 7. background set and classification
        cum = np.cumsum(w_s, axis=0)                                  # cum[b-1] = c_b
        above = cum > p.T
        B = np.where(above.any(axis=0), above.argmax(axis=0) + 1, M)
        B = np.minimum(B, M)
        fg = nm | (q >= B)

        # decision margins
        c_q = np.where(q >= 1, np.take_along_axis(cum, np.maximum(q - 1, 0)[None, :], axis=0)[0], 0.0)
        weight_margin = np.where(matched & (q >= 1), np.abs(c_q - p.T), np.inf)
        if M > 1:
            nxt_live = key_s[1:] > 0.0
            gaps = np.where(nxt_live, (key_s[:-1] - key_s[1:]) / np.where(key_s[:-1] > 0, key_s[:-1], 1.0),
                            np.inf)
            key_gap = gaps.min(axis=0)
        else:
            key_gap = np.full(n, np.inf)

        # holes: state untouched, background, no decisions taken
        if hole.any():
            keep = hole
            mu_s = np.where(keep[None, None, :], mu, mu_s)
            var_s = np.where(keep[None, :], var, var_s)
            w_s = np.where(keep[None, :], w, w_s)
            fg = fg & ~keep
            matched = matched & ~keep
            j = np.where(keep, -1, j)
            match_margin = np.where(keep, np.inf, match_margin)
            weight_margin = np.where(keep, np.inf, weight_margin)
            key_gap = np.where(keep, np.inf, key_gap)

        if self.storage is not None:
            mu_s = round_to_storage(mu_s, self.storage)
            var_s = round_to_storage(var_s, self.storage)
            w_s = round_to_storage(w_s, self.storage)

        self.mu, self.var, self.w = mu_s, var_s, w_s
        return StepInfo(fg=fg, matched=matched, j=j, q=q, B=B, hole=hole,
                        match_margin=match_margin, weight_margin=weight_margin, key_gap=key_gap)

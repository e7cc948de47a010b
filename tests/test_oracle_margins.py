"""Pins of the oracle's decision margins (``StepInfo.match_margin``, ``weight_margin``,
``key_gap``) against values derived by hand from the definitions of Sec. III.A.

The parity tests excuse a GPU/oracle mask difference only at pixels whose deciding quantity was
within a margin of its threshold, so these margins decide what parity lets through. Each case
below is a state small enough to work through on paper; the expected numbers are written out
from that working, not computed by the oracle's own formulas, so a wrong unit (variance for
standard deviation), a wrong cumulative index, a margin taken over untested or empty ranks, or
keys taken before the re-sort fails a case.

Definitions pinned (a pixel, one modality, components in stored rank order):
  * match margin: over the live ranks the match walk tests (up to and including the matched
    one), the smallest |distance - k sigma| / sigma, in units of sigma;
  * weight margin: for a matched component that lands at rank q >= 1 after the re-sort,
    |w_0 + ... + w_{q-1} - T| (the sum that decides whether q < B); infinite otherwise;
  * key gap: the smallest relative drop (key_r - key_{r+1}) / key_r between adjacent live
    ranks of the re-sorted mixture.
"""
import math

import numpy as np
import pytest

from oracle import MixParams, MixtureOracle


def _one_pixel(M, mus, vars_, ws, alpha=0.5, k=2.5, T=0.7, sigma0=10.0, var_min=1e-2):
    p = MixParams(M=M, alpha=alpha, k=k, T=T, sigma0=sigma0, var_min=var_min, w_init=alpha)
    o = MixtureOracle(p, 1, 1)
    o.set_state(np.array(mus, dtype=np.float64).reshape(M, 1, 1), np.array(vars_, dtype=np.float64).reshape(M, 1),
                np.array(ws, dtype=np.float64).reshape(M, 1))
    return o


def test_match_margin_is_zero_exactly_on_the_boundary():
    # mu = 100, var = 100 (sigma 10), k = 2.5: x = 125 lies exactly 25 = k sigma away
    o = _one_pixel(1, [100.0], [100.0], [1.0])
    info = o.step(np.array([125.0]))
    assert not info.matched[0]             # strict test: on the boundary is no match
    assert info.match_margin[0] == 0.0


def test_match_margin_of_the_hand_trace_step_with_no_match():
    # worked trace, frame 3: state a(mu 105, var 37.5, w 1) and two empty slots; x = 200.
    # distance 95, sigma = sqrt(37.5) = 6.1237..., so the margin is 95 / sqrt(37.5) - 2.5
    o = _one_pixel(3, [105.0, 0.0, 0.0], [37.5, 100.0, 100.0], [1.0, 0.0, 0.0], sigma0=10.0, var_min=1.0)
    info = o.step(np.array([200.0]))
    assert not info.matched[0]
    assert info.match_margin[0] == pytest.approx(13.013435037626794, rel=1e-12)


def test_match_margin_counts_only_the_ranks_the_walk_tests():
    # ranks (mu, var, w): (0, 100, 0.5), (100, 400, 0.4), (160, 100, 0.1); keys 0.05, 0.02, 0.01
    # x = 130, k = 2.5:
    #   rank 0: distance 130, sigma 10, k sigma 25 -> margin (130 - 25) / 10 = 10.5, no match
    #   rank 1: distance 30, sigma 20, k sigma 50 -> margin (50 - 30) / 20 = 1.0, match
    #   rank 2 would give (30 vs 25) / 10 = 0.5 but the walk stops at rank 1
    o = _one_pixel(3, [0.0, 100.0, 160.0], [100.0, 400.0, 100.0], [0.5, 0.4, 0.1], alpha=0.01)
    info = o.step(np.array([130.0]))
    assert info.matched[0] and info.j[0] == 1
    assert info.match_margin[0] == pytest.approx(1.0, rel=1e-14)


def test_match_margin_ignores_empty_components():
    # one live rank (0, 100, 1) and two empty slots (var 900 = sigma0^2); x = 74:
    #   rank 0: distance 74, sigma 10 -> (74 - 25) / 10 = 4.9, no match
    #   an empty slot would give |74 - 75| / 30 = 0.033 but is never tested
    o = _one_pixel(3, [0.0, 0.0, 0.0], [100.0, 900.0, 900.0], [1.0, 0.0, 0.0], sigma0=30.0)
    info = o.step(np.array([74.0]))
    assert not info.matched[0]
    assert info.match_margin[0] == pytest.approx(4.9, rel=1e-14)


def test_weight_margin_uses_the_weights_ranked_before_the_component():
    # ranks (mu, var, w): (0, 1, 0.5), (50, 1, 0.3), (100, 1, 0.2); alpha = 0.01, T = 0.7; x = 100
    # matches rank 2 only. Weights after decay: 0.495, 0.297, 0.198 + 0.01 = 0.208 (sum 1);
    # var_2 = 0.99, key_2 = 0.208 / sqrt(0.99) = 0.20905 < 0.297, so the order stays and q = 2.
    # The deciding sum is 0.495 + 0.297 = 0.792 > T: foreground, margin 0.792 - 0.7 = 0.092.
    o = _one_pixel(3, [0.0, 50.0, 100.0], [1.0, 1.0, 1.0], [0.5, 0.3, 0.2], alpha=0.01)
    info = o.step(np.array([100.0]))
    assert info.matched[0] and info.j[0] == 2 and info.q[0] == 2
    assert info.B[0] == 2 and info.fg[0]
    assert info.weight_margin[0] == pytest.approx(0.092, abs=1e-12)


def test_weight_margin_after_a_reordering_and_the_key_gap_after_the_sort():
    # same ranks, alpha = 0.1, x = 100 matches rank 2: weights 0.45, 0.27, 0.18 + 0.1 = 0.28,
    # var_2 = 0.9, keys 0.45, 0.27, 0.28 / sqrt(0.9) = 0.295146 -> the updated component passes
    # rank 1: order (0.45, 0.295146, 0.27), q = 1. Deciding sum 0.45: background, margin 0.25.
    # Adjacent relative drops after the sort: (0.45 - 0.295146) / 0.45 = 0.344120 and
    # 1 - 0.27 sqrt(0.9) / 0.28 = 0.085198 (before the sort the second drop would be negative).
    o = _one_pixel(3, [0.0, 50.0, 100.0], [1.0, 1.0, 1.0], [0.5, 0.3, 0.2], alpha=0.1)
    info = o.step(np.array([100.0]))
    assert info.matched[0] and info.j[0] == 2 and info.q[0] == 1
    assert info.B[0] == 2 and not info.fg[0]
    assert info.weight_margin[0] == pytest.approx(0.25, abs=1e-12)
    assert info.key_gap[0] == pytest.approx(0.0851982, abs=1e-7)
    assert info.key_gap[0] == pytest.approx(1.0 - 0.27 * math.sqrt(0.9) / 0.28, rel=1e-12)


def test_weight_margin_is_infinite_at_rank_zero_and_without_a_match():
    # the top component matched and stays on top: no cumulative sum decides anything
    o = _one_pixel(2, [0.0, 50.0], [1.0, 1.0], [0.7, 0.3], alpha=0.1)
    info = o.step(np.array([0.0]))
    assert info.q[0] == 0 and info.weight_margin[0] == np.inf
    # nothing matched: the pixel is foreground whatever the weights
    info = o.step(np.array([1000.0]))
    assert not info.matched[0] and info.weight_margin[0] == np.inf


def test_key_gap_of_a_near_tie_in_closed_form():
    # ranks (mu, var, w): (100, 0.125 (1 + d)^2, 0.4), (0, 4, 0.6) with d = 2e-6; keys
    # 0.4 / (sqrt(0.125)(1 + d)) = 1.131 and 0.3, in order. alpha = 0.5, x = 0 matches rank 1.
    # After the step: weights 0.2, 0.8; var_1 = 2; keys 0.2 / (sqrt(0.125)(1 + d)) = 0.5657 / (1 + d)
    # and 0.8 / sqrt(2) = 0.5657: the updated component goes first by a factor (1 + d), so the
    # key gap is 1 - 1 / (1 + d) = d / (1 + d) (keys taken before the sort would give -d).
    d = 2e-6
    o = _one_pixel(2, [100.0, 0.0], [0.125 * (1 + d) ** 2, 4.0], [0.4, 0.6], alpha=0.5)
    info = o.step(np.array([0.0]))
    assert info.matched[0] and info.j[0] == 1 and info.q[0] == 0
    assert info.key_gap[0] == pytest.approx(d / (1 + d), rel=1e-8)


def test_key_gap_ignores_empty_slots():
    # one live component and an empty slot: no adjacent live pair, the gap is infinite
    o = _one_pixel(2, [10.0, 0.0], [4.0, 100.0], [1.0, 0.0], alpha=0.1)
    info = o.step(np.array([10.0]))
    assert info.matched[0] and info.key_gap[0] == np.inf


def test_holes_take_no_decision():
    p = MixParams(M=2, alpha=0.1, k=2.5, T=0.7, sigma0=50.0, var_min=25.0, w_init=0.1, hole_skip=True)
    o = MixtureOracle(p, 1, 1)
    o.step(np.array([1000.0]))
    info = o.step(np.array([0.0]))
    assert info.hole[0]
    assert info.match_margin[0] == np.inf and info.weight_margin[0] == np.inf and info.key_gap[0] == np.inf

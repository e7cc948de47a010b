"""Helpers of the parity tests: mask unpacking, the canonical state layout of the C ABI,
decision-margin excusal and the comparison tolerances.

Tolerances (fp32 device arithmetic against the float64 oracle):
  * parameters: |gpu - oracle| <= 1e-4 * max(|oracle|, 1) for means and variances and
    <= 1e-4 * max(|oracle|, 1e-3) for weights;
  * masks: a pixel may differ only where the oracle's own decision was within a small margin
    of flipping, and the differing fraction of pixel-frames must stay <= 1e-4.
Margins (from the oracle's StepInfo):
  * match: |sqrt(d2) - k sigma| / sigma below MATCH_MARGIN (1e-3, in units of sigma);
  * weight threshold: |cumulative weight - T| below WEIGHT_MARGIN;
  * ordering: relative gap of two adjacent keys w/sigma below KEY_GAP.
"""
from __future__ import annotations

import numpy as np

MATCH_MARGIN = 1e-3
# one fp32 step: a sum of <= 5 weights carries a few ulps (~1e-7 relative); free running lets
# rounding errors of the exponential recurrences accumulate to ~u/alpha (~1e-5 at alpha=0.01)
WEIGHT_MARGIN_LOCKSTEP = 1e-6
KEY_GAP_LOCKSTEP = 1e-6
WEIGHT_MARGIN_FREE = 1e-4
KEY_GAP_FREE = 1e-4
PARAM_RTOL = 1e-4
MASK_FRACTION = 1e-4


def unpack_mask(words, npix: int) -> np.ndarray:
    """Bit-packed uint64 words (torch int64 tensor or numpy) -> bool array of npix pixels."""
    if hasattr(words, "cpu"):
        words = words.cpu().numpy()
    w = np.ascontiguousarray(words).view(np.uint64)
    bits = np.unpackbits(w.view(np.uint8), bitorder="little")
    return bits[:npix].astype(bool)


def pack_mask(bits: np.ndarray) -> np.ndarray:
    """bool array -> uint64 words viewed as int64 (LSB first, pad bits 0)."""
    n = bits.size
    nw = (n + 63) // 64
    padded = np.zeros(nw * 64, dtype=np.uint8)
    padded[:n] = bits.astype(np.uint8)
    return np.packbits(padded, bitorder="little").view(np.int64)


def to_canonical(col=None, dep=None, fus=None) -> np.ndarray:
    """Oracle state -> the canonical float64 layout of gmm_read_state / gmm_write_state."""
    parts = []
    if col is not None:
        for c in range(3):
            parts.append(col.mu[:, c, :].ravel())
        parts += [col.var.ravel(), col.w.ravel()]
    if dep is not None:
        parts += [dep.mu[:, 0, :].ravel(), dep.var.ravel(), dep.w.ravel()]
    if fus is not None:
        parts += [fus.I.astype(np.float64), fus.cpt.astype(np.float64)]
    return np.concatenate(parts)


def from_canonical(flat: np.ndarray, M: int, n: int, rgb: bool, depth: bool):
    """Canonical layout -> dict with 'rgb' (mu (M,3,n), var, w), 'depth' (...), 'I', 'cpt'."""
    out = {}
    off = 0
    if rgb:
        blk = flat[off:off + 5 * M * n].reshape(5, M, n)
        out["rgb"] = (np.stack([blk[0], blk[1], blk[2]], axis=1), blk[3], blk[4])
        off += 5 * M * n
    if depth:
        blk = flat[off:off + 3 * M * n].reshape(3, M, n)
        out["depth"] = (blk[0][:, None, :], blk[1], blk[2])
        off += 3 * M * n
    if rgb and depth:
        out["I"] = flat[off:off + n]
        out["cpt"] = flat[off + n:off + 2 * n]
    return out


def excused(info, weight_margin=WEIGHT_MARGIN_LOCKSTEP, key_gap=KEY_GAP_LOCKSTEP) -> np.ndarray:
    return (info.match_margin < MATCH_MARGIN) | (info.weight_margin < weight_margin) | (info.key_gap < key_gap)


def param_mismatch(gpu, ora) -> np.ndarray:
    """Per-pixel bool: any parameter outside tolerance. gpu/ora are (mu, var, w) tuples."""
    gmu, gvar, gw = gpu
    omu, ovar, ow = ora
    bad = (np.abs(gmu - omu) > PARAM_RTOL * np.maximum(np.abs(omu), 1.0)).any(axis=(0, 1))
    bad |= (np.abs(gvar - ovar) > PARAM_RTOL * np.maximum(np.abs(ovar), 1.0)).any(axis=0)
    bad |= (np.abs(gw - ow) > PARAM_RTOL * np.maximum(np.abs(ow), 1e-3)).any(axis=0)
    return bad


def oracle_state(o):
    return (o.mu, o.var, o.w)


def aug_to_canonical(o) -> np.ndarray:
    """Four-channel oracle state -> canonical layout (muR, muG, muB, muD8, var, w; rank-major)."""
    mu, var, w = o.get_state()
    return np.concatenate([mu[:, c, :].ravel() for c in range(4)] + [var.ravel(), w.ravel()])


def aug_from_canonical(flat: np.ndarray, M: int, n: int):
    blk = flat.reshape(6, M, n)
    return (np.stack([blk[0], blk[1], blk[2], blk[3]], axis=1), blk[4], blk[5])

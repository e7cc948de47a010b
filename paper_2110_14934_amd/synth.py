"""Seeded synthetic Kinect-shaped RGB-D streams: the inputs of tests and benchmarks.

The paper evaluates on its own Kinect captures (Sec. V.A), which are not available, so
synthetic co-registered colour/depth streams of the same shapes stand in for them:
640x480 and 320x240 (Kinect v1), 512x424 depth and 1920x1080 colour (Kinect v2).

This module holds none of the segmentation arithmetic. It only draws frames. Every random
value is a pure function of (seed, stream, frame, channel, pixel) through a counter-based
32-bit integer hash, evaluated with integer tensor operations, so the same frame comes out
bit-identical on the CPU and on the GPU, and any subset of pixels can be generated alone
(which lets a CPU oracle follow sampled pixels of a full-size stream).

Scene model (one stream):
  * colour background: U{0..255} per pixel and channel, fixed for the stream;
  * depth background: a plane at ``depth_bg`` mm;
  * moving square boxes: colour 200 in every channel, depth ``depth_box`` mm, integer
    velocity along one of the 8 compass directions, reflecting at the borders; later boxes
    occlude earlier ones;
  * colour frame t: round_half_even(g(t) * scene + sigma_c * z), clipped to [0, 255];
  * depth frame t: round_half_even(scene + sigma_d * z), clipped to [1, 65535], then each
    pixel independently set to 0 (a hole, "no reading") with probability ``hole_p``;
  * z is an Irwin-Hall(12) standard-normal approximation: the sum of twelve 16-bit uniforms
    (mean 0, variance 1, tails to +-6), built from integers so it is exact on any device;
  * g(t) is a global colour gain: 1, or a ramp from ``gain_lo`` to ``gain_hi`` over frames
    [ramp_t0, ramp_t1] (constant outside it).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

MASK32 = 0xFFFFFFFF
_C1 = 0x7FEB352D
_C2 = 0x846CA68B

# channel tags used to derive independent hash keys
_TAG_BG = 1
_TAG_NOISE_C = 2
_TAG_NOISE_D = 3
_TAG_HOLE = 4


def _mix32_int(x: int) -> int:
    """32-bit avalanche hash on a Python int: two xorshift-multiply rounds with the shifts and
    multipliers of Chris Wellons' published "lowbias32" integer hash (hash-prospector)."""
    x &= MASK32
    x ^= x >> 16
    x = (x * _C1) & MASK32
    x ^= x >> 15
    x = (x * _C2) & MASK32
    x ^= x >> 16
    return x


def _mix32(x: torch.Tensor) -> torch.Tensor:
    """Same hash on an int64 tensor holding values in [0, 2^32).

    The products overflow int64 and wrap; masking keeps the exact low 32 bits."""
    x = x ^ (x >> 16)
    x = (x * _C1) & MASK32
    x = x ^ (x >> 15)
    x = (x * _C2) & MASK32
    x = x ^ (x >> 16)
    return x


def derive_key(*parts: int) -> int:
    """Fold integers into one 32-bit key (a chain of hashes)."""
    h = 0x9E3779B9
    for p in parts:
        h = _mix32_int(h ^ _mix32_int(int(p) & MASK32) ^ ((int(p) >> 32) & MASK32))
    return h


def _uniform32(idx: torch.Tensor, key: int) -> torch.Tensor:
    return _mix32(idx ^ key)


def _normal(idx: torch.Tensor, key: int) -> torch.Tensor:
    """Irwin-Hall(12) approximation of N(0,1), exact in float64 on any device."""
    acc = torch.zeros_like(idx)
    for i in range(6):
        h = _uniform32(idx, derive_key(key, i))
        acc = acc + (h & 0xFFFF) + (h >> 16)
    # sum of twelve (u + 0.5) / 65536 terms, each with mean exactly 1/2
    return (acc + 6).to(torch.float64) / 65536.0 - 6.0


def _reflect(v: int, span: int) -> int:
    """Position v folded into [0, span] by reflection at both ends."""
    if span <= 0:
        return 0
    period = 2 * span
    m = v % period
    return period - m if m > span else m


@dataclass(frozen=True)
class Box:
    size: int
    x0: int
    y0: int
    vx: int
    vy: int


@dataclass(frozen=True)
class StreamSpec:
    width: int
    height: int
    rgb: bool = True
    depth: bool = True
    n_boxes: int = 1
    box_min: int = 20
    box_max: int = 20
    speed_min: int = 2
    speed_max: int = 2
    hole_p: float = 0.02
    gain_ramp: Optional[Tuple[int, int, float, float]] = None  # (t0, t1, g_lo, g_hi)
    sigma_c: float = 2.0          # colour noise std (variance 4)
    sigma_d: float = math.sqrt(10.0)  # depth noise std (variance 10)
    depth_bg: int = 2000
    depth_box: int = 1200
    colour_box: int = 200
    seed: int = 211014934
    index: int = 0

    @property
    def npix(self) -> int:
        return self.width * self.height


class Stream:
    """One synthetic stream; frames are generated on demand, on any torch device."""

    def __init__(self, spec: StreamSpec):
        self.spec = spec
        rng = np.random.default_rng([spec.seed & MASK32, spec.index, 0x5EED])
        dirs = [(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1)]
        boxes = []
        for _ in range(spec.n_boxes):
            size = int(rng.integers(spec.box_min, spec.box_max + 1))
            size = max(1, min(size, spec.width, spec.height))
            x0 = int(rng.integers(0, spec.width - size + 1))
            y0 = int(rng.integers(0, spec.height - size + 1))
            d = dirs[int(rng.integers(0, 8))]
            s = int(rng.integers(spec.speed_min, spec.speed_max + 1))
            boxes.append(Box(size, x0, y0, d[0] * s, d[1] * s))
        self.boxes: List[Box] = boxes
        self._bg_cache = {}

    # ---- scene geometry (host, tiny) -------------------------------------------------
    def box_positions(self, t: int) -> List[Tuple[int, int, int]]:
        sp = self.spec
        out = []
        for b in self.boxes:
            x = _reflect(b.x0 + b.vx * t, sp.width - b.size)
            y = _reflect(b.y0 + b.vy * t, sp.height - b.size)
            out.append((x, y, b.size))
        return out

    def gain(self, t: int) -> float:
        g = self.spec.gain_ramp
        if g is None:
            return 1.0
        t0, t1, lo, hi = g
        if t <= t0:
            return float(lo)
        if t >= t1:
            return float(hi)
        return float(lo + (hi - lo) * (t - t0) / (t1 - t0))

    def _pix(self, device, pix: Optional[torch.Tensor]) -> torch.Tensor:
        if pix is None:
            return torch.arange(self.spec.npix, dtype=torch.int64, device=device)
        return pix.to(device=device, dtype=torch.int64)

    def truth(self, t: int, device="cpu", pix: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Ground-truth foreground: the union of the box footprints (bool, per pixel)."""
        idx = self._pix(device, pix)
        W = self.spec.width
        xs, ys = idx % W, idx // W
        fg = torch.zeros(idx.shape, dtype=torch.bool, device=idx.device)
        for (x, y, s) in self.box_positions(t):
            fg |= (xs >= x) & (xs < x + s) & (ys >= y) & (ys < y + s)
        return fg

    def _box_id(self, t: int, idx: torch.Tensor) -> torch.Tensor:
        """Index+1 of the topmost box covering each pixel, 0 for background."""
        W = self.spec.width
        xs, ys = idx % W, idx // W
        bid = torch.zeros(idx.shape, dtype=torch.int64, device=idx.device)
        for i, (x, y, s) in enumerate(self.box_positions(t)):
            inside = (xs >= x) & (xs < x + s) & (ys >= y) & (ys < y + s)
            bid = torch.where(inside, torch.full_like(bid, i + 1), bid)
        return bid

    # ---- frames ------------------------------------------------------------------------
    def colour_background(self, device="cpu", pix: Optional[torch.Tensor] = None) -> torch.Tensor:
        """(n, 3) int64 background colour, U{0..255} per channel."""
        idx = self._pix(device, pix)
        sp = self.spec
        chans = [(_uniform32(idx, derive_key(sp.seed, sp.index, _TAG_BG, c)) & 0xFF) for c in range(3)]
        return torch.stack(chans, dim=1)

    def rgb(self, t: int, device="cpu", pix: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Colour frame t as uint8: (H, W, 3) HWC interleaved, or (n, 3) for a pixel subset."""
        sp = self.spec
        if not sp.rgb:
            raise ValueError("stream has no colour modality")
        idx = self._pix(device, pix)
        bg = self.colour_background(device, idx)
        bid = self._box_id(t, idx)
        g = self.gain(t)
        out = []
        for c in range(3):
            scene = torch.where(bid > 0, torch.full_like(bg[:, c], sp.colour_box), bg[:, c]).to(torch.float64)
            z = _normal(idx, derive_key(sp.seed, sp.index, _TAG_NOISE_C, t, c))
            v = scene * g
            v = v + z * sp.sigma_c
            v = torch.clamp(torch.round(v), 0.0, 255.0)
            out.append(v.to(torch.uint8))
        f = torch.stack(out, dim=1)
        if pix is None:
            f = f.reshape(sp.height, sp.width, 3)
        return f

    def depth(self, t: int, device="cpu", pix: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Depth frame t in mm as uint16: (H, W), or (n,) for a pixel subset; 0 = hole."""
        sp = self.spec
        if not sp.depth:
            raise ValueError("stream has no depth modality")
        idx = self._pix(device, pix)
        bid = self._box_id(t, idx)
        scene = torch.where(bid > 0, torch.full_like(bid, sp.depth_box),
                            torch.full_like(bid, sp.depth_bg)).to(torch.float64)
        z = _normal(idx, derive_key(sp.seed, sp.index, _TAG_NOISE_D, t))
        v = scene + z * sp.sigma_d
        v = torch.clamp(torch.round(v), 1.0, 65535.0).to(torch.int64)
        if sp.hole_p > 0:
            thr = int(round(sp.hole_p * 2.0 ** 32))
            hole = _uniform32(idx, derive_key(sp.seed, sp.index, _TAG_HOLE, t)) < thr
            v = torch.where(hole, torch.zeros_like(v), v)
        f = v.to(torch.int32).to(torch.uint16)
        if pix is None:
            f = f.reshape(sp.height, sp.width)
        return f


# ---- mixture parameters and workload presets ------------------------------------------

@dataclass(frozen=True)
class MixtureSettings:
    """Method parameters shared by every preset (the paper's M, k, alpha, T; Sec. III.A)."""
    M: int = 5
    alpha: float = 0.01
    k: float = 2.5
    T: float = 0.7
    sigma0_rgb: float = 30.0
    sigma0_depth: float = 50.0
    var_min_rgb: float = 9.0      # (0.1 * sigma0)^2
    var_min_depth: float = 25.0
    w_init: float = 0.01          # = alpha
    hole_skip: bool = True


@dataclass
class Workload:
    name: str
    streams: List[StreamSpec]
    frames: int
    mix: MixtureSettings
    state_dtype: str = "f32"
    notes: str = ""

    @property
    def pixel_updates_per_frame(self) -> int:
        return sum(s.npix * (int(s.rgb) + int(s.depth)) for s in self.streams)


_BASE_SEED = 211014934


def _plain_small(seed: int, index: int = 0) -> StreamSpec:
    return StreamSpec(160, 120, True, True, n_boxes=1, box_min=20, box_max=20,
                      speed_min=2, speed_max=2, hole_p=0.02, gain_ramp=None,
                      seed=seed, index=index)


def _vga_like(w: int, h: int, rgb: bool, depth: bool, seed: int, index: int) -> StreamSpec:
    return StreamSpec(w, h, rgb, depth, n_boxes=3, box_min=40, box_max=120,
                      speed_min=1, speed_max=4, hole_p=0.05, gain_ramp=(100, 150, 0.6, 1.2),
                      seed=seed, index=index)


def _mixed_streams(seed: int, counts: Sequence[int]) -> List[StreamSpec]:
    n320, n640, n512, n1080 = counts
    specs: List[StreamSpec] = []
    i = 0
    for (n, w, h, rgb, dep) in ((n320, 320, 240, True, True), (n640, 640, 480, True, True),
                                (n512, 512, 424, False, True), (n1080, 1920, 1080, True, False)):
        for _ in range(n):
            specs.append(_vga_like(w, h, rgb, dep, seed, i))
            i += 1
    return specs


def workload(name: str) -> Workload:
    """Named presets.

    plain-160x120 : 1 stream 160x120 RGB+D, M=3, 60 frames (small parity case)
    plain-640x480 : 1 stream 640x480 RGB+D, M=5, 300 frames, gain ramp, 3 boxes, 5% holes
    batch-64      : 16x320x240 + 32x640x480 RGB+D, 8x512x424 depth, 8x1920x1080 colour; 120 frames
    precision-256 : 256x640x480 RGB+D, M=5, 120 frames, reduced-precision state
    serve-1024    : 1024-stream mix (batch-64 x 16) for the serving loop
    """
    if name == "plain-160x120":
        return Workload(name, [_plain_small(_BASE_SEED + 0)], 60, MixtureSettings(M=3))
    if name == "plain-640x480":
        return Workload(name, [_vga_like(640, 480, True, True, _BASE_SEED + 1, 0)], 300, MixtureSettings(M=5))
    if name == "batch-64":
        return Workload(name, _mixed_streams(_BASE_SEED + 2, (16, 32, 8, 8)), 120, MixtureSettings(M=5))
    if name == "precision-256":
        specs = [_vga_like(640, 480, True, True, _BASE_SEED + 3, i) for i in range(256)]
        return Workload(name, specs, 120, MixtureSettings(M=5), state_dtype="f16")
    if name == "serve-1024":
        return Workload(name, _mixed_streams(_BASE_SEED + 4, (256, 512, 128, 128)), 1800,
                        MixtureSettings(M=5), state_dtype="f16")
    raise KeyError(name)


WORKLOADS = ("plain-160x120", "plain-640x480", "batch-64", "precision-256", "serve-1024")

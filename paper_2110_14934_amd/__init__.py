"""MI355X-native RGB-D mixture-of-Gaussians background segmentation.

The per-frame path runs in the HIP library ``libgmm.so`` (C ABI in include/gmm.h); this
package holds its ctypes binding (``_abi``, same names as the C functions), a small
convenience wrapper (``Segmenter``), the build step and the seeded synthetic input
generator (``synth``). Nothing here computes the method on the CPU: if the library is
missing, every call raises.
"""
from __future__ import annotations

from . import _abi
from ._abi import (GMM_RGB, GMM_DEPTH, GMM_F32, GMM_F16, GMM_BF16, GMM_HOLE_SKIP, GMM_HOLE_AS_VALUE,
                   GMM_SEPARATE, GMM_AUGMENTED, GMM_RHO_ALPHA, GMM_RHO_DENSITY, gmm_apply_frame_augmented,
                   GmmError, gmm_config, gmm_config_default, gmm_create, gmm_destroy, gmm_apply_frame,
                   gmm_fuse, gmm_apply_frame_fused, gmm_last_error, gmm_state_bytes, gmm_state_size,
                   gmm_read_state, gmm_write_state, gmm_version, stream_io, gmm_batch_create,
                   gmm_batch_destroy, gmm_batch_set_tuning, gmm_batch_get_tuning, gmm_batch_set_frames,
                   gmm_batch_run, gmm_batch_apply, gmm_batch_autotune, gmm_batch_tiles,
                   gmm_state_save, gmm_state_restore, gmm_device_copy)


def mask_words(npix: int) -> int:
    """Number of uint64 words of a bit-packed mask of npix pixels."""
    return (npix + 63) // 64


RHO_MODES = {"alpha": GMM_RHO_ALPHA, "density": GMM_RHO_DENSITY}


class Segmenter:
    """One stream's handle plus its output masks (torch tensors on the handle's device).

    ``rho`` = "alpha" | "density" picks the rate of the mean and variance updates. ``augmented``
    builds the four-channel variant (both modalities, one mixture, mask in ``fg``) used by
    ``apply_augmented``."""

    def __init__(self, width: int, height: int, modalities: int = GMM_RGB | GMM_DEPTH, M: int = 5,
                 state_dtype: str = "f32", device: int = 0, rho: str = "alpha", augmented: bool = False,
                 **params):
        import torch
        self.width, self.height, self.M = width, height, M
        self.modalities = modalities
        self.npix = width * height
        self.augmented = augmented
        self.cfg = gmm_config_default(width, height, modalities, M, state_dtype=_abi.DTYPES[state_dtype],
                                      device=device, rho_mode=RHO_MODES[rho],
                                      variant=GMM_AUGMENTED if augmented else GMM_SEPARATE, **params)
        self.handle = gmm_create(self.cfg)
        dev = torch.device("cuda", device)
        n = mask_words(self.npix)
        if augmented:
            self.fg = torch.zeros(n, dtype=torch.int64, device=dev)
            self.fg_rgb = self.fg_depth = self.fused = None
            return
        self.fg_rgb = torch.zeros(n, dtype=torch.int64, device=dev) if modalities & GMM_RGB else None
        self.fg_depth = torch.zeros(n, dtype=torch.int64, device=dev) if modalities & GMM_DEPTH else None
        both = (modalities & GMM_RGB) and (modalities & GMM_DEPTH)
        self.fused = torch.zeros(n, dtype=torch.int64, device=dev) if both else None

    def _pitches(self, rgb, depth):
        rp = rgb.stride(0) * rgb.element_size() if rgb is not None else 0
        dp = depth.stride(0) * depth.element_size() if depth is not None else 0
        return rp, dp

    def apply(self, rgb=None, depth=None, stream=None):
        rp, dp = self._pitches(rgb, depth)
        gmm_apply_frame(self.handle, rgb, rp, depth, dp, self.fg_rgb, self.fg_depth, stream)
        return self.fg_rgb, self.fg_depth

    def apply_fused(self, rgb, depth, stream=None):
        rp, dp = self._pitches(rgb, depth)
        gmm_apply_frame_fused(self.handle, rgb, rp, depth, dp, self.fg_rgb, self.fg_depth, self.fused, stream)
        return self.fg_rgb, self.fg_depth, self.fused

    def apply_augmented(self, rgb, depth, stream=None):
        rp, dp = self._pitches(rgb, depth)
        gmm_apply_frame_augmented(self.handle, rgb, rp, depth, dp, self.fg, stream)
        return self.fg

    def fuse(self, fg_rgb, fg_depth, stream=None):
        gmm_fuse(self.handle, fg_rgb, fg_depth, self.fused, stream)
        return self.fused

    def read_state(self, stream=None):
        return gmm_read_state(self.handle, stream)

    def write_state(self, state, stream=None):
        gmm_write_state(self.handle, state, stream)

    def state_bytes(self) -> int:
        return gmm_state_bytes(self.handle)

    def save_state(self, device_dst, stream=None):
        """Device-side snapshot of the state into a caller-owned device tensor."""
        gmm_state_save(self.handle, device_dst, stream)

    def restore_state(self, device_src, stream=None):
        gmm_state_restore(self.handle, device_src, stream)

    def close(self):
        if self.handle is not None:
            gmm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A set of Segmenters advanced together by one persistent launch per frame-set."""

    def __init__(self, segmenters, n_slots: int = 1):
        self.segs = list(segmenters)
        self.handle = gmm_batch_create([s.handle for s in self.segs], n_slots)

    def ios(self, frames, fuse=True):
        """frames: list of (rgb or None, depth or None) per stream, in batch order."""
        out = []
        for seg, (rgb, depth) in zip(self.segs, frames):
            out.append(stream_io(rgb, depth, seg.fg_rgb, seg.fg_depth, seg.fused if fuse else None))
        return out

    def set_frames(self, slot, frames, fuse=True, stream=None):
        gmm_batch_set_frames(self.handle, slot, self.ios(frames, fuse), stream)

    def run(self, slot=0, stream=None):
        gmm_batch_run(self.handle, slot, stream)

    def apply(self, frames, fuse=True, stream=None):
        gmm_batch_apply(self.handle, self.ios(frames, fuse), stream)

    def set_tuning(self, block_threads, tile_pixels, blocks_per_cu):
        gmm_batch_set_tuning(self.handle, block_threads, tile_pixels, blocks_per_cu)

    def tuning(self):
        return gmm_batch_get_tuning(self.handle)

    def autotune(self, slot=0, stream=None):
        return gmm_batch_autotune(self.handle, slot, stream)

    def close(self):
        if self.handle is not None:
            gmm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""ctypes binding of the C ABI in include/gmm.h (argument marshalling only).

Every function keeps the C name. Device buffers are passed as torch tensors (their
``data_ptr()``), streams as ``torch.cuda.Stream`` (or None for torch's current stream).
A non-OK status raises ``GmmError`` carrying ``gmm_last_error()``. There is no fallback:
if the library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmm.so")

GMM_OK = 0
GMM_ERR_INVALID_ARG = -1
GMM_ERR_OUT_OF_MEMORY = -2
GMM_ERR_DEVICE = -3
GMM_ERR_STATE = -4
GMM_ERR_UNSUPPORTED = -5

GMM_RGB = 1
GMM_DEPTH = 2
GMM_F32, GMM_F16, GMM_BF16 = 0, 1, 2
GMM_HOLE_SKIP, GMM_HOLE_AS_VALUE = 0, 1
GMM_SEPARATE, GMM_AUGMENTED = 0, 1
GMM_RHO_ALPHA, GMM_RHO_DENSITY = 0, 1

DTYPES = {"f32": GMM_F32, "f16": GMM_F16, "bf16": GMM_BF16}

# every symbol the header declares
EXPORTS = (
    "gmm_config_default", "gmm_create", "gmm_destroy", "gmm_apply_frame", "gmm_fuse",
    "gmm_apply_frame_fused", "gmm_last_error", "gmm_state_bytes", "gmm_state_size",
    "gmm_read_state", "gmm_write_state", "gmm_version",
    "gmm_batch_create", "gmm_batch_destroy", "gmm_batch_set_tuning", "gmm_batch_get_tuning",
    "gmm_batch_set_frames", "gmm_batch_run", "gmm_batch_apply", "gmm_batch_autotune", "gmm_batch_tiles",
    "gmm_mask_confusion",
    "gmm_exec_create", "gmm_exec_destroy", "gmm_exec_set_tuning", "gmm_exec_attach", "gmm_exec_detach",
    "gmm_exec_launch", "gmm_exec_poll", "gmm_exec_drain", "gmm_exec_now",
    "gmm_exec_stream_bytes", "gmm_exec_create_stream", "gmm_exec_destroy_stream",
    "gmm_set_traffic_record", "gmm_apply_frame_augmented",
    "gmm_state_save", "gmm_state_restore", "gmm_device_copy", "gmm_batch_apply_static",
)
GMM_STATIC_MAX_STREAMS = 1024


class GmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gmm status {status}: {msg}")
        self.status = status


class gmm_config(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("modalities", ctypes.c_int32), ("M", ctypes.c_int32),
        ("alpha", ctypes.c_float), ("k", ctypes.c_float), ("T", ctypes.c_float),
        ("sigma0", ctypes.c_float * 2), ("var_min", ctypes.c_float * 2),
        ("w_init", ctypes.c_float),
        ("hole_policy", ctypes.c_int32), ("state_dtype", ctypes.c_int32), ("device", ctypes.c_int32),
        ("variant", ctypes.c_int32), ("rho_mode", ctypes.c_int32),
    ]


class gmm_stream_io(ctypes.Structure):
    _fields_ = [
        ("rgb", ctypes.c_void_p), ("rgb_pitch_bytes", ctypes.c_int64),
        ("depth", ctypes.c_void_p), ("depth_pitch_bytes", ctypes.c_int64),
        ("fg_rgb", ctypes.c_void_p), ("fg_depth", ctypes.c_void_p), ("fused", ctypes.c_void_p),
    ]


class gmm_batch_tuning(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_int32), ("tile_pixels", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32)]

    def as_tuple(self):
        return (self.block_threads, self.tile_pixels, self.blocks_per_cu)


class gmm_exec_item(ctypes.Structure):
    _fields_ = [
        ("handle", ctypes.c_void_p), ("host_rgb", ctypes.c_void_p), ("host_depth", ctypes.c_void_p),
        ("host_fg_rgb", ctypes.c_void_p), ("host_fg_depth", ctypes.c_void_p), ("host_fused", ctypes.c_void_p),
    ]


_lib = None


def load(path: Optional[str] = None) -> ctypes.CDLL:
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(p)
    H = ctypes.c_void_p
    vp, i64, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    sig = {
        "gmm_config_default": (st, [ctypes.POINTER(gmm_config), ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32]),
        "gmm_create": (st, [ctypes.POINTER(gmm_config), ctypes.POINTER(H)]),
        "gmm_destroy": (st, [H]),
        "gmm_apply_frame": (st, [H, vp, i64, vp, i64, vp, vp, vp]),
        "gmm_fuse": (st, [H, vp, vp, vp, vp]),
        "gmm_apply_frame_fused": (st, [H, vp, i64, vp, i64, vp, vp, vp, vp]),
        "gmm_last_error": (ctypes.c_char_p, []),
        "gmm_state_bytes": (st, [H, ctypes.POINTER(ctypes.c_size_t)]),
        "gmm_state_size": (st, [H, ctypes.POINTER(ctypes.c_size_t)]),
        "gmm_read_state": (st, [H, vp, vp]),
        "gmm_write_state": (st, [H, vp, vp]),
        "gmm_version": (ctypes.c_int32, []),
        "gmm_batch_create": (st, [ctypes.POINTER(H), ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(H)]),
        "gmm_batch_destroy": (st, [H]),
        "gmm_batch_set_tuning": (st, [H, ctypes.POINTER(gmm_batch_tuning)]),
        "gmm_batch_get_tuning": (st, [H, ctypes.POINTER(gmm_batch_tuning)]),
        "gmm_batch_set_frames": (st, [H, ctypes.c_int32, ctypes.POINTER(gmm_stream_io), vp]),
        "gmm_batch_run": (st, [H, ctypes.c_int32, vp]),
        "gmm_batch_apply": (st, [H, ctypes.POINTER(gmm_stream_io), vp]),
        "gmm_batch_autotune": (st, [H, ctypes.c_int32, vp, ctypes.POINTER(gmm_batch_tuning),
                                    ctypes.POINTER(ctypes.c_double)]),
        "gmm_batch_tiles": (st, [H, ctypes.POINTER(ctypes.c_uint32)]),
        "gmm_mask_confusion": (st, [vp, vp, i64, vp, vp]),
        "gmm_exec_create": (st, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(H)]),
        "gmm_exec_destroy": (st, [H]),
        "gmm_exec_set_tuning": (st, [H, ctypes.POINTER(gmm_batch_tuning)]),
        "gmm_exec_attach": (st, [H, H, ctypes.POINTER(ctypes.c_size_t)]),
        "gmm_exec_detach": (st, [H, H]),
        "gmm_exec_launch": (st, [H, ctypes.POINTER(gmm_exec_item), ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
        "gmm_exec_poll": (st, [H, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_int32)]),
        "gmm_exec_drain": (st, [H]),
        "gmm_exec_now": (ctypes.c_double, []),
        "gmm_exec_stream_bytes": (st, [ctypes.POINTER(gmm_config), ctypes.POINTER(ctypes.c_size_t)]),
        "gmm_exec_create_stream": (st, [H, ctypes.POINTER(gmm_config), vp, ctypes.c_size_t, ctypes.POINTER(H)]),
        "gmm_exec_destroy_stream": (st, [H, H]),
        "gmm_set_traffic_record": (st, [H, vp]),
        "gmm_apply_frame_augmented": (st, [H, vp, i64, vp, i64, vp, vp]),
        "gmm_state_save": (st, [H, vp, vp]),
        "gmm_state_restore": (st, [H, vp, vp]),
        "gmm_device_copy": (st, [vp, vp, ctypes.c_size_t, vp]),
        "gmm_batch_apply_static": (st, [ctypes.POINTER(H), ctypes.c_int32, ctypes.POINTER(gmm_stream_io),
                                        ctypes.POINTER(gmm_batch_tuning), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(status: int):
    if status != GMM_OK:
        msg = load().gmm_last_error()
        raise GmmError(status, msg.decode() if msg else "")


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def gmm_config_default(width: int, height: int, modalities: int = GMM_RGB | GMM_DEPTH, M: int = 5,
                       **overrides) -> gmm_config:
    cfg = gmm_config()
    _check(load().gmm_config_default(ctypes.byref(cfg), width, height, modalities, M))
    for k, v in overrides.items():
        if k in ("sigma0", "var_min"):
            getattr(cfg, k)[0], getattr(cfg, k)[1] = float(v[0]), float(v[1])
        else:
            setattr(cfg, k, v)
    return cfg


def gmm_create(cfg: gmm_config) -> int:
    h = ctypes.c_void_p()
    _check(load().gmm_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def gmm_destroy(h: Optional[int]):
    _check(load().gmm_destroy(h))


def gmm_apply_frame(h, rgb, rgb_pitch, depth, depth_pitch, fg_rgb, fg_depth, stream=None):
    _check(load().gmm_apply_frame(h, _ptr(rgb), rgb_pitch, _ptr(depth), depth_pitch, _ptr(fg_rgb),
                                  _ptr(fg_depth), _stream(stream)))


def gmm_fuse(h, fg_rgb, fg_depth, fused, stream=None):
    _check(load().gmm_fuse(h, _ptr(fg_rgb), _ptr(fg_depth), _ptr(fused), _stream(stream)))


def gmm_apply_frame_fused(h, rgb, rgb_pitch, depth, depth_pitch, fg_rgb, fg_depth, fused, stream=None):
    _check(load().gmm_apply_frame_fused(h, _ptr(rgb), rgb_pitch, _ptr(depth), depth_pitch, _ptr(fg_rgb),
                                        _ptr(fg_depth), _ptr(fused), _stream(stream)))


def gmm_apply_frame_augmented(h, rgb, rgb_pitch, depth, depth_pitch, fg, stream=None):
    _check(load().gmm_apply_frame_augmented(h, _ptr(rgb), rgb_pitch, _ptr(depth), depth_pitch, _ptr(fg),
                                            _stream(stream)))


def gmm_last_error() -> str:
    m = load().gmm_last_error()
    return m.decode() if m else ""


def gmm_state_bytes(h) -> int:
    n = ctypes.c_size_t()
    _check(load().gmm_state_bytes(h, ctypes.byref(n)))
    return n.value


def gmm_state_size(h) -> int:
    n = ctypes.c_size_t()
    _check(load().gmm_state_size(h, ctypes.byref(n)))
    return n.value


def gmm_read_state(h, stream=None):
    """Returns the canonical float64 state as a NumPy array."""
    import numpy as np
    out = np.empty(gmm_state_size(h), dtype=np.float64)
    _check(load().gmm_read_state(h, out.ctypes.data, _stream(stream)))
    return out


def gmm_write_state(h, state, stream=None):
    import numpy as np
    arr = np.ascontiguousarray(state, dtype=np.float64)
    if arr.size != gmm_state_size(h):
        raise ValueError(f"state has {arr.size} values, handle needs {gmm_state_size(h)}")
    _check(load().gmm_write_state(h, arr.ctypes.data, _stream(stream)))


def gmm_state_save(h, device_dst, stream=None):
    """device_dst: a device tensor of at least gmm_state_bytes(h) bytes."""
    if device_dst.numel() * device_dst.element_size() < gmm_state_bytes(h):
        raise ValueError("snapshot buffer smaller than the state")
    _check(load().gmm_state_save(h, _ptr(device_dst), _stream(stream)))


def gmm_state_restore(h, device_src, stream=None):
    if device_src.numel() * device_src.element_size() < gmm_state_bytes(h):
        raise ValueError("snapshot buffer smaller than the state")
    _check(load().gmm_state_restore(h, _ptr(device_src), _stream(stream)))


def gmm_device_copy(dst, src, nbytes: int, stream=None):
    """Copy nbytes between two device tensors with the library's streaming copy kernel."""
    for t in (dst, src):
        if t.numel() * t.element_size() < nbytes:
            raise ValueError("tensor smaller than the copy")
    _check(load().gmm_device_copy(_ptr(dst), _ptr(src), nbytes, _stream(stream)))


def gmm_version() -> int:
    return load().gmm_version()


# ---- batched path ------------------------------------------------------------------------

def stream_io(rgb=None, depth=None, fg_rgb=None, fg_depth=None, fused=None) -> gmm_stream_io:
    """One stream's entry of a batched call; pitches are taken from the tensors' row strides."""
    io = gmm_stream_io()
    io.rgb = _ptr(rgb)
    io.rgb_pitch_bytes = rgb.stride(0) * rgb.element_size() if rgb is not None else 0
    io.depth = _ptr(depth)
    io.depth_pitch_bytes = depth.stride(0) * depth.element_size() if depth is not None else 0
    io.fg_rgb = _ptr(fg_rgb)
    io.fg_depth = _ptr(fg_depth)
    io.fused = _ptr(fused)
    return io


def gmm_batch_create(handles, n_slots: int = 1) -> int:
    arr = (ctypes.c_void_p * len(handles))(*handles)
    b = ctypes.c_void_p()
    _check(load().gmm_batch_create(arr, len(handles), n_slots, ctypes.byref(b)))
    return b.value


def gmm_batch_destroy(b):
    _check(load().gmm_batch_destroy(b))


def gmm_batch_set_tuning(b, block_threads: int, tile_pixels: int, blocks_per_cu: int):
    t = gmm_batch_tuning(block_threads, tile_pixels, blocks_per_cu)
    _check(load().gmm_batch_set_tuning(b, ctypes.byref(t)))


def gmm_batch_get_tuning(b):
    t = gmm_batch_tuning()
    _check(load().gmm_batch_get_tuning(b, ctypes.byref(t)))
    return t.as_tuple()


def _io_array(ios):
    return (gmm_stream_io * len(ios))(*ios)


def gmm_batch_set_frames(b, slot: int, ios, stream=None):
    _check(load().gmm_batch_set_frames(b, slot, _io_array(ios), _stream(stream)))


def gmm_batch_run(b, slot: int = 0, stream=None):
    _check(load().gmm_batch_run(b, slot, _stream(stream)))


def gmm_batch_apply(b, ios, stream=None):
    _check(load().gmm_batch_apply(b, _io_array(ios), _stream(stream)))


def gmm_batch_autotune(b, slot: int = 0, stream=None):
    """Returns ((block_threads, tile_pixels, blocks_per_cu), ms per launch)."""
    t = gmm_batch_tuning()
    ms = ctypes.c_double()
    _check(load().gmm_batch_autotune(b, slot, _stream(stream), ctypes.byref(t), ctypes.byref(ms)))
    return t.as_tuple(), ms.value


def gmm_batch_apply_static(handles, ios, tuning=None, stream=None):
    """One batched launch over `handles` with the library's static tables (no allocation).
    tuning: (block_threads, tile_pixels, blocks_per_cu) or None for the default."""
    hs = (ctypes.c_void_p * len(handles))(*handles)
    arr = (gmm_stream_io * len(ios))(*ios) if ios else None
    t = None if tuning is None else ctypes.byref(gmm_batch_tuning(*tuning))
    _check(load().gmm_batch_apply_static(hs, len(handles), arr, t, _stream(stream)))


def gmm_batch_tiles(b) -> int:
    n = ctypes.c_uint32()
    _check(load().gmm_batch_tiles(b, ctypes.byref(n)))
    return n.value


def gmm_mask_confusion(pred, truth, npix: int, counts, stream=None):
    """TP, FP, TN, FN of two bit-packed device masks into `counts` (4 int64, device)."""
    _check(load().gmm_mask_confusion(_ptr(pred), _ptr(truth), npix, _ptr(counts), _stream(stream)))


# ---- serving executor --------------------------------------------------------------------

def gmm_exec_create(device: int = 0, ring: int = 4) -> int:
    x = ctypes.c_void_p()
    _check(load().gmm_exec_create(device, ring, ctypes.byref(x)))
    return x.value


def gmm_exec_destroy(x):
    _check(load().gmm_exec_destroy(x))


def gmm_exec_set_tuning(x, block_threads: int, tile_pixels: int, blocks_per_cu: int):
    t = gmm_batch_tuning(block_threads, tile_pixels, blocks_per_cu)
    _check(load().gmm_exec_set_tuning(x, ctypes.byref(t)))


def gmm_exec_attach(x, h) -> int:
    n = ctypes.c_size_t()
    _check(load().gmm_exec_attach(x, h, ctypes.byref(n)))
    return n.value


def gmm_exec_detach(x, h):
    _check(load().gmm_exec_detach(x, h))


def gmm_exec_launch(x, items) -> int:
    """items: list of gmm_exec_item (host pointers as ints)."""
    arr = (gmm_exec_item * len(items))(*items)
    tid = ctypes.c_uint64()
    _check(load().gmm_exec_launch(x, arr, len(items), ctypes.byref(tid)))
    return tid.value


def gmm_exec_poll(x, cap: int = 256):
    """[(tick id, completion time)] of ticks completed since the last poll, in launch order."""
    ids = (ctypes.c_uint64 * cap)()
    ts = (ctypes.c_double * cap)()
    n = ctypes.c_int32()
    _check(load().gmm_exec_poll(x, ids, ts, cap, ctypes.byref(n)))
    return [(ids[i], ts[i]) for i in range(n.value)]


def gmm_exec_drain(x):
    _check(load().gmm_exec_drain(x))


def gmm_exec_now() -> float:
    return load().gmm_exec_now()


def gmm_exec_stream_bytes(cfg: gmm_config) -> int:
    n = ctypes.c_size_t()
    _check(load().gmm_exec_stream_bytes(ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


def gmm_exec_create_stream(x, cfg: gmm_config, mem_ptr: int, nbytes: int) -> int:
    h = ctypes.c_void_p()
    _check(load().gmm_exec_create_stream(x, ctypes.byref(cfg), mem_ptr, nbytes, ctypes.byref(h)))
    return h.value


def gmm_exec_destroy_stream(x, h):
    _check(load().gmm_exec_destroy_stream(x, h))


def gmm_set_traffic_record(h, wave_bytes):
    """wave_bytes: device int64 tensor of ceil(npix/64) entries (accumulated into), or None."""
    _check(load().gmm_set_traffic_record(h, _ptr(wave_bytes)))

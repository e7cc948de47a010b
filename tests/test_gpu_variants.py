"""Parity of the two ablation variants with the FP64 oracle, through the C ABI:

  * the density rate of the mean and variance updates, rho = alpha N(x | mu, var I), the rate
    of the paper's reference [6] (Stauffer and Grimson), on both separate models and List 1;
  * the four-channel augmentation (R, G, B, D8) of Sec. III.B, the design the paper rejects.

Same bars as the method's own parity tests: lockstep parameters within 1e-4 relative and masks
equal except at near-threshold decisions; free run with every disagreement explained by such a
decision and at most 1e-4 of pixel-frames differing.
"""
import sys
from dataclasses import replace

import numpy as np
import pytest
import torch

from oracle import AugmentedOracle, MixParams, MixtureOracle, round_to_storage
from paper_2110_14934_amd import GMM_RGB, GMM_DEPTH, GmmError, Segmenter, Batch, _abi
from paper_2110_14934_amd.synth import Stream, StreamSpec, workload
from tests.parity import (unpack_mask, excused, param_mismatch, aug_to_canonical, aug_from_canonical,
                          WEIGHT_MARGIN_FREE, KEY_GAP_FREE, MASK_FRACTION)
from tests.test_gpu_parity import _lockstep, _ulp_mismatch, seg_kwargs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ---- density rate --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_lockstep_density_rate(dtype):
    wl = workload("plain-160x120")
    spec = StreamSpec(97, 61, n_boxes=2, box_min=8, box_max=20, hole_p=0.05, seed=91)
    say(f"density rate lockstep {dtype} 97x61 M={wl.mix.M}")
    _lockstep(spec, wl.mix, 24, dtype=dtype, rho="density")


def test_lockstep_density_rate_small_variances():
    # variances near their floor make rho largest (colour: alpha (2 pi 9)^-1.5 ~ 2e-5 at
    # alpha = 0.01); a large alpha and small floors push it to ~1e-2, where the increment form of
    # the update matters
    wl = workload("plain-160x120")
    mix = replace(wl.mix, alpha=0.5, var_min_rgb=0.5, var_min_depth=0.5, sigma0_rgb=3.0, sigma0_depth=4.0)
    spec = StreamSpec(65, 33, n_boxes=1, box_min=8, box_max=12, hole_p=0.02, seed=92, sigma_c=0.7,
                      sigma_d=0.8)
    say("density rate lockstep, small variances")
    _lockstep(spec, mix, 16, rho="density")


def test_free_run_density_rate():
    wl = workload("plain-160x120")
    spec, mix = wl.streams[0], wl.mix
    st = Stream(spec)
    n = spec.npix
    kw = seg_kwargs(mix)
    seg = Segmenter(spec.width, spec.height, GMM_RGB | GMM_DEPTH, mix.M, rho="density", **kw)
    col = MixtureOracle(MixParams(mix.M, mix.alpha, mix.k, mix.T, mix.sigma0_rgb, mix.var_min_rgb, mix.w_init,
                                  rho="density"), 3, n)
    dep = MixtureOracle(MixParams(mix.M, mix.alpha, mix.k, mix.T, mix.sigma0_depth, mix.var_min_depth,
                                  mix.w_init, hole_skip=mix.hole_skip, rho="density"), 1, n)
    risky_c = np.zeros(n, bool)
    risky_d = np.zeros(n, bool)
    dis = 0
    try:
        for t in range(wl.frames):
            rgb, depth = st.rgb(t), st.depth(t)
            ic = col.step(rgb.reshape(-1, 3).numpy())
            idd = dep.step(depth.reshape(-1).numpy())
            risky_c |= excused(ic, WEIGHT_MARGIN_FREE, KEY_GAP_FREE)
            risky_d |= excused(idd, WEIGHT_MARGIN_FREE, KEY_GAP_FREE)
            seg.apply_fused(rgb.to(DEV), depth.to(DEV))
            gc = unpack_mask(seg.fg_rgb, n)
            gd = unpack_mask(seg.fg_depth, n)
            assert not np.any((gc != ic.fg) & ~risky_c), t
            assert not np.any((gd != idd.fg) & ~risky_d), t
            dis += int((gc != ic.fg).sum() + (gd != idd.fg).sum())
        from tests.parity import from_canonical, oracle_state
        got = from_canonical(seg.read_state(), mix.M, n, True, True)
        assert not np.any(param_mismatch(got["rgb"], oracle_state(col)) & ~risky_c)
        assert not np.any(param_mismatch(got["depth"], oracle_state(dep)) & ~risky_d)
    finally:
        seg.close()
    frac = dis / (2 * n * wl.frames)
    say(f"density free run: disagreement {frac:.2e}")
    assert frac <= MASK_FRACTION


# ---- four-channel augmentation -------------------------------------------------------------

def _aug_params(mix):
    return MixParams(M=mix.M, alpha=mix.alpha, k=mix.k, T=mix.T, sigma0=mix.sigma0_rgb, var_min=mix.var_min_rgb,
                     w_init=mix.w_init, hole_skip=mix.hole_skip)


@pytest.mark.parametrize("w,h,M,dtype,pad", [(97, 61, 5, "f32", 0), (17, 13, 3, "f32", 5), (160, 120, 4, "f16", 0),
                                             (65, 3, 2, "bf16", 3)])
def test_lockstep_augmented(w, h, M, dtype, pad):
    wl = workload("plain-160x120")
    mix = replace(wl.mix, M=M)
    spec = StreamSpec(w, h, n_boxes=2, box_min=4, box_max=20, hole_p=0.05, seed=93)
    st = Stream(spec)
    n = spec.npix
    say(f"augmented lockstep {w}x{h} M={M} {dtype} pad={pad}")
    seg = Segmenter(w, h, GMM_RGB | GMM_DEPTH, M, state_dtype=dtype, augmented=True, **seg_kwargs(mix))
    o = AugmentedOracle(_aug_params(mix), n)
    try:
        for t in range(20):
            rgb, depth = st.rgb(t), st.depth(t)
            flat = round_to_storage(aug_to_canonical(o), dtype)
            seg.write_state(flat)
            o.set_state(*aug_from_canonical(flat, M, n))
            if dtype != "f32":
                o.model.storage = dtype
            info = o.step(rgb.reshape(-1, 3).numpy(), depth.reshape(-1).numpy())
            br = torch.zeros(h, w + pad, 3, dtype=torch.uint8, device=DEV)
            bd = torch.zeros(h, w + pad, dtype=torch.uint16, device=DEV)
            br[:, :w].copy_(rgb.to(DEV))
            bd[:, :w].copy_(depth.to(DEV))
            seg.apply_augmented(br[:, :w], bd[:, :w])
            torch.cuda.synchronize()
            gm = unpack_mask(seg.fg, n)
            ex = excused(info)
            assert not np.any((gm != info.fg) & ~ex), (t, np.flatnonzero((gm != info.fg) & ~ex)[:8])
            got = aug_from_canonical(seg.read_state(), M, n)
            ora = o.get_state()
            bad = (param_mismatch(got, ora) if dtype == "f32" else _ulp_mismatch(got, ora, dtype)) & ~ex
            assert not np.any(bad), (t, np.flatnonzero(bad)[:8])
            assert not np.any(gm[info.hole]), t                     # holes are background
    finally:
        seg.close()


def test_free_run_augmented_full_size_sampled():
    """640x480, M=5, all 300 frames of the VGA clip (gain ramp included) on the GPU; the oracle
    follows 4096 sampled pixels plus the ragged last rows."""
    wl = workload("plain-640x480")
    spec, mix = wl.streams[0], wl.mix
    st = Stream(spec)
    n = spec.npix
    rng = np.random.default_rng(23)
    sample = np.unique(np.concatenate([rng.choice(n, 4096, replace=False), np.arange(n - 700, n)]))
    pix = torch.from_numpy(sample)
    k = sample.size
    seg = Segmenter(spec.width, spec.height, GMM_RGB | GMM_DEPTH, mix.M, augmented=True, **seg_kwargs(mix))
    o = AugmentedOracle(_aug_params(mix), k)
    risky = np.zeros(k, bool)
    dis = 0
    say(f"augmented free run 640x480, {wl.frames} frames, {k} sampled pixels")
    try:
        for t in range(wl.frames):
            seg.apply_augmented(st.rgb(t, device=DEV), st.depth(t, device=DEV))
            info = o.step(st.rgb(t, pix=pix).numpy(), st.depth(t, pix=pix).numpy())
            risky |= excused(info, WEIGHT_MARGIN_FREE, KEY_GAP_FREE)
            gm = unpack_mask(seg.fg, n)[sample]
            assert not np.any((gm != info.fg) & ~risky), t
            dis += int((gm != info.fg).sum())
        got = aug_from_canonical(seg.read_state(), mix.M, n)
        got = tuple(a[..., sample] for a in got)
        assert not np.any(param_mismatch(got, o.get_state()) & ~risky)
    finally:
        seg.close()
    assert dis <= MASK_FRACTION * k * wl.frames + 1, dis


def test_augmented_error_paths():
    aug = Segmenter(64, 48, GMM_RGB | GMM_DEPTH, 3, augmented=True)
    sep = Segmenter(64, 48, GMM_RGB | GMM_DEPTH, 3)
    rgb = torch.zeros(48, 64, 3, dtype=torch.uint8, device=DEV)
    dep = torch.zeros(48, 64, dtype=torch.uint16, device=DEV)
    m = torch.zeros(48, dtype=torch.int64, device=DEV)
    try:
        with pytest.raises(GmmError) as e:
            _abi.gmm_apply_frame(aug.handle, rgb, 192, dep, 128, m, m)
        assert e.value.status == _abi.GMM_ERR_STATE
        with pytest.raises(GmmError) as e:
            _abi.gmm_apply_frame_fused(aug.handle, rgb, 192, dep, 128, m, m, m)
        assert e.value.status == _abi.GMM_ERR_STATE
        with pytest.raises(GmmError) as e:
            _abi.gmm_apply_frame_augmented(sep.handle, rgb, 192, dep, 128, m)
        assert e.value.status == _abi.GMM_ERR_STATE
        with pytest.raises(GmmError) as e:
            _abi.gmm_apply_frame_augmented(aug.handle, rgb, 191, dep, 128, m)
        assert e.value.status == _abi.GMM_ERR_INVALID_ARG
        with pytest.raises(GmmError) as e:
            Batch([aug, sep])
        assert e.value.status == _abi.GMM_ERR_UNSUPPORTED
        x = _abi.gmm_exec_create(0, 2)
        try:
            with pytest.raises(GmmError) as e:
                _abi.gmm_exec_attach(x, aug.handle)
            assert e.value.status == _abi.GMM_ERR_UNSUPPORTED
        finally:
            _abi.gmm_exec_destroy(x)
        assert _abi.gmm_state_size(aug.handle) == 6 * 3 * 64 * 48
        # a frame of holes leaves the initial state as it was
        s0 = aug.read_state()
        aug.apply_augmented(rgb, dep)
        torch.cuda.synchronize()
        assert np.array_equal(aug.read_state(), s0) and int(aug.fg.abs().sum()) == 0
    finally:
        aug.close()
        sep.close()

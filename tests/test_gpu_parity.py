"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on seeded synthetic streams.

Lockstep: every frame both sides start from the oracle's state rounded to the storage type,
take one step, and are compared element by element (parameters within 1e-4 relative; masks
equal except at pixels whose decision was within a small margin of flipping).
Free run: both sides run on their own; every disagreement must be explained by a near-threshold
decision at that pixel (then the pixel is counted as diverged), and the disagreeing fraction of
pixel-frames is bounded.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import MixParams, MixtureOracle, FusionOracle, fuse_step, round_to_storage
from paper_2110_14934_amd import (GMM_RGB, GMM_DEPTH, GmmError, Segmenter, _abi, mask_words,
                                  gmm_fuse)
from paper_2110_14934_amd.synth import Stream, StreamSpec, workload, MixtureSettings
from tests.parity import (unpack_mask, pack_mask, to_canonical, from_canonical, excused, param_mismatch,
                          oracle_state, WEIGHT_MARGIN_FREE, KEY_GAP_FREE, MASK_FRACTION)

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mix_params(mix: MixtureSettings, modality: str, rho: str = "alpha") -> MixParams:
    if modality == "rgb":
        return MixParams(M=mix.M, alpha=mix.alpha, k=mix.k, T=mix.T, sigma0=mix.sigma0_rgb,
                         var_min=mix.var_min_rgb, w_init=mix.w_init, rho=rho)
    return MixParams(M=mix.M, alpha=mix.alpha, k=mix.k, T=mix.T, sigma0=mix.sigma0_depth,
                     var_min=mix.var_min_depth, w_init=mix.w_init, hole_skip=mix.hole_skip, rho=rho)


def seg_kwargs(mix: MixtureSettings):
    return dict(alpha=mix.alpha, k=mix.k, T=mix.T, sigma0=(mix.sigma0_rgb, mix.sigma0_depth),
                var_min=(mix.var_min_rgb, mix.var_min_depth), w_init=mix.w_init,
                hole_policy=_abi.GMM_HOLE_SKIP if mix.hole_skip else _abi.GMM_HOLE_AS_VALUE)


def _frames(st: Stream, t: int):
    return st.rgb(t) if st.spec.rgb else None, st.depth(t) if st.spec.depth else None


def _lockstep(spec: StreamSpec, mix: MixtureSettings, frames: int, dtype: str = "f32", fused=True,
              pitch_pad=0, misalign=False, rho="alpha"):
    """Run lockstep parity; returns (mask disagreements, pixel-frames)."""
    st = Stream(spec)
    n, M = spec.npix, mix.M
    mods = (GMM_RGB if spec.rgb else 0) | (GMM_DEPTH if spec.depth else 0)
    seg = Segmenter(spec.width, spec.height, mods, M, state_dtype=dtype, rho=rho, **seg_kwargs(mix))
    col = MixtureOracle(mix_params(mix, "rgb", rho), 3, n) if spec.rgb else None
    dep = MixtureOracle(mix_params(mix, "depth", rho), 1, n) if spec.depth else None
    both = spec.rgb and spec.depth
    fus = FusionOracle(n) if both else None
    storage = dtype
    disagree = 0
    total = 0
    try:
        for t in range(frames):
            rgb, depth = _frames(st, t)
            flat = round_to_storage(to_canonical(col, dep, fus), storage)
            if fus is not None:   # integers, restore exactly
                flat[-2 * n:] = to_canonical(None, None, fus)
            seg.write_state(flat)
            s = from_canonical(flat, M, n, spec.rgb, spec.depth)
            if col is not None:
                col.set_state(*s["rgb"])
            if dep is not None:
                dep.set_state(*s["depth"])
            if storage != "f32":
                if col is not None:
                    col.storage = storage
                if dep is not None:
                    dep.storage = storage
            ic = col.step(rgb.reshape(-1, 3).numpy()) if col is not None else None
            idd = dep.step(depth.reshape(-1).numpy()) if dep is not None else None

            # device side, with optionally pitched or misaligned input buffers
            g_rgb = g_dep = None
            if rgb is not None:
                if misalign:
                    buf = torch.zeros(rgb.numel() + 1, dtype=torch.uint8, device=DEV)
                    g_rgb = buf[1:].view(spec.height, spec.width, 3)
                    g_rgb.copy_(rgb.to(DEV))
                else:
                    buf = torch.zeros(spec.height, spec.width + pitch_pad, 3, dtype=torch.uint8, device=DEV)
                    g_rgb = buf[:, :spec.width, :]
                    g_rgb.copy_(rgb.to(DEV))
            if depth is not None:
                bufd = torch.zeros(spec.height, spec.width + pitch_pad, dtype=torch.uint16, device=DEV)
                g_dep = bufd[:, :spec.width]
                g_dep.copy_(depth.to(DEV))
            prev_I = fus.I.copy() if fus is not None else None
            prev_c = fus.cpt.copy() if fus is not None else None
            if both and fused:
                seg.apply_fused(g_rgb, g_dep)
            else:
                seg.apply(g_rgb, g_dep)
                if both:
                    seg.fuse(seg.fg_rgb, seg.fg_depth)
            torch.cuda.synchronize()
            got = from_canonical(seg.read_state(), M, n, spec.rgb, spec.depth)

            for name, info, o in (("rgb", ic, col), ("depth", idd, dep)):
                if info is None:
                    continue
                words = seg.fg_rgb if name == "rgb" else seg.fg_depth
                gm = unpack_mask(words, n)
                ex = excused(info)
                diff = gm != info.fg
                assert not np.any(diff & ~ex), (name, t, np.flatnonzero(diff & ~ex)[:10])
                bad = param_mismatch(got[name], oracle_state(o)) & ~ex
                if storage != "f32":
                    bad = _ulp_mismatch(got[name], oracle_state(o), storage) & ~ex
                assert not np.any(bad), (name, t, np.flatnonzero(bad)[:10])
                # pad bits of the last word are zero
                w = words.cpu().numpy().view(np.uint64)
                if n % 64:
                    assert int(w[-1]) >> (n % 64) == 0
                disagree += int(diff.sum())
                total += n
            if both:
                gr = unpack_mask(seg.fg_rgb, n)
                gd = unpack_mask(seg.fg_depth, n)
                eI, ec = fuse_step(gr, gd, prev_I, prev_c)
                assert np.array_equal(got["I"], eI) and np.array_equal(got["cpt"], ec), t
                assert np.array_equal(unpack_mask(seg.fused, n), eI.astype(bool)), t
                fus.step(ic.fg, idd.fg)
    finally:
        seg.close()
    assert disagree <= MASK_FRACTION * total + 1, (disagree, total)
    return disagree, total


def _ulp(v, storage):
    a = np.abs(v)
    if storage == "f16":
        e = np.floor(np.log2(np.maximum(a, 2.0 ** -14)))
        return 2.0 ** (e - 10)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -126)))
    return 2.0 ** (e - 7)


def _ulp_mismatch(gpu, ora, storage):
    bad = None
    for g, o in zip(gpu, ora):
        d = np.abs(g - o) > _ulp(o, storage) * 1.0001
        d = d.reshape(d.shape[0], -1, d.shape[-1]).any(axis=(0, 1))
        bad = d if bad is None else bad | d
    return bad


def test_generator_identical_on_gpu_and_cpu():
    wl = workload("plain-640x480")
    st = Stream(wl.streams[0])
    for t in (0, 125):
        assert torch.equal(st.rgb(t, device=DEV).cpu(), st.rgb(t))
        assert torch.equal(st.depth(t, device=DEV).cpu(), st.depth(t))


def test_lockstep_fused_small_workload():
    wl = workload("plain-160x120")
    say("lockstep plain-160x120 M=3 fused, 60 frames")
    d, n = _lockstep(wl.streams[0], wl.mix, wl.frames)
    say(f"mask disagreements {d}/{n}")


def test_lockstep_apply_then_fuse_small_workload():
    wl = workload("plain-160x120")
    say("lockstep plain-160x120 apply+fuse, 20 frames")
    _lockstep(wl.streams[0], wl.mix, 20, fused=False)


@pytest.mark.parametrize("w,h,M", [(17, 13, 1), (17, 13, 5), (161, 121, 4), (64, 1, 2), (1, 1, 3), (65, 3, 5)])
def test_lockstep_odd_shapes_pitched(w, h, M):
    spec = StreamSpec(w, h, n_boxes=1, box_min=max(1, min(w, h) // 3), box_max=max(1, min(w, h) // 2),
                      speed_min=1, speed_max=3, hole_p=0.1, seed=999 + w * 7 + h, index=M)
    mix = MixtureSettings(M=M, alpha=0.05, w_init=0.05)
    say(f"lockstep {w}x{h} M={M} pitched")
    _lockstep(spec, mix, 12, pitch_pad=5)


@pytest.mark.parametrize("kw", [
    dict(alpha=1.0, w_init=1.0),       # full replacement: every unmatched weight decays to 0
    dict(k=0.01),                      # almost nothing matches: the last rank is replaced each frame
    dict(T=1e-3),                      # B = 1: only rank 0 is background
    dict(T=0.999),                     # B = M for most pixels
    dict(alpha=1e-4, w_init=1e-4),     # very slow learning
    dict(hole_skip=False),             # depth 0 is a distance like any other value
], ids=["alpha1", "k_tiny", "T_tiny", "T_near1", "alpha_tiny", "holes_as_values"])
def test_lockstep_degenerate_parameters(kw):
    spec = StreamSpec(96, 40, n_boxes=2, box_min=6, box_max=12, hole_p=0.1, seed=77)
    say(f"lockstep degenerate {kw}")
    _lockstep(spec, MixtureSettings(M=4, **kw), 10)


def test_lockstep_misaligned_rgb_base():
    spec = StreamSpec(128, 8, n_boxes=1, box_min=4, box_max=6, hole_p=0.05, seed=4242)
    _lockstep(spec, MixtureSettings(M=3, alpha=0.05, w_init=0.05), 8, misalign=True)


@pytest.mark.parametrize("rgb,depth", [(True, False), (False, True)])
def test_lockstep_single_modality(rgb, depth):
    spec = StreamSpec(96, 40, rgb=rgb, depth=depth, n_boxes=2, box_min=6, box_max=12, hole_p=0.05, seed=31)
    _lockstep(spec, MixtureSettings(M=4, alpha=0.05, w_init=0.05), 15)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_lockstep_reduced_precision_state(dtype):
    wl = workload("plain-160x120")
    say(f"lockstep plain-160x120 state {dtype}")
    _lockstep(wl.streams[0], MixtureSettings(M=5), 25, dtype=dtype)


def test_free_run_small_workload():
    wl = workload("plain-160x120")
    spec, mix = wl.streams[0], wl.mix
    st = Stream(spec)
    n = spec.npix
    seg = Segmenter(spec.width, spec.height, GMM_RGB | GMM_DEPTH, mix.M, **seg_kwargs(mix))
    col = MixtureOracle(mix_params(mix, "rgb"), 3, n)
    dep = MixtureOracle(mix_params(mix, "depth"), 1, n)
    fus = FusionOracle(n)
    risky_c = np.zeros(n, bool)
    risky_d = np.zeros(n, bool)
    dis = 0
    try:
        for t in range(wl.frames):
            rgb, depth = _frames(st, t)
            ic = col.step(rgb.reshape(-1, 3).numpy())
            idd = dep.step(depth.reshape(-1).numpy())
            fo = fus.step(ic.fg, idd.fg)
            risky_c |= excused(ic, WEIGHT_MARGIN_FREE, KEY_GAP_FREE)
            risky_d |= excused(idd, WEIGHT_MARGIN_FREE, KEY_GAP_FREE)
            seg.apply_fused(rgb.to(DEV), depth.to(DEV))
            gc = unpack_mask(seg.fg_rgb, n)
            gd = unpack_mask(seg.fg_depth, n)
            gf = unpack_mask(seg.fused, n)
            assert not np.any((gc != ic.fg) & ~risky_c), t
            assert not np.any((gd != idd.fg) & ~risky_d), t
            assert not np.any((gf != fo) & ~(risky_c | risky_d)), t
            dis += int((gc != ic.fg).sum() + (gd != idd.fg).sum())
        got = from_canonical(seg.read_state(), mix.M, n, True, True)
        assert not np.any(param_mismatch(got["rgb"], oracle_state(col)) & ~risky_c)
        assert not np.any(param_mismatch(got["depth"], oracle_state(dep)) & ~risky_d)
    finally:
        seg.close()
    frac = dis / (2 * n * wl.frames)
    say(f"free run: mask disagreement fraction {frac:.2e}, diverged-risk pixels "
        f"{risky_c.mean():.2e} (rgb) {risky_d.mean():.2e} (depth)")
    assert frac <= MASK_FRACTION


def test_full_size_vga_sampled_pixels():
    """640x480, M=5, all 300 frames on the GPU in the benchmark's launch configuration (one fused
    launch per frame); the oracle follows 4096 sampled pixels (plus the ragged last rows)."""
    wl = workload("plain-640x480")
    spec, mix = wl.streams[0], wl.mix
    st = Stream(spec)
    n = spec.npix
    rng = np.random.default_rng(17)
    sample = np.unique(np.concatenate([rng.choice(n, 4096, replace=False), np.arange(n - 700, n)]))
    pix = torch.from_numpy(sample)
    k = sample.size
    seg = Segmenter(spec.width, spec.height, GMM_RGB | GMM_DEPTH, mix.M, **seg_kwargs(mix))
    col = MixtureOracle(mix_params(mix, "rgb"), 3, k)
    dep = MixtureOracle(mix_params(mix, "depth"), 1, k)
    fus = FusionOracle(k)
    risky_c = np.zeros(k, bool)
    risky_d = np.zeros(k, bool)
    dis = 0
    say(f"full-size 640x480 M=5, 300 frames, {k} sampled pixels")
    try:
        for t in range(wl.frames):
            rgb_g = st.rgb(t, device=DEV)
            dep_g = st.depth(t, device=DEV)
            seg.apply_fused(rgb_g, dep_g)
            ic = col.step(st.rgb(t, pix=pix).numpy())
            idd = dep.step(st.depth(t, pix=pix).numpy())
            fo = fus.step(ic.fg, idd.fg)
            risky_c |= excused(ic, WEIGHT_MARGIN_FREE, KEY_GAP_FREE)
            risky_d |= excused(idd, WEIGHT_MARGIN_FREE, KEY_GAP_FREE)
            gc = unpack_mask(seg.fg_rgb, n)[sample]
            gd = unpack_mask(seg.fg_depth, n)[sample]
            gf = unpack_mask(seg.fused, n)[sample]
            assert not np.any((gc != ic.fg) & ~risky_c), t
            assert not np.any((gd != idd.fg) & ~risky_d), t
            assert not np.any((gf != fo) & ~(risky_c | risky_d)), t
            dis += int((gc != ic.fg).sum() + (gd != idd.fg).sum())
            if t % 100 == 99:
                got = from_canonical(seg.read_state(), mix.M, n, True, True)
                g_rgb = tuple(a[..., sample] for a in got["rgb"])
                g_dep = tuple(a[..., sample] for a in got["depth"])
                assert not np.any(param_mismatch(g_rgb, oracle_state(col)) & ~risky_c), t
                assert not np.any(param_mismatch(g_dep, oracle_state(dep)) & ~risky_d), t
                say(f"  frame {t}: ok")
    finally:
        seg.close()
    frac = dis / (2 * k * wl.frames)
    say(f"full-size: mask disagreement fraction {frac:.2e}")
    assert frac <= MASK_FRACTION


def test_apply_then_fuse_bit_identical_to_fused():
    wl = workload("plain-160x120")
    spec, mix = wl.streams[0], wl.mix
    st = Stream(spec)
    a = Segmenter(spec.width, spec.height, GMM_RGB | GMM_DEPTH, mix.M, **seg_kwargs(mix))
    b = Segmenter(spec.width, spec.height, GMM_RGB | GMM_DEPTH, mix.M, **seg_kwargs(mix))
    try:
        for t in range(30):
            rgb, depth = st.rgb(t, device=DEV), st.depth(t, device=DEV)
            a.apply(rgb, depth)
            a.fuse(a.fg_rgb, a.fg_depth)
            b.apply_fused(rgb, depth)
            for x, y in ((a.fg_rgb, b.fg_rgb), (a.fg_depth, b.fg_depth), (a.fused, b.fused)):
                assert torch.equal(x, y), t
        assert np.array_equal(a.read_state(), b.read_state())
    finally:
        a.close()
        b.close()


def test_pixel_permutation_metamorphic():
    spec = StreamSpec(97, 33, n_boxes=2, box_min=5, box_max=12, hole_p=0.05, seed=5)
    st = Stream(spec)
    n = spec.npix
    perm = torch.from_numpy(np.random.default_rng(1).permutation(n))
    mix = MixtureSettings(M=5, alpha=0.05, w_init=0.05)
    a = Segmenter(spec.width, spec.height, GMM_RGB | GMM_DEPTH, 5, **seg_kwargs(mix))
    b = Segmenter(spec.width, spec.height, GMM_RGB | GMM_DEPTH, 5, **seg_kwargs(mix))
    try:
        for t in range(20):
            rgb, depth = st.rgb(t), st.depth(t)
            rp = rgb.reshape(-1, 3)[perm].reshape(rgb.shape)
            dp = depth.reshape(-1)[perm].reshape(depth.shape)
            a.apply_fused(rgb.to(DEV), depth.to(DEV))
            b.apply_fused(rp.to(DEV), dp.to(DEV))
            for x, y in ((a.fg_rgb, b.fg_rgb), (a.fg_depth, b.fg_depth), (a.fused, b.fused)):
                assert np.array_equal(unpack_mask(x, n)[perm.numpy()], unpack_mask(y, n)), t
        sa = from_canonical(a.read_state(), 5, n, True, True)
        sb = from_canonical(b.read_state(), 5, n, True, True)
        p = perm.numpy()
        for key in ("rgb", "depth"):
            for x, y in zip(sa[key], sb[key]):
                assert np.array_equal(x[..., p], y)
    finally:
        a.close()
        b.close()


def test_fuse_kernel_exhaustive_sequences():
    # all 4^8 (r, d) sequences, one per pixel of a 256x256 handle
    L, n = 8, 4 ** 8
    seg = Segmenter(256, 256, GMM_RGB | GMM_DEPTH, 1)
    codes = np.arange(n)
    I = np.zeros(n, np.int64)
    c = np.zeros(n, np.int64)
    try:
        for s in range(L):
            sym = (codes >> (2 * s)) & 3
            r, d = (sym & 1).astype(bool), (sym >> 1).astype(bool)
            fr = torch.from_numpy(pack_mask(r)).to(DEV)
            fd = torch.from_numpy(pack_mask(d)).to(DEV)
            out = seg.fuse(fr, fd)
            torch.cuda.synchronize()
            I, c = fuse_step(r, d, I, c)
            got = from_canonical(seg.read_state(), 1, n, True, True)
            assert np.array_equal(got["I"], I) and np.array_equal(got["cpt"], c), s
            assert np.array_equal(unpack_mask(out, n), I.astype(bool)), s
    finally:
        seg.close()


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_state_roundtrip(dtype):
    rng = np.random.default_rng(8)
    n, M = 1000, 4
    seg = Segmenter(40, 25, GMM_RGB | GMM_DEPTH, M, state_dtype=dtype)
    try:
        size = _abi.gmm_state_size(seg.handle)
        assert size == (5 * M + 3 * M + 2) * n
        flat = rng.uniform(0, 3000, size)
        flat[-2 * n:-n] = rng.integers(0, 2, n)
        flat[-n:] = rng.integers(-3, 4, n)
        seg.write_state(flat)
        back = seg.read_state()
        expect = round_to_storage(flat[:-2 * n], dtype)
        assert np.array_equal(back[:-2 * n], expect)
        assert np.array_equal(back[-2 * n:], flat[-2 * n:])
        bad = flat.copy()
        bad[-1] = 4
        with pytest.raises(GmmError):
            seg.write_state(bad)
    finally:
        seg.close()


def test_error_paths_on_device():
    seg = Segmenter(32, 8, GMM_RGB, 3)
    try:
        rgb = torch.zeros(8, 32, 3, dtype=torch.uint8, device=DEV)
        with pytest.raises(GmmError) as e:
            gmm_fuse(seg.handle, seg.fg_rgb, seg.fg_rgb, seg.fg_rgb)
        assert e.value.status == _abi.GMM_ERR_STATE
        with pytest.raises(GmmError) as e:
            _abi.gmm_apply_frame(seg.handle, rgb, 10, None, 0, seg.fg_rgb, None)
        assert e.value.status == _abi.GMM_ERR_INVALID_ARG
        with pytest.raises(GmmError) as e:
            _abi.gmm_apply_frame(seg.handle, rgb, 96, None, 0, None, None)
        assert e.value.status == _abi.GMM_ERR_INVALID_ARG
        seg.apply(rgb)
        torch.cuda.synchronize()
        # fp32: 15 values and rank 1's key per pixel, a scale per 64-pixel tile, rounded up to 256 B
        assert seg.state_bytes() == ((5 * 3 + 1) * 256 * 4 + 4 * 4 + 255) // 256 * 256
    finally:
        seg.close()


def test_traffic_record_counts_only_the_changed_pieces():
    """Colour only, M=3, fp32 (scaled weights): a lane's 16 values are 3 hot rows of 16, 4 and
    4 bytes (rank 0, which the fast path writes, then rank 1's key, which it only reads) and a
    40-byte suffix (rank 1, rank 2) written as two 16-byte groups and two words; each frame also
    reads and writes the tile's scale (8 B per wave). Frame 0 creates a component that walks
    from the last rank to rank 0: the whole state is read and written (2 x 64 B). Frame 1
    matches rank 0 (fast path: 24 B read, 20 B written). Frame 2 (x = 250) matches nothing; the
    new component takes rank 2 and walks to rank 1, and every scaled weight is renormalised:
    128 B. Frames 3 and 4 match rank 1, which keeps its rank (the oracle's j = q = 1): 64 B
    read, the rows and the two suffix groups holding rank 1's values written (24 + 32 B)."""
    seg = Segmenter(64, 1, GMM_RGB, 3)
    rec = torch.zeros(1, dtype=torch.int64, device=DEV)
    try:
        _abi.gmm_set_traffic_record(seg.handle, rec)
        want = 0
        for v, lane_bytes in ((100, 128), (100, 44), (250, 128), (250, 120), (250, 120)):
            seg.apply(torch.full((1, 64, 3), v, dtype=torch.uint8, device=DEV))
            torch.cuda.synchronize()
            want += 64 * lane_bytes + 8
            assert int(rec[0]) == want, (v, lane_bytes, int(rec[0]), want)
    finally:
        _abi.gmm_set_traffic_record(seg.handle, None)
        seg.close()


def test_traffic_record_counts_fast_and_full_lanes():
    """Traffic is decided per lane (M=5, fp32, scaled weights; each modality also reads and writes
    its tile's scale, 2 x 8 B per wave). Frame 0 matches nothing: every colour lane reads and
    writes its whole state (2 x (26 values x 4 B) = 208 B), every depth lane with a reading too
    (2 x 64 B = 128 B), while a depth hole only counts the frame in its flags byte: it moves the
    fast rows, read and written back unchanged (16 + 12 B). The same frame again matches rank 0
    everywhere and keeps the order, so every lane with a reading moves only rank 0 (+ rank 1's key
    on the read side), exactly: colour 24 + 20 B, depth 16 + 12 B; a hole again 28 B."""
    spec = StreamSpec(160, 120, n_boxes=1, box_min=20, box_max=20, hole_p=0.05, seed=61)
    st = Stream(spec)
    seg = Segmenter(160, 120, GMM_RGB | GMM_DEPTH, 5)
    rec = torch.zeros(spec.npix // 64, dtype=torch.int64, device=DEV)
    try:
        _abi.gmm_set_traffic_record(seg.handle, rec)
        rgb, depth = st.rgb(0, device=DEV), st.depth(0, device=DEV)
        holes = (depth.reshape(-1, 64) == 0).sum(dim=1).to(torch.int64)
        assert int(holes.sum()) > 0
        seg.apply_fused(rgb, depth)
        torch.cuda.synchronize()
        first = 64 * 208 + (64 - holes) * 128 + holes * 28 + 16
        assert torch.equal(rec, first)
        seg.apply_fused(rgb, depth)
        torch.cuda.synchronize()
        second = first + 64 * 44 + 64 * 28 + 16
        assert torch.equal(rec, second)
        _abi.gmm_set_traffic_record(seg.handle, None)
        seg.apply_fused(rgb, depth)
        torch.cuda.synchronize()
        assert torch.equal(rec, second)
    finally:
        seg.close()

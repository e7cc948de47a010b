"""The seeded input generator: determinism, shapes, statistics, geometry."""
import numpy as np
import pytest
import torch

from paper_2110_14934_amd.synth import Stream, StreamSpec, workload, WORKLOADS, _mix32, _mix32_int


def test_hash_tensor_matches_python_ints():
    vals = [0, 1, 2, 12345, 0xFFFFFFFF, 0x80000000, 0x7FEB352D]
    t = _mix32(torch.tensor(vals, dtype=torch.int64))
    assert t.tolist() == [_mix32_int(v) for v in vals]
    assert all(0 <= v <= 0xFFFFFFFF for v in t.tolist())


def test_frames_deterministic_and_typed():
    wl = workload("plain-160x120")
    s1, s2 = Stream(wl.streams[0]), Stream(wl.streams[0])
    for t in (0, 7, 59):
        a, b = s1.rgb(t), s2.rgb(t)
        assert a.dtype == torch.uint8 and a.shape == (120, 160, 3)
        assert torch.equal(a, b)
        da, db = s1.depth(t), s2.depth(t)
        assert da.dtype == torch.uint16 and da.shape == (120, 160)
        assert torch.equal(da, db)
    assert not torch.equal(s1.rgb(0), s1.rgb(1))


def test_pixel_subset_equals_full_frame():
    wl = workload("plain-640x480")
    st = Stream(wl.streams[0])
    pix = torch.tensor([0, 1, 639, 640, 123456, 307199], dtype=torch.int64)
    for t in (0, 120):
        full_c = st.rgb(t).reshape(-1, 3)
        full_d = st.depth(t).reshape(-1)
        assert torch.equal(st.rgb(t, pix=pix), full_c[pix])
        assert torch.equal(st.depth(t, pix=pix), full_d[pix])
        assert torch.equal(st.truth(t, pix=pix), st.truth(t).reshape(-1)[pix])


def test_noise_statistics_and_holes():
    spec = StreamSpec(256, 256, n_boxes=0, hole_p=0.05, sigma_c=2.0, seed=77)
    st = Stream(spec)
    bg = st.colour_background().numpy().astype(np.float64)
    f = st.rgb(3).reshape(-1, 3).numpy().astype(np.float64)
    inner = (bg > 10) & (bg < 245)
    resid = (f - bg)[inner]
    assert abs(resid.mean()) < 0.05
    assert resid.var() == pytest.approx(4.0 + 1 / 12, rel=0.05)   # noise plus rounding
    d = st.depth(3).reshape(-1).numpy().astype(np.float64)
    holes = d == 0
    assert holes.mean() == pytest.approx(0.05, abs=0.005)
    dv = d[~holes] - 2000
    assert dv.var() == pytest.approx(10.0 + 1 / 12, rel=0.05)
    # background colour is uniform over 0..255
    assert bg.min() == 0 and bg.max() == 255
    assert bg.mean() == pytest.approx(127.5, abs=1.5)


def test_boxes_move_reflect_and_occlude():
    wl = workload("plain-160x120")
    st = Stream(wl.streams[0])
    b = st.boxes[0]
    assert b.size == 20 and max(abs(b.vx), abs(b.vy)) == 2
    for t in range(0, 200, 7):
        (x, y, s), = st.box_positions(t)
        assert 0 <= x <= 160 - s and 0 <= y <= 120 - s
        m = st.truth(t).reshape(120, 160)
        assert int(m.sum()) == s * s
        assert bool(m[y, x]) and bool(m[y + s - 1, x + s - 1])
        f = st.rgb(t).reshape(120, 160, 3).numpy().astype(int)
        box = f[y:y + s, x:x + s]
        assert abs(box.mean() - 200) < 1.0
        d = st.depth(t).numpy().astype(int)[y:y + s, x:x + s]
        assert abs(np.median(d[d > 0]) - 1200) <= 2


def test_gain_ramp():
    wl = workload("plain-640x480")
    st = Stream(wl.streams[0])
    assert st.gain(0) == 0.6 and st.gain(100) == 0.6 and st.gain(150) == 1.2 and st.gain(299) == 1.2
    assert st.gain(125) == pytest.approx(0.9)


def test_workload_presets():
    sizes = {}
    for name in WORKLOADS:
        wl = workload(name)
        sizes[name] = (len(wl.streams), wl.frames, wl.mix.M)
    assert sizes["plain-160x120"] == (1, 60, 3)
    assert sizes["plain-640x480"] == (1, 300, 5)
    assert sizes["batch-64"] == (64, 120, 5)
    assert sizes["precision-256"] == (256, 120, 5)
    b = workload("batch-64")
    assert b.pixel_updates_per_frame == 16 * 320 * 240 * 2 + 32 * 640 * 480 * 2 + 8 * 512 * 424 + 8 * 1920 * 1080

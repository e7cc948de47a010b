"""bench.kernel_source_digest: the counter-measured traffic is reported only while the kernel's
code hashes to the value recorded with the counters; wording in comments must not change the
hash, code must."""
import os

import bench


def _digest_of(tmp_path, monkeypatch, texts):
    pkg = tmp_path / "paper_2110_14934_amd"
    (pkg / "csrc").mkdir(parents=True)
    names = []
    for name, text in texts.items():
        (pkg / name).write_text(text)
        names.append(name)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", {"frame": tuple(names)})
    return bench.kernel_source_digest("frame")


def test_comments_do_not_change_the_digest_code_does(tmp_path, monkeypatch):
    base = {"csrc/k.hip": "int f(int x) {\n  return x + 1;\n}\n", "build.py": "FLAGS = ['-O3']\n"}
    d0 = _digest_of(tmp_path / "a", monkeypatch, base)
    commented = {"csrc/k.hip": "// one more\nint f(int x) {  // add one\n  /* block\n comment */ return x + 1;\n}\n\n",
                 "build.py": "# flags\nFLAGS = ['-O3']\n"}
    assert _digest_of(tmp_path / "b", monkeypatch, commented) == d0
    changed = {"csrc/k.hip": "int f(int x) {\n  return x + 2;\n}\n", "build.py": "FLAGS = ['-O3']\n"}
    assert _digest_of(tmp_path / "c", monkeypatch, changed) != d0
    flags = {"csrc/k.hip": "int f(int x) {\n  return x + 1;\n}\n", "build.py": "FLAGS = ['-O2']\n"}
    assert _digest_of(tmp_path / "d", monkeypatch, flags) != d0


def test_recorded_traffic_is_reported_only_for_the_kernel_it_was_measured_on(tmp_path, monkeypatch):
    import json
    for wl, kind in (("plain-640x480", "frame"), ("batch-64", "batch")):
        path = bench.PROFILE_TRAFFIC[wl]
        assert os.path.exists(path), path
        rec = json.load(open(path))
        assert rec["hbm_bytes_per_launch"] > 0 and rec["kernel_source_digest"]
        traffic, _ = bench._traffic(wl, kind)
        assert traffic == (rec["hbm_bytes_per_launch"] if rec["kernel_source_digest"] == bench.kernel_source_digest(kind)
                           else None)
        # a record whose digest is the current kernel's is reported
        fake = dict(rec, kernel_source_digest=bench.kernel_source_digest(kind))
        p = tmp_path / f"{wl}.json"
        p.write_text(json.dumps(fake))
        monkeypatch.setitem(bench.PROFILE_TRAFFIC, wl, str(p))
        assert bench._traffic(wl, kind)[0] == rec["hbm_bytes_per_launch"]
        fake["kernel_source_digest"] = "0" * 16
        p.write_text(json.dumps(fake))
        assert bench._traffic(wl, kind)[0] is None


def test_clip_plays_forwards_then_backwards_without_a_jump():
    F = 120
    seq = [bench.clip_frame(i, F) for i in range(3 * (2 * F - 2) + 7)]
    assert seq[:F] == list(range(F))
    assert seq[F:2 * F - 2] == list(range(F - 2, 0, -1))
    assert all(abs(a - b) == 1 for a, b in zip(seq, seq[1:]))
    assert set(seq) == set(range(F))
    assert bench.clip_frame(5, 1) == 0

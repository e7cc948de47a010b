"""The serving executor and loop on the GPU: ticks of host frames give the same masks and state
as the single-stream path, memory accounting matches what is allocated, and a stream's results
are the same alone and in a churning mix."""
import numpy as np
import pytest
import torch

from paper_2110_14934_amd import GMM_RGB, GMM_DEPTH, Segmenter, _abi
from paper_2110_14934_amd.serve import FrameRequest, NativeExecutor, Server, StreamKind, run_load
from paper_2110_14934_amd.synth import Stream, StreamSpec

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)

SPECS = [
    StreamSpec(160, 120, n_boxes=1, box_min=20, box_max=20, hole_p=0.02, seed=71, index=0),
    StreamSpec(97, 33, n_boxes=2, box_min=5, box_max=10, hole_p=0.05, seed=71, index=1),
    StreamSpec(64, 48, rgb=False, depth=True, n_boxes=1, box_min=8, box_max=12, hole_p=0.05, seed=71, index=2),
    StreamSpec(200, 100, rgb=True, depth=False, n_boxes=2, box_min=10, box_max=30, seed=71, index=3),
]


def mods(sp):
    return (GMM_RGB if sp.rgb else 0) | (GMM_DEPTH if sp.depth else 0)


def pinned(t):
    return t.contiguous().pin_memory()


def words(sp):
    return (sp.npix + 63) // 64


# a wider frame whose byte counts are not multiples of 64 KiB
WIDE = StreamSpec(330, 241, n_boxes=2, box_min=20, box_max=40, hole_p=0.02, seed=71, index=4)


def host_frame(t, how, k):
    """Frame t in host memory, as the executor's copies meet it: pinned, pageable, or pinned at
    an odd offset inside a larger pinned allocation (an unaligned source address)."""
    t = t.contiguous()
    if how == "pageable":
        return t.clone()
    if how == "offset":
        flat = t.reshape(-1)
        e = flat.element_size()
        buf = torch.empty(flat.numel() + 16 // e, dtype=flat.dtype).pin_memory()
        view = buf[1 + k % 3:1 + k % 3 + flat.numel()]
        view.copy_(flat)
        return view
    return t.pin_memory()


@pytest.mark.parametrize("host_mem", ["pinned", "pageable", "mixed"])
def test_executor_ticks_bit_identical_to_plain_path(host_mem):
    specs = SPECS + [WIDE]
    streams = [Stream(s) for s in specs]
    x = _abi.gmm_exec_create(0, 3)
    handles, refs, outs = [], [], []
    how = {"pinned": ["pinned"], "pageable": ["pageable"], "mixed": ["pinned", "pageable", "offset"]}[host_mem]
    try:
        for sp in specs:
            cfg = _abi.gmm_config_default(sp.width, sp.height, mods(sp), 5, state_dtype=_abi.GMM_F16)
            h = _abi.gmm_create(cfg)
            handles.append(h)
            _abi.gmm_exec_attach(x, h)
            refs.append(Segmenter(sp.width, sp.height, mods(sp), 5, state_dtype="f16"))
        for t in range(12):
            items, keep = [], []
            for k, (sp, st, h) in enumerate(zip(specs, streams, handles)):
                hw = how[(k + t) % len(how)]
                rgb = host_frame(st.rgb(t), hw, k) if sp.rgb else None
                dep = host_frame(st.depth(t), hw, k + 1) if sp.depth else None
                o = [torch.zeros(words(sp), dtype=torch.int64).pin_memory() if on else None
                     for on in (sp.rgb, sp.depth, sp.rgb and sp.depth)]
                it = _abi.gmm_exec_item()
                it.handle = h
                it.host_rgb = rgb.data_ptr() if rgb is not None else None
                it.host_depth = dep.data_ptr() if dep is not None else None
                it.host_fg_rgb = o[0].data_ptr() if o[0] is not None else None
                it.host_fg_depth = o[1].data_ptr() if o[1] is not None else None
                it.host_fused = o[2].data_ptr() if o[2] is not None else None
                items.append(it)
                keep.append((rgb, dep, o))
            tick = _abi.gmm_exec_launch(x, items)
            assert tick == t + 1
            for sp, st, ref in zip(specs, streams, refs):
                rgb = st.rgb(t, device=DEV) if sp.rgb else None
                dep = st.depth(t, device=DEV) if sp.depth else None
                if sp.rgb and sp.depth:
                    ref.apply_fused(rgb, dep)
                else:
                    ref.apply(rgb, dep)
            _abi.gmm_exec_drain(x)
            done = _abi.gmm_exec_poll(x)
            assert [d[0] for d in done] == [tick]
            torch.cuda.synchronize()
            for (rgb, dep, o), ref in zip(keep, refs):
                for got, want in zip(o, (ref.fg_rgb, ref.fg_depth, ref.fused)):
                    if got is not None:
                        assert torch.equal(got, want.cpu()), t
        for h, ref in zip(handles, refs):
            assert np.array_equal(_abi.gmm_read_state(h), ref.read_state())
    finally:
        for h in handles:
            _abi.gmm_exec_detach(x, h)
            _abi.gmm_destroy(h)
        _abi.gmm_exec_destroy(x)
        for r in refs:
            r.close()


def _item(h, rgb, dep, o):
    it = _abi.gmm_exec_item()
    it.handle = h
    it.host_rgb = rgb.data_ptr() if rgb is not None else None
    it.host_depth = dep.data_ptr() if dep is not None else None
    for name, b in zip(("host_fg_rgb", "host_fg_depth", "host_fused"), o):
        setattr(it, name, b.data_ptr() if b is not None else None)
    return it


@pytest.mark.parametrize("ring", [2, 4])
def test_two_frames_per_stream_in_flight(ring):
    """Tick t+1 is launched before tick t completes, so every stream has two frames on the
    device (one per frame slot) and the copy-in of one overlaps the compute of the other; masks
    of every tick and the final state equal the plain path's."""
    specs = SPECS + [WIDE]
    streams = [Stream(s) for s in specs]
    x = _abi.gmm_exec_create(0, ring)
    handles, refs = [], []
    T = 14
    how = ["pinned", "pageable", "offset"]
    try:
        for sp in specs:
            cfg = _abi.gmm_config_default(sp.width, sp.height, mods(sp), 5, state_dtype=_abi.GMM_F16)
            h = _abi.gmm_create(cfg)
            handles.append(h)
            _abi.gmm_exec_attach(x, h)
            refs.append(Segmenter(sp.width, sp.height, mods(sp), 5, state_dtype="f16"))
        keep, want, done = {}, {}, []
        for t in range(T):
            items, kt = [], []
            for k, (sp, st, h) in enumerate(zip(specs, streams, handles)):
                hw = how[(k + t) % len(how)]
                rgb = host_frame(st.rgb(t), hw, k) if sp.rgb else None
                dep = host_frame(st.depth(t), hw, k + 1) if sp.depth else None
                o = [torch.zeros(words(sp), dtype=torch.int64).pin_memory() if on else None
                     for on in (sp.rgb, sp.depth, sp.rgb and sp.depth)]
                items.append(_item(h, rgb, dep, o))
                kt.append((rgb, dep, o))
            tick = _abi.gmm_exec_launch(x, items)
            keep[tick] = kt
            w = []
            for sp, st, ref in zip(specs, streams, refs):
                rgb = st.rgb(t, device=DEV) if sp.rgb else None
                dep = st.depth(t, device=DEV) if sp.depth else None
                if sp.rgb and sp.depth:
                    ref.apply_fused(rgb, dep)
                else:
                    ref.apply(rgb, dep)
                w.append([m.cpu() if m is not None else None for m in (ref.fg_rgb, ref.fg_depth, ref.fused)])
            want[tick] = w
            # before the next launch, the tick before this one has to be complete
            while not any(d[0] == tick - 1 for d in done) and tick > 1:
                done += _abi.gmm_exec_poll(x)
        _abi.gmm_exec_drain(x)
        done += _abi.gmm_exec_poll(x)
        assert [d[0] for d in done] == list(range(1, T + 1))
        for tick in range(1, T + 1):
            for (rgb, dep, o), w in zip(keep[tick], want[tick]):
                for got, ref in zip(o, w):
                    if got is not None:
                        assert torch.equal(got, ref), tick
        for h, ref in zip(handles, refs):
            assert np.array_equal(_abi.gmm_read_state(h), ref.read_state())
    finally:
        _abi.gmm_exec_drain(x)
        for h in handles:
            _abi.gmm_exec_detach(x, h)
            _abi.gmm_destroy(h)
        _abi.gmm_exec_destroy(x)
        for r in refs:
            r.close()


def test_memory_accounting_matches_allocation():
    ex = NativeExecutor(ring=2, state_dtype="f16", arena_bytes=256 << 20)
    try:
        free0 = ex.arena.free_bytes()
        for sp in SPECS + [StreamSpec(1920, 1080, rgb=True, depth=False), StreamSpec(512, 424, rgb=False)]:
            h, nbytes = ex.open_stream(sp.width, sp.height, mods(sp))
            assert nbytes == ex.bytes_needed(sp.width, sp.height, mods(sp)), sp
            assert nbytes >= _abi.gmm_state_bytes(h) + sp.npix * (3 * sp.rgb + 2 * sp.depth)
            ex.close_stream(h)
        assert ex.arena.free_bytes() == free0
    finally:
        ex.close()


def test_stream_alone_equals_stream_in_churning_mix():
    sp = SPECS[0]
    st = Stream(sp)
    frames = [(pinned(st.rgb(t)), pinned(st.depth(t))) for t in range(20)]
    others = [Stream(StreamSpec(120, 90, n_boxes=1, box_min=10, box_max=20, seed=72, index=i)) for i in range(6)]
    other_frames = [[(pinned(o.rgb(t)), pinned(o.depth(t))) for t in range(20)] for o in others]

    def run(mixed):
        ex = NativeExecutor(ring=3, state_dtype="f16", arena_bytes=512 << 20)
        srv = Server(ex, 512 << 20, max_queue=64)
        a = srv.join(sp.width, sp.height, GMM_RGB | GMM_DEPTH)
        live = []
        out = {}
        nw = words(sp)
        masks = [[torch.zeros(nw, dtype=torch.int64).pin_memory() for _ in range(3)] for _ in range(20)]
        try:
            if mixed:
                live = [srv.join(120, 90, GMM_RGB | GMM_DEPTH) for _ in range(4)]
            for t in range(20):
                m = masks[t]
                srv.submit(FrameRequest(a, t, 0.0, frames[t][0], frames[t][1], m[0], m[1], m[2]))
                if mixed:
                    for k, sid in enumerate(list(live)):
                        f = other_frames[(sid + k) % 6][t]
                        srv.submit(FrameRequest(sid, t, 0.0, f[0], f[1]))
                    if t % 5 == 2:
                        srv.leave(live.pop(0))
                        live.append(srv.join(120, 90, GMM_RGB | GMM_DEPTH))
                for req in srv.step():
                    if req.stream_id == a:
                        out[req.seq] = [b.clone() for b in masks[req.seq]]
            ex.drain()
            for _ in range(50):
                for req in srv.step():
                    if req.stream_id == a:
                        out[req.seq] = [b.clone() for b in masks[req.seq]]
                if len(out) == 20:
                    break
                ex.drain()
            state = _abi.gmm_read_state(srv.streams[a].handle)
            return out, state
        finally:
            srv.close()
            ex.close()

    alone, s1 = run(False)
    mixed, s2 = run(True)
    assert sorted(alone) == list(range(20)) and sorted(mixed) == list(range(20))
    for t in range(20):
        for p, q in zip(alone[t], mixed[t]):
            assert torch.equal(p, q), t
    assert np.array_equal(s1, s2)


def test_short_serving_run():
    mix = (StreamKind(160, 120, GMM_RGB | GMM_DEPTH, 3), StreamKind(320, 240, GMM_DEPTH, 1))
    pools = {}
    for k in mix:
        st = Stream(StreamSpec(k.width, k.height, rgb=bool(k.modalities & GMM_RGB), depth=bool(k.modalities & GMM_DEPTH),
                               n_boxes=1, box_min=10, box_max=20, seed=73))
        pools[(k.width, k.height, k.modalities)] = [
            (pinned(st.rgb(t)) if k.modalities & GMM_RGB else None, pinned(st.depth(t)) if k.modalities & GMM_DEPTH else None)
            for t in range(4)]
    ex = NativeExecutor(ring=4, state_dtype="f16", arena_bytes=1 << 30)
    srv = Server(ex, 1 << 30)
    try:
        rep = run_load(srv, pools, n_streams=48, duration_s=3.0, churn_per_s=2.0, mix=mix, warmup_s=0.5)
    finally:
        srv.close()
        ex.close()
    print("SERVE_SMOKE", rep, flush=True)
    assert rep["frames_completed"] > 48 * 30 * 2
    assert rep["p99_latency_ms"] < 33.0
    assert rep["stats"]["dropped"] == 0


# ---- served streams against the FP64 oracle ------------------------------------------------

def _serve_and_follow(dtype, T=30):
    """Three target streams (colour+depth, depth only, colour only) served in a churning mix with
    two frames per stream in flight; returns per target the masks of every frame and the final
    state, beside the oracle that stepped the same frames (emulating the storage rounding for
    16-bit state)."""
    from oracle import MixParams, MixtureOracle, FusionOracle
    from tests.parity import unpack_mask
    targets = [StreamSpec(160, 120, n_boxes=2, box_min=10, box_max=30, hole_p=0.05, seed=74, index=0),
               StreamSpec(96, 40, rgb=False, depth=True, n_boxes=1, box_min=6, box_max=12, hole_p=0.05, seed=74, index=1),
               StreamSpec(120, 64, rgb=True, depth=False, n_boxes=2, box_min=8, box_max=20, seed=74, index=2)]
    tstreams = [Stream(s) for s in targets]
    frames = [[(pinned(st.rgb(t)) if sp.rgb else None, pinned(st.depth(t)) if sp.depth else None)
               for t in range(T)] for sp, st in zip(targets, tstreams)]
    bg = [Stream(StreamSpec(80, 60, n_boxes=1, box_min=5, box_max=15, seed=75, index=i)) for i in range(4)]
    bg_frames = [[(pinned(o.rgb(t)), pinned(o.depth(t))) for t in range(T)] for o in bg]
    storage = None if dtype == "f32" else dtype
    oracles = []
    for sp in targets:
        col = MixtureOracle(MixParams(5, 0.01, 2.5, 0.7, 30.0, 9.0, 0.01), 3, sp.npix, storage) if sp.rgb else None
        dep = (MixtureOracle(MixParams(5, 0.01, 2.5, 0.7, 50.0, 25.0, 0.01, hole_skip=True), 1, sp.npix, storage)
               if sp.depth else None)
        oracles.append((col, dep, FusionOracle(sp.npix) if sp.rgb and sp.depth else None))
    ex = NativeExecutor(ring=3, state_dtype=dtype, arena_bytes=256 << 20)
    srv = Server(ex, 256 << 20, max_queue=64)
    masks = [[[torch.zeros(words(sp), dtype=torch.int64).pin_memory() if on else None
               for on in (sp.rgb, sp.depth, sp.rgb and sp.depth)] for _ in range(T)] for sp in targets]
    got = {}
    try:
        sids = [srv.join(sp.width, sp.height, mods(sp)) for sp in targets]
        live = [srv.join(80, 60, GMM_RGB | GMM_DEPTH) for _ in range(3)]
        for t in range(T):
            for k, (sid, sp) in enumerate(zip(sids, targets)):
                m = masks[k][t]
                assert srv.submit(FrameRequest(sid, t, 0.0, frames[k][t][0], frames[k][t][1], m[0], m[1], m[2]))
            for j, sid in enumerate(live):
                f = bg_frames[(sid + j) % 4][t]
                srv.submit(FrameRequest(sid, t, 0.0, f[0], f[1]))
            if t % 6 == 3:   # churn: one background stream leaves, another joins
                srv.leave(live.pop(0))
                live.append(srv.join(80, 60, GMM_RGB | GMM_DEPTH))
            # two launches per frame period: each stream's next frame goes out before its last
            # one has completed (two frames per stream on the device)
            for _ in range(2):
                for req in srv.step():
                    got[(req.stream_id, req.seq)] = True
        for _ in range(200):
            ex.drain()
            for req in srv.step():
                got[(req.stream_id, req.seq)] = True
            if all((sid, t) in got for sid in sids for t in range(T)):
                break
        assert all((sid, t) in got for sid in sids for t in range(T))
        states = [_abi.gmm_read_state(srv.streams[sid].handle) for sid in sids]
    finally:
        srv.close()
        ex.close()
    assert srv.stats["ticks"] >= T
    results = []
    for k, (sp, st) in enumerate(zip(targets, tstreams)):
        col, dep, fus = oracles[k]
        per_frame = []
        for t in range(T):
            ic = col.step(st.rgb(t).reshape(-1, 3).numpy()) if col is not None else None
            idd = dep.step(st.depth(t).reshape(-1).numpy()) if dep is not None else None
            fo = fus.step(ic.fg, idd.fg) if fus is not None else None
            m = masks[k][t]
            per_frame.append((ic, idd, fo, [unpack_mask(w, sp.npix) if w is not None else None for w in m]))
        results.append((sp, (col, dep, fus), per_frame, states[k]))
    return results


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_served_streams_follow_the_oracle(dtype):
    """Served frames against the FP64 oracle in free run. fp32 state: masks equal except at
    pixels whose decision was within the free-run margins (these count as diverged from then on),
    parameters within 1e-4 relative elsewhere, differing pixel-frames <= 1e-4. fp16 state: the
    oracle rounds every stored value to fp16 as the device does; parameters within 4 fp16 ulps
    (the device computes in fp32, the oracle in fp64, so a value can round the other way when it
    falls within a few fp32 ulps of an fp16 midpoint, about once in a thousand updates, and such
    one-ulp steps can add up over a free run; 2 ulps measured), decisions excused within
    fp16-sized margins."""
    from tests.parity import (excused, from_canonical, param_mismatch, oracle_state, WEIGHT_MARGIN_FREE,
                              KEY_GAP_FREE, MASK_FRACTION)
    from tests.test_gpu_parity import _ulp
    res = _serve_and_follow(dtype)
    wm, kg = (WEIGHT_MARGIN_FREE, KEY_GAP_FREE) if dtype == "f32" else (4e-3, 4e-3)
    dis = total = 0
    worst_ulps = 0.0
    for sp, (col, dep, fus), per_frame, state in res:
        n = sp.npix
        risky = {"rgb": np.zeros(n, bool), "depth": np.zeros(n, bool)}
        for t, (ic, idd, fo, (gr, gd, gf)) in enumerate(per_frame):
            for name, info, g in (("rgb", ic, gr), ("depth", idd, gd)):
                if info is None:
                    continue
                ex = excused(info, wm, kg)
                if dtype != "f32":
                    ex |= info.match_margin < 4e-3
                risky[name] |= ex
                diff = g != info.fg
                assert not np.any(diff & ~risky[name]), (sp, name, t, np.flatnonzero(diff & ~risky[name])[:8])
                dis += int(diff.sum())
                total += n
            if fo is not None:
                assert not np.any((gf != fo) & ~(risky["rgb"] | risky["depth"])), (sp, t)
        got = from_canonical(state, 5, n, sp.rgb, sp.depth)
        for name, o in (("rgb", col), ("depth", dep)):
            if o is None:
                continue
            if dtype == "f32":
                bad = param_mismatch(got[name], oracle_state(o)) & ~risky[name]
                assert not np.any(bad), (sp, name, np.flatnonzero(bad)[:8])
            else:
                for g, ov in zip(got[name], oracle_state(o)):
                    u = np.abs(g - ov) / _ulp(ov, dtype)
                    u = u.reshape(-1, n)[:, ~risky[name]]
                    worst_ulps = max(worst_ulps, float(u.max()) if u.size else 0.0)
        print(f"SERVE_ORACLE {dtype} {sp.width}x{sp.height} risky rgb {risky['rgb'].mean():.2e} "
              f"depth {risky['depth'].mean():.2e}", flush=True)
    print(f"SERVE_ORACLE {dtype}: mask disagreement {dis}/{total} = {dis / total:.2e}, worst non-risky "
          f"parameter error {worst_ulps:.2f} storage ulps", flush=True)
    assert dis <= (MASK_FRACTION if dtype == "f32" else 1e-3) * total + 1
    if dtype != "f32":
        assert worst_ulps <= 4.0001

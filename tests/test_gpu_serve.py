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


# a frame of several 64 KiB ingest pieces with a ragged last piece
WIDE = StreamSpec(330, 241, n_boxes=2, box_min=20, box_max=40, hole_p=0.02, seed=71, index=4)


def host_frame(t, how, k):
    """Frame t in host memory: pinned (read by the ingest kernel), pageable (copied by DMA), or
    pinned at an odd offset inside a larger pinned allocation (ingest, unaligned pieces)."""
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

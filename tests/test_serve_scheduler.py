"""The serving scheduler on the CPU, against a fake executor: admission by memory budget, at
most the executor's number of frames per stream in flight (one or two), FIFO order, continuous batching, leave while in flight, dropped
frames, and each stream's results identical alone and in a mix (the fake computes masks with
the FP64 oracle, so a mixed-up frame or state would show)."""
import math

import numpy as np
import pytest

from oracle import MixParams, MixtureOracle
from paper_2110_14934_amd.serve import Arena, FrameRequest, Server, run_load, StreamKind, GMM_RGB, GMM_DEPTH


class FakeExecutor:
    """Completes ticks when told to (or after `latency` of its own clock); checks invariants."""

    def __init__(self, latency=0.0, dt=0.0, depth=1):
        self.frames_in_flight = depth
        self.t = 0.0
        self.dt = dt
        self.latency = latency
        self.next_tick = 1
        self.inflight = {}          # tick -> (t_launch, [stream ids])
        self.busy = {}              # stream -> frames on the "device"
        self.opened = {}
        self.last_seq = {}
        self.models = {}            # stream -> oracle (depth only, 1 channel)
        self.results = {}           # (stream, seq) -> fg mask
        self.launches = []

    # clock
    def now(self):
        self.t += self.dt
        return self.t

    def bytes_needed(self, w, h, mods):
        return w * h * 10

    def open_stream(self, w, h, mods):
        hid = object()
        self.opened[hid] = (w, h, mods)
        self.models[hid] = MixtureOracle(MixParams(3, 0.1, 2.5, 0.7, 20.0, 4.0, 0.1), 1, w * h)
        return hid, self.bytes_needed(w, h, mods)

    def close_stream(self, hid):
        assert hid not in self.busy, "stream closed with a frame in flight"
        del self.opened[hid]

    def launch(self, reqs):
        ids = []
        for st, r in reqs:
            assert st.handle in self.opened
            assert self.busy.get(st.handle, 0) < self.frames_in_flight, "too many frames of one stream in flight"
            assert st.handle not in ids, "stream twice in a tick"
            assert self.last_seq.get(st.handle, -1) < r.seq, "frames out of order"
            self.last_seq[st.handle] = r.seq
            self.busy[st.handle] = self.busy.get(st.handle, 0) + 1
            ids.append(st.handle)
            fg = self.models[st.handle].step(np.asarray(r.depth, np.float64).reshape(-1, 1)).fg
            self.results[(st.id, r.seq)] = fg
        tick = self.next_tick
        self.next_tick += 1
        self.inflight[tick] = (self.t, ids)
        self.launches.append(len(reqs))
        return tick

    def complete_all(self):
        for tick in list(self.inflight):
            self._done.append((tick, self.t))
            for h in self.inflight.pop(tick)[1]:
                self._free(h)

    _done = None

    def _free(self, h):
        self.busy[h] -= 1
        if self.busy[h] == 0:
            del self.busy[h]

    def poll(self):
        if self._done is None:
            self._done = []
        if self.latency > 0:
            for tick, (t0, ids) in sorted(self.inflight.items()):
                if self.t - t0 >= self.latency:
                    self._done.append((tick, self.t))
                    del self.inflight[tick]
                    for h in ids:
                        self._free(h)
        out, self._done = self._done, []
        return out

    def drain(self):
        if self._done is None:
            self._done = []
        self.complete_all()


def _req(sid, seq, t=0.0, n=4, value=100):
    return FrameRequest(sid, seq, t, None, np.full(n, value + seq, np.uint16))


def test_admission_by_memory_budget():
    x = FakeExecutor()
    srv = Server(x, hbm_budget_bytes=100)
    assert srv.join(4, 4, GMM_DEPTH) is None            # 160 bytes > 100
    srv = Server(x, hbm_budget_bytes=100)
    assert srv.join(2, 2, GMM_DEPTH) == 0               # 40
    assert srv.join(2, 2, GMM_DEPTH) == 1               # 80
    assert srv.join(2, 2, GMM_DEPTH) is None            # 120 > 100
    assert srv.stats["rejected"] == 1
    srv.leave(0)
    assert srv.used == 40
    assert srv.join(2, 2, GMM_DEPTH) == 2


def test_one_frame_in_flight_fifo_and_continuous_batching():
    x = FakeExecutor()
    x._done = []
    srv = Server(x, 10 ** 6)
    a, b = srv.join(2, 2, GMM_DEPTH), srv.join(2, 2, GMM_DEPTH)
    for s in range(3):
        assert srv.submit(_req(a, s))
    assert srv.step() == [] and x.launches == [1]       # only a's oldest frame
    assert srv.submit(_req(b, 0))                        # arrives while a's frame is on the device
    srv.step()
    assert x.launches == [1, 1]                          # b joins the next tick, a waits
    x.complete_all()
    done = srv.step()
    assert sorted((r.stream_id, r.seq) for r in done) == [(a, 0), (b, 0)]
    assert x.launches == [1, 1, 1]                       # a's seq 1
    x.complete_all()
    srv.step()
    x.complete_all()
    done = srv.step()
    assert [(r.stream_id, r.seq) for r in done] == [(a, 2)]
    assert srv.in_flight() == 0


def test_two_frames_in_flight_when_the_executor_has_two_slots():
    x = FakeExecutor(depth=2)
    x._done = []
    srv = Server(x, 10 ** 6)
    a, b = srv.join(2, 2, GMM_DEPTH), srv.join(2, 2, GMM_DEPTH)
    for s in range(4):
        assert srv.submit(_req(a, s))
    srv.step()
    srv.step()
    srv.step()
    assert x.launches == [1, 1]                          # a's seq 0 and 1; seq 2 waits for a slot
    assert srv.streams[a].in_flight == 2 and [r.seq for r in srv.streams[a].queue] == [2, 3]
    assert srv.submit(_req(b, 0))
    srv.step()
    assert x.launches == [1, 1, 1]                       # b is not held back by a
    x.complete_all()
    done = srv.step()
    assert [(r.stream_id, r.seq) for r in done] == [(a, 0), (a, 1), (b, 0)]
    assert x.launches == [1, 1, 1, 1]                    # a's seq 2 (seq 3 joins the next tick)
    srv.step()
    x.complete_all()
    done = srv.step()
    assert [(r.stream_id, r.seq) for r in done] == [(a, 2), (a, 3)]
    assert srv.in_flight() == 0 and x.busy == {}
    srv.submit(_req(a, 4))
    srv.submit(_req(a, 5))
    srv.step()
    srv.step()
    srv.leave(a)                                         # two in flight: memory held until both end
    assert a in srv.streams
    x.complete_all()
    srv.step()
    assert a not in srv.streams


def test_leave_while_in_flight_releases_after_completion():
    x = FakeExecutor()
    x._done = []
    srv = Server(x, 10 ** 6)
    a = srv.join(2, 2, GMM_DEPTH)
    for s in range(3):
        srv.submit(_req(a, s))
    srv.step()
    srv.leave(a)                                         # one in flight, two queued
    assert srv.stats["cancelled"] == 2
    assert a in srv.streams and srv.used == 40           # memory held until the frame completes
    assert not srv.submit(_req(a, 9))
    x.complete_all()
    done = srv.step()
    assert [(r.stream_id, r.seq) for r in done] == [(a, 0)]
    assert a not in srv.streams and srv.used == 0


def test_full_queue_drops_and_counts():
    x = FakeExecutor()
    x._done = []
    srv = Server(x, 10 ** 6, max_queue=2)
    a = srv.join(2, 2, GMM_DEPTH)
    assert srv.submit(_req(a, 0)) and srv.submit(_req(a, 1))
    assert not srv.submit(_req(a, 2))
    assert srv.stats["dropped"] == 1 and srv.stats["submitted"] == 3


@pytest.mark.parametrize("depth", [1, 2])
def test_results_alone_equal_results_in_the_mix(depth):
    rng = np.random.default_rng(4)
    frames = [rng.integers(90, 110, 16).astype(np.uint16) for _ in range(30)]

    def run(mixed: bool):
        x = FakeExecutor(depth=depth)
        x._done = []
        srv = Server(x, 10 ** 6, max_queue=64)
        others = []
        a = srv.join(4, 4, GMM_DEPTH)
        if mixed:
            others = [srv.join(4, 4, GMM_DEPTH) for _ in range(5)]
        for t, f in enumerate(frames):
            srv.submit(FrameRequest(a, t, float(t), None, f))
            for o in list(others):
                srv.submit(FrameRequest(o, t, float(t), None, rng.integers(0, 60000, 16).astype(np.uint16)))
            if mixed and t % 7 == 3:                 # churn: one leaves, one joins
                srv.leave(others.pop(0))
                others.append(srv.join(4, 4, GMM_DEPTH))
            srv.step()
            if t % 3 == 2:
                x.complete_all()
        x.complete_all()
        while srv.in_flight() or any(s.queue for s in srv.streams.values()):
            srv.step()
            x.complete_all()
        srv.step()
        return [x.results[(a, t)] for t in range(len(frames))]

    alone, mixed = run(False), run(True)
    for t, (p, q) in enumerate(zip(alone, mixed)):
        assert np.array_equal(p, q), t


@pytest.mark.parametrize("depth", [1, 2])
def test_run_load_accounting_with_fake_clock(depth):
    x = FakeExecutor(latency=0.010, dt=0.0005, depth=depth)
    srv = Server(x, 10 ** 9)

    class Px:   # a stand-in for a pinned frame; the fake only reads it as depth values
        def __init__(self, n):
            self.a = np.full(n, 2000, np.uint16)

        def __array__(self, dtype=None):
            return self.a if dtype is None else self.a.astype(dtype)

    mix = (StreamKind(4, 4, GMM_DEPTH, 1.0),)
    pools = {(4, 4, GMM_DEPTH): [(None, Px(16))]}
    rep = run_load(srv, pools, n_streams=8, duration_s=2.0, fps=30, jitter=0.2, churn_per_s=2.0, mix=mix,
                   warmup_s=0.5, mask_alloc=lambda nw: np.empty(nw, np.int64))
    assert rep["frames_completed"] > 8 * 30 * 1.2
    assert rep["p50_latency_ms"] >= 10.0 - 1e-6
    assert rep["p99_latency_ms"] < 40.0
    assert rep["stats"]["left"] >= 3 and rep["stats"]["joined"] >= 8 + 3
    assert math.isfinite(rep["pixel_updates_per_s"])
    assert [e["t"] for e in rep["timeline"]] == [0, 1]
    assert sum(e["frames"] for e in rep["timeline"]) == rep["frames_completed"]
    assert sum(e["dropped"] for e in rep["timeline"]) <= rep["stats"]["dropped"]


def test_arena_first_fit_and_coalescing():
    a = Arena(10 * 256 + 100)
    assert a.size == 10 * 256
    x = a.alloc(300)        # 2 granules
    y = a.alloc(256)
    z = a.alloc(1)
    assert (x, y, z) == (0, 512, 768)
    assert a.alloc(7 * 256) is None          # only 6 granules left
    a.release(y)
    assert a.alloc(256) == 512               # first fit reuses the hole
    a.release(x)
    a.release(512)
    a.release(z)
    assert a.free == [(0, 10 * 256)] and a.free_bytes() == 10 * 256
    rng = np.random.default_rng(0)
    live = {}
    for _ in range(500):
        if live and rng.random() < 0.5:
            off = list(live)[rng.integers(len(live))]
            a.release(off)
            del live[off]
        else:
            n = int(rng.integers(1, 700))
            off = a.alloc(n)
            if off is not None:
                for o, ln in live.items():   # no overlap with live blocks
                    assert off + n <= o or o + ln <= off
                live[off] = n
    assert a.free_bytes() + sum(a.used.values()) == a.size


def test_failed_launch_leaves_the_server_consistent():
    class Failing(FakeExecutor):
        fail_next = True

        def launch(self, reqs):
            if self.fail_next:
                self.fail_next = False
                raise RuntimeError("device error")
            return super().launch(reqs)

    x = Failing()
    x._done = []
    srv = Server(x, 10 ** 6)
    a, b = srv.join(2, 2, GMM_DEPTH), srv.join(2, 2, GMM_DEPTH)
    srv.submit(_req(a, 0))
    srv.submit(_req(a, 1))
    srv.submit(_req(b, 0))
    with pytest.raises(RuntimeError):
        srv.step()
    assert srv.in_flight() == 0
    assert [r.seq for r in srv.streams[a].queue] == [0, 1] and [r.seq for r in srv.streams[b].queue] == [0]
    srv.step()                                      # the retry launches the same frames, in order
    x.complete_all()
    done = srv.step()
    assert sorted((r.stream_id, r.seq) for r in done) == [(a, 0), (b, 0)]


def test_percentile_counts_dropped_frames_as_infinitely_late():
    import math
    from paper_2110_14934_amd.serve import percentile_with_drops
    lat = [float(i) for i in range(1, 101)]          # 1 .. 100
    assert percentile_with_drops(lat, 0, 99) == 99.0
    assert percentile_with_drops(lat, 0, 50) == 50.0
    # one drop among 101 frames: the 99th percentile (rank 100) is still a completed frame
    assert percentile_with_drops(lat, 1, 99) == 100.0
    # two drops among 102: rank ceil(0.99 * 102) = 101 lands on a drop
    assert percentile_with_drops(lat, 2, 99) == math.inf
    assert math.isnan(percentile_with_drops([], 0, 99))
    assert percentile_with_drops([], 3, 50) == math.inf

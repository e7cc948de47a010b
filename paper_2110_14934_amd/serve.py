"""Serving loop: frames of many camera streams arrive over time and are advanced by continuous
batching through the native executor (gmm_exec_*), with every stream's mixture state resident
in device memory.

Policy (``Server``):
  * admission: a stream joins only if its device bytes (state + frame slot + masks) fit in the
    memory budget next to the streams already admitted; otherwise the join is refused and the
    caller may retry later, when leaves have freed memory;
  * each stream keeps a FIFO of submitted frames (bounded; a frame arriving to a full queue is
    dropped and counted). At most ``executor.frames_in_flight`` frames per stream are on the
    device at a time (the native executor: two, one per device frame slot; every frame reads
    and rewrites the stream's state, and the executor applies a stream's frames in launch
    order, so frame n+1 can be copied in while frame n computes);
  * continuous batching: every ``step`` first collects completed ticks, then launches ONE tick
    holding the oldest queued frame of every stream below that limit. Frames that arrive while
    earlier ticks run join the next tick; up to the executor's ring of ticks are on the device
    at once, overlapping their copies and kernels;
  * leave: queued frames of the stream are cancelled, its in-flight frames complete, then its
    memory is released.

The scheduling logic only talks to an executor object (``open_stream``, ``close_stream``,
``launch``, ``poll``, ``now``); ``NativeExecutor`` drives the GPU, and tests drive the same
scheduler with a fake executor on the CPU.

``run_load`` is the load generator of the serving benchmark: seeded jittered 30 fps arrivals per
stream, streams joining and leaving at a fixed rate, frames replayed from pinned pools.
"""
from __future__ import annotations

import heapq
import math
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _abi

GMM_RGB, GMM_DEPTH = _abi.GMM_RGB, _abi.GMM_DEPTH


@dataclass
class FrameRequest:
    stream_id: int
    seq: int
    t_arrival: float
    rgb: object = None            # host (pinned) uint8 tensor, HWC dense, or None
    depth: object = None          # host (pinned) uint16 tensor, dense, or None
    out_rgb: object = None        # host (pinned) int64 mask words, or None
    out_depth: object = None
    out_fused: object = None
    t_done: float = math.nan
    tick: int = 0


@dataclass
class ServedStream:
    id: int
    width: int
    height: int
    modalities: int
    handle: object
    bytes: int
    queue: deque = field(default_factory=deque)
    in_flight: int = 0           # frames of the stream on the device
    leaving: bool = False

    @property
    def npix(self) -> int:
        return self.width * self.height

    @property
    def pixel_updates(self) -> int:
        return self.npix * ((self.modalities & GMM_RGB != 0) + (self.modalities & GMM_DEPTH != 0))


class Server:
    def __init__(self, executor, hbm_budget_bytes: int, max_queue: int = 8):
        self.x = executor
        self.depth = int(getattr(executor, "frames_in_flight", 1))
        self.budget = int(hbm_budget_bytes)
        self.max_queue = max_queue
        self.streams: Dict[int, ServedStream] = {}
        self.used = 0
        self.next_id = 0
        self.ticks: Dict[int, List[FrameRequest]] = {}
        self.stats = dict(joined=0, rejected=0, left=0, submitted=0, dropped=0, cancelled=0, completed=0,
                          ticks=0, frames_launched=0)

    # -- membership ----------------------------------------------------------------------
    def join(self, width: int, height: int, modalities: int) -> Optional[int]:
        need = self.x.bytes_needed(width, height, modalities)
        if self.used + need > self.budget:
            self.stats["rejected"] += 1
            return None
        handle, nbytes = self.x.open_stream(width, height, modalities)
        sid = self.next_id
        self.next_id += 1
        self.streams[sid] = ServedStream(sid, width, height, modalities, handle, nbytes)
        self.used += nbytes
        self.stats["joined"] += 1
        return sid

    def leave(self, sid: int):
        st = self.streams.get(sid)
        if st is None or st.leaving:
            return
        st.leaving = True
        self.stats["cancelled"] += len(st.queue)
        st.queue.clear()
        self.stats["left"] += 1
        if st.in_flight == 0:
            self._release(st)

    def _release(self, st: ServedStream):
        self.x.close_stream(st.handle)
        self.used -= st.bytes
        del self.streams[st.id]

    # -- frames --------------------------------------------------------------------------
    def submit(self, req: FrameRequest) -> bool:
        st = self.streams.get(req.stream_id)
        if st is None or st.leaving:
            return False
        self.stats["submitted"] += 1
        if len(st.queue) >= self.max_queue:
            self.stats["dropped"] += 1
            return False
        st.queue.append(req)
        return True

    def ready(self) -> List[ServedStream]:
        return [s for s in self.streams.values() if s.in_flight < self.depth and s.queue and not s.leaving]

    def collect(self) -> List[FrameRequest]:
        """Frames of completed ticks (each with t_done and tick set)."""
        done: List[FrameRequest] = []
        for tick, t_done in self.x.poll():
            for req in self.ticks.pop(tick):
                req.t_done = t_done
                done.append(req)
                st = self.streams.get(req.stream_id)
                if st is not None:
                    st.in_flight -= 1
                    if st.leaving and st.in_flight == 0:
                        self._release(st)
        self.stats["completed"] += len(done)
        return done

    def launch_ready(self) -> int:
        batch = self.ready()
        if not batch:
            return 0
        reqs = []
        for st in batch:
            req = st.queue.popleft()
            st.in_flight += 1
            reqs.append((st, req))
        try:
            tick = self.x.launch(reqs)
        except Exception:
            # nothing was enqueued: the frames go back to the head of their queues
            for st, req in reqs:
                st.in_flight -= 1
                st.queue.appendleft(req)
            raise
        for _, req in reqs:
            req.tick = tick
        self.ticks[tick] = [r for _, r in reqs]
        self.stats["ticks"] += 1
        self.stats["frames_launched"] += len(reqs)
        return len(reqs)

    def step(self) -> List[FrameRequest]:
        done = self.collect()
        self.launch_ready()
        return done

    def in_flight(self) -> int:
        return sum(len(v) for v in self.ticks.values())

    def close(self):
        self.x.drain()
        self.collect()
        for st in list(self.streams.values()):
            st.queue.clear()
            if st.in_flight == 0:
                self._release(st)


class Arena:
    """First-fit sub-allocator over one device reservation (offsets only; 256-byte granules).
    Stream memory is carved from it at join and returned at leave, so the serving loop never
    calls the device allocator while it runs."""

    GRAIN = 256

    def __init__(self, size: int):
        self.size = size // self.GRAIN * self.GRAIN
        self.free = [(0, self.size)]           # sorted, coalesced (offset, length)
        self.used = {}                         # offset -> length

    def alloc(self, nbytes: int) -> Optional[int]:
        n = (nbytes + self.GRAIN - 1) // self.GRAIN * self.GRAIN
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    del self.free[i]
                else:
                    self.free[i] = (off + n, ln - n)
                self.used[off] = n
                return off
        return None

    def release(self, off: int):
        n = self.used.pop(off)
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged

    def free_bytes(self) -> int:
        return sum(ln for _, ln in self.free)


class NativeExecutor:
    """The GPU executor (gmm_exec_*). Stream state and frame slots are carved from one device
    reservation of `arena_bytes`, so joins and leaves allocate, free and synchronise nothing."""

    frames_in_flight = 2  # a stream's two device frame slots

    def __init__(self, device: int = 0, ring: int = 4, M: int = 5, state_dtype: str = "f16",
                 tuning: Optional[Tuple[int, int, int]] = None, arena_bytes: int = 1 << 30, **params):
        import torch
        self.device, self.M, self.dtype, self.params = device, M, state_dtype, params
        self.handle = _abi.gmm_exec_create(device, ring)
        if tuning:
            _abi.gmm_exec_set_tuning(self.handle, *tuning)
        self.mem = torch.empty(arena_bytes, dtype=torch.uint8, device=torch.device("cuda", device))
        self.base = self.mem.data_ptr()
        self.arena = Arena(arena_bytes)
        self.offsets = {}

    def _cfg(self, width: int, height: int, modalities: int):
        return _abi.gmm_config_default(width, height, modalities, self.M, state_dtype=_abi.DTYPES[self.dtype],
                                       device=self.device, **self.params)

    def bytes_needed(self, width: int, height: int, modalities: int) -> int:
        return _abi.gmm_exec_stream_bytes(self._cfg(width, height, modalities))

    def open_stream(self, width: int, height: int, modalities: int):
        cfg = self._cfg(width, height, modalities)
        need = _abi.gmm_exec_stream_bytes(cfg)
        off = self.arena.alloc(need)
        if off is None:
            raise MemoryError("executor arena exhausted")
        h = _abi.gmm_exec_create_stream(self.handle, cfg, self.base + off, need)
        self.offsets[h] = off
        return h, need

    def close_stream(self, h):
        _abi.gmm_exec_destroy_stream(self.handle, h)
        self.arena.release(self.offsets.pop(h))

    def launch(self, reqs) -> int:
        items = []
        for st, r in reqs:
            it = _abi.gmm_exec_item()
            it.handle = st.handle
            it.host_rgb = r.rgb.data_ptr() if r.rgb is not None else None
            it.host_depth = r.depth.data_ptr() if r.depth is not None else None
            it.host_fg_rgb = r.out_rgb.data_ptr() if r.out_rgb is not None else None
            it.host_fg_depth = r.out_depth.data_ptr() if r.out_depth is not None else None
            it.host_fused = r.out_fused.data_ptr() if r.out_fused is not None else None
            items.append(it)
        return _abi.gmm_exec_launch(self.handle, items)

    def poll(self):
        out = []
        while True:
            got = _abi.gmm_exec_poll(self.handle, 256)
            out += got
            if len(got) < 256:
                return out

    def drain(self):
        _abi.gmm_exec_drain(self.handle)

    def now(self) -> float:
        return _abi.gmm_exec_now()

    def close(self):
        if self.handle is not None:
            _abi.gmm_exec_drain(self.handle)
            for h in list(self.offsets):
                self.close_stream(h)
            _abi.gmm_exec_destroy(self.handle)
            self.handle = None
            self.mem = None


# ---- load generator --------------------------------------------------------------------------

@dataclass(frozen=True)
class StreamKind:
    width: int
    height: int
    modalities: int
    weight: float


# the serving mix: the batched 64-stream mix scaled up (16:32:8:8 of 320x240 and 640x480 RGB-D,
# 512x424 depth, 1920x1080 colour)
SERVE_MIX = (StreamKind(320, 240, GMM_RGB | GMM_DEPTH, 16), StreamKind(640, 480, GMM_RGB | GMM_DEPTH, 32),
             StreamKind(512, 424, GMM_DEPTH, 8), StreamKind(1920, 1080, GMM_RGB, 8))


def percentile(values: Sequence[float], q: float) -> float:
    if not len(values):
        return math.nan
    return float(np.percentile(np.asarray(values), q))


def percentile_with_drops(values: Sequence[float], n_dropped: int, q: float) -> float:
    """Nearest-rank q-th percentile of the latencies with every dropped frame counted as an
    infinite latency (inf once the dropped share exceeds 100 - q percent)."""
    n = len(values) + n_dropped
    if n == 0:
        return math.nan
    rank = max(1, int(math.ceil(q / 100.0 * n)))
    if rank > len(values):
        return math.inf
    return float(np.sort(np.asarray(values))[rank - 1])


def run_load(server: Server, pools: Dict[Tuple[int, int, int], list], n_streams: int, duration_s: float,
             fps: float = 30.0, jitter: float = 0.2, churn_per_s: float = 1.0, seed: int = 211014938,
             mix: Sequence[StreamKind] = SERVE_MIX, warmup_s: float = 1.0, progress=None,
             mask_alloc=None) -> dict:
    """Drive `server` in real time. pools[(w, h, modalities)] = list of (rgb, depth) pinned host
    frames replayed per stream. Returns latency percentiles (arrival -> masks in host memory) and
    throughput over the measured window (after `warmup_s`). `mask_alloc(n_words)` allocates one
    host mask buffer (default: pinned torch int64)."""
    if mask_alloc is None:
        import torch
        mask_alloc = lambda nw: torch.empty(nw, dtype=torch.int64).pin_memory()
    rng = np.random.default_rng(seed)
    weights = np.array([k.weight for k in mix], float)
    weights /= weights.sum()
    kinds = {}        # sid -> StreamKind
    next_seq = {}
    heap: List[Tuple[float, int]] = []
    masks = {}        # sid -> two sets of pinned mask buffers (alternating by seq)
    t0 = server.x.now()

    def mask_set(k: StreamKind):
        nw = (k.width * k.height + 63) // 64
        mk = lambda on: mask_alloc(nw) if on else None
        both = (k.modalities & GMM_RGB) and (k.modalities & GMM_DEPTH)
        return [(mk(k.modalities & GMM_RGB), mk(k.modalities & GMM_DEPTH), mk(both)) for _ in range(2)]

    spare: Dict[StreamKind, list] = {}   # mask sets made before the run for the streams that join

    def add_stream(now: float) -> bool:
        k = mix[int(rng.choice(len(mix), p=weights))]
        sid = server.join(k.width, k.height, k.modalities)
        if sid is None:
            return False
        kinds[sid] = k
        next_seq[sid] = int(rng.integers(0, 1 << 20))
        masks[sid] = spare[k].pop() if spare.get(k) else mask_set(k)
        heapq.heappush(heap, (now + rng.uniform(0, 1.0 / fps), sid))
        return True

    for _ in range(n_streams):
        if not add_stream(t0):
            break
    # pinned host memory is slow to allocate (pages are locked and mapped for the device): the
    # mask buffers of every stream that may join during the run are made now
    n_joins = int(math.ceil(churn_per_s * duration_s)) + 1 if churn_per_s > 0 else 0
    for k in mix:
        spare[k] = [mask_set(k) for _ in range(n_joins)]
    start = server.x.now()
    # the initial streams' first arrivals count from the start of the run, not from before the
    # joins (which allocate and initialise state for every stream)
    heap = [(t + (start - t0), sid) for t, sid in heap]
    heapq.heapify(heap)
    end = start + duration_s
    measure_from = start + warmup_s
    next_churn = start + (1.0 / churn_per_s if churn_per_s > 0 else math.inf)
    pending_joins = 0
    lat: List[float] = []
    lat_t: List[float] = []       # arrival time of each measured frame, from the start
    drops_at: List[int] = []      # server drop count at each whole second of the run
    gap_max: List[float] = []     # longest pass of the loop below in each second of the run
    churn_s: List[float] = []     # time spent in leaves and joins in each second of the run
    prev = start
    pu_done = 0
    frames_done = 0
    arrived_measured = dropped_measured = 0   # arrivals in the measured window, and those refused
    last_report = start
    while True:
        now = server.x.now()
        if now >= end:
            break
        while len(drops_at) <= int(now - start):
            drops_at.append(server.stats["dropped"])
            gap_max.append(0.0)
            churn_s.append(0.0)
        gap_max[int(now - start)] = max(gap_max[int(now - start)], now - prev)
        prev = now
        # churn: one stream leaves and one joins per period (joins retried until admitted)
        churned = pending_joins > 0
        if now >= next_churn:
            live = [s for s in server.streams if not server.streams[s].leaving]
            if live:
                server.leave(int(rng.choice(live)))
            pending_joins += 1
            next_churn += 1.0 / churn_per_s
            churned = True
        while pending_joins and add_stream(now):
            pending_joins -= 1
        if churned:
            churn_s[int(now - start)] += server.x.now() - now
        # arrivals due
        while heap and heap[0][0] <= now:
            t_arr, sid = heapq.heappop(heap)
            if sid not in server.streams or server.streams[sid].leaving:
                continue
            k = kinds[sid]
            seq = next_seq[sid]
            next_seq[sid] = seq + 1
            pool = pools[(k.width, k.height, k.modalities)]
            rgb, dep = pool[seq % len(pool)]
            o = masks[sid][seq & 1]
            accepted = server.submit(FrameRequest(sid, seq, t_arr, rgb, dep, o[0], o[1], o[2]))
            if t_arr >= measure_from:
                arrived_measured += 1
                dropped_measured += 0 if accepted else 1
            heapq.heappush(heap, (t_arr + rng.uniform(1 - jitter, 1 + jitter) / fps, sid))
        for req in server.step():
            if req.t_arrival >= measure_from:
                lat.append(req.t_done - req.t_arrival)
                lat_t.append(req.t_arrival - start)
                k = kinds[req.stream_id]
                pu_done += k.width * k.height * ((k.modalities & GMM_RGB != 0) + (k.modalities & GMM_DEPTH != 0))
                frames_done += 1
        if progress and now - last_report >= 5.0:
            last_report = now
            # counts only: a percentile over every latency so far would hold the loop up for
            # milliseconds as the list grows
            progress(f"t={now - start:5.1f}s streams={len(server.streams)} in_flight={server.in_flight()} "
                     f"done={frames_done} dropped={server.stats['dropped']}")
    window = end - measure_from
    server.x.drain()
    server.collect()
    drops_at.append(server.stats["dropped"])
    # one entry per second of the measured window (by arrival time): frames completed, their p99
    # latency, frames dropped in that second, and the longest pass of the serving loop (a long
    # pass means the host thread itself was held up)
    timeline = []
    lat_a, lat_ta = np.asarray(lat), np.asarray(lat_t)
    for sec in range(int(math.floor(warmup_s)), int(math.ceil(duration_s))):
        sel = lat_a[(lat_ta >= sec) & (lat_ta < sec + 1)]
        dropped = drops_at[min(sec + 1, len(drops_at) - 1)] - drops_at[min(sec, len(drops_at) - 1)]
        timeline.append({"t": sec, "frames": int(sel.size), "dropped": int(dropped),
                         "p99_ms": round(float(np.percentile(sel, 99)) * 1e3, 3) if sel.size else None,
                         "loop_max_ms": round(gap_max[sec] * 1e3, 3) if sec < len(gap_max) else None,
                         "churn_ms": round(churn_s[sec] * 1e3, 3) if sec < len(churn_s) else None})
    return {
        "streams_target": n_streams,
        "streams_end": len(server.streams),
        "duration_s": duration_s,
        "measured_s": window,
        "frames_completed": frames_done,
        "pixel_updates_per_s": pu_done / window if window > 0 else math.nan,
        "p50_latency_ms": percentile(lat, 50) * 1e3,
        "p99_latency_ms": percentile(lat, 99) * 1e3,
        # over every frame that arrived in the window, a dropped one counting as infinitely late
        "p50_latency_ms_arrivals": percentile_with_drops(lat, dropped_measured, 50) * 1e3,
        "p99_latency_ms_arrivals": percentile_with_drops(lat, dropped_measured, 99) * 1e3,
        "arrived_in_window": arrived_measured,
        "dropped_in_window": dropped_measured,
        "max_latency_ms": (max(lat) * 1e3) if lat else math.nan,
        "stats": dict(server.stats),
        "timeline": timeline,
        "hbm_used_bytes": server.used,
        "hbm_budget_bytes": server.budget,
    }

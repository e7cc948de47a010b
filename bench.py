"""Throughput of the per-frame RGB-D mixture path on one MI355X.

A step is one frame-set of the workload through the whole per-frame path (colour and depth
mixture update and classification, bit-packed masks, List 1 fusion).

Default workload (batch-64): 64 Kinect-shaped streams of uneven size - 16 x 320x240 and
32 x 640x480 colour+depth, 8 x 512x424 depth only, 8 x 1920x1080 colour only - M=5, fp32
state, advanced together by one persistent launch per frame-set, the launches replayed from a
captured hipGraph. The synthetic clip has 120 frames per stream (gain ramp from frame 100,
three moving boxes, 5% depth holes), resident in HBM before timing starts. Step i plays clip
frame W+i; past the clip's end the clip plays backwards, then forwards again, so the sequence of
frames never jumps. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

Other workloads: plain-640x480 (one stream, one fused launch per frame, the single-stream
comparison path; 300-frame clip), precision-256 (256 x 640x480, fp16 state; --state-dtype bf16
or f32 to compare), serve-1024 (the serving loop: p50/p99 latency under arrivals). The
ablations of the plain workload: --rho density and --variant augmented.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
PROFILE_TRAFFIC = {
    "plain-640x480": os.path.join(PROFILES, "traffic_frame_kernel_plain-640x480.json"),
    "batch-64": os.path.join(PROFILES, "traffic_batch_kernel_batch-64.json"),
}
# the sources (and the build script, which holds the compiler flags) of each timed kernel
KERNEL_SOURCES = {
    "frame": ("csrc/gmm_device.hpp", "csrc/gmm_frame.hpp", "csrc/gmm_internal.hpp", "csrc/gmm_kernels.hip",
              "build.py"),
    "batch": ("csrc/gmm_device.hpp", "csrc/gmm_frame.hpp", "csrc/gmm_internal.hpp", "csrc/gmm_batch.hip",
              "build.py"),
}
FRAME_KERNEL_SOURCES = KERNEL_SOURCES["frame"]
MAX_POOL = 16   # host worker processes of the oracle leg (the GPU machine's CPU share for one GPU)


def kernel_source_digest(kind: str = "frame") -> str:
    """Hash of a kernel's code: its sources with comments, blank lines and the whitespace around
    each line removed, so a change of wording alone does not count as a new kernel."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2110_14934_amd")
    for f in KERNEL_SOURCES[kind]:
        text = open(os.path.join(pkg, f), encoding="utf-8").read()
        if f.endswith(".py"):
            text = re.sub(r"(?m)^\s*#.*$", "", text)
        else:
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
        text = "\n".join(line.strip() for line in text.splitlines() if line.strip())
        h.update(text.encode())
    return h.hexdigest()[:16]


def clip_frame(i: int, F: int) -> int:
    """Clip frame of step i when a clip of F frames is played forwards, backwards, forwards ...
    (F-1 -> F-2 at the turn, so consecutive steps never jump)."""
    if F <= 1:
        return 0
    period = 2 * F - 2
    r = i % period
    return r if r < F else period - r


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def bytes_per_frame(npix: int, holes: float, M: int, esize: int) -> float:
    """Bytes of one fused launch on one paired stream when the whole sorted state is read and
    rewritten (the full-rewrite byte model): colour 5*M values and depth 3*M values per pixel,
    read and written (a depth hole leaves its state untouched), the input bytes, one mask bit per
    modality, the fusion state byte read and written and the fused bit."""
    colour = npix * (2 * 5 * M * esize + 3 + 1 / 8)
    depth = npix * (2 + 1 / 8) + (npix - holes) * (2 * 3 * M * esize)
    fusion = npix * (2 + 1 / 8)
    return colour + depth + fusion


def stream_bytes(spec, holes: float, M: int, esize: int, fused: bool) -> float:
    """Full-rewrite bytes of one stream in one batched launch (see bytes_per_frame)."""
    n = spec.npix
    b = 0.0
    if spec.rgb:
        b += n * (2 * 5 * M * esize + 3 + 1 / 8)
    if spec.depth:
        b += n * (2 + 1 / 8) + (n - holes) * (2 * 3 * M * esize)
    if fused:
        b += n * (2 + 1 / 8)
    return b


def io_bytes_per_frame(npix: int, rgb: bool = True, depth: bool = True, fused: bool = True,
                       scaled: bool = True) -> float:
    """Bytes besides the mixture state: input pixels (3 B colour, 2 B depth), one mask bit per
    modality, the pixel's flags byte read and written (List 1 state with fusion; with fp32 state
    (scaled weights) also the depth hole count), and the fused bit."""
    b = 0.0
    if rgb:
        b += npix * (3 + 1 / 8)
    if depth:
        b += npix * (2 + 1 / 8)
    if fused or (depth and scaled):
        b += npix * 2
    if fused:
        b += npix / 8
    return b


def device_copy_gbs(nbytes: float, stream, reps: int) -> float:
    """The practical read+write ceiling next to a launch: GB/s of the library's streaming copy
    kernel reading nbytes/2 and writing nbytes/2 (the bytes of one launch), timed on `stream`."""
    import torch
    from paper_2110_14934_amd import gmm_device_copy
    half = int(nbytes // 2) // 16 * 16
    src = torch.empty(half, dtype=torch.uint8, device=stream.device)
    dst = torch.empty_like(src)
    for _ in range(3):
        gmm_device_copy(dst, src, half, stream)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(reps):
        gmm_device_copy(dst, src, half, stream)
    c1.record(stream)
    torch.cuda.synchronize()
    return 2 * half / (c0.elapsed_time(c1) / reps / 1e3) / 1e9


# ---- the oracle on the host ------------------------------------------------------------------

def _oracle_worker(wl_name, stream_idx, row_lo, row_hi, n_frames, seconds, rho, augmented, barrier, out_q):
    """One host process: the FP64 oracle on rows [row_lo, row_hi) of one stream of the workload,
    cycling its first n_frames frames until `seconds` of oracle work have run. Frame generation
    happens before the barrier and is not timed."""
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    import numpy as np
    import torch
    torch.set_num_threads(1)
    from oracle import MixParams, MixtureOracle, FusionOracle, AugmentedOracle
    from paper_2110_14934_amd.synth import Stream, workload
    wl = workload(wl_name)
    spec, mix = wl.streams[stream_idx], wl.mix
    st = Stream(spec)
    pix = torch.arange(row_lo * spec.width, row_hi * spec.width, dtype=torch.int64)
    n = int(pix.numel())
    frames = []
    for t in range(n_frames):
        rgb = st.rgb(t, pix=pix).numpy() if spec.rgb else None
        dep = st.depth(t, pix=pix).numpy() if spec.depth else None
        frames.append((rgb, dep))
    pc = MixParams(mix.M, mix.alpha, mix.k, mix.T, mix.sigma0_rgb, mix.var_min_rgb, mix.w_init, rho=rho)
    pd = MixParams(mix.M, mix.alpha, mix.k, mix.T, mix.sigma0_depth, mix.var_min_depth, mix.w_init,
                   hole_skip=True, rho=rho)
    if augmented:
        aug = AugmentedOracle(MixParams(mix.M, mix.alpha, mix.k, mix.T, mix.sigma0_rgb, mix.var_min_rgb,
                                        mix.w_init, hole_skip=True, rho=rho), n)
    col = MixtureOracle(pc, 3, n) if spec.rgb and not augmented else None
    dep_o = MixtureOracle(pd, 1, n) if spec.depth and not augmented else None
    fus = FusionOracle(n) if spec.rgb and spec.depth and not augmented else None
    if barrier is not None:
        barrier.wait()
    t0 = time.perf_counter()
    done = pu = 0
    while True:
        rgb, dep = frames[done % n_frames]
        if augmented:
            aug.step(rgb, dep)
            pu += n
        else:
            ic = col.step(rgb) if col is not None else None
            idd = dep_o.step(dep) if dep_o is not None else None
            if fus is not None:
                fus.step(ic.fg, idd.fg)
            pu += n * (int(col is not None) + int(dep_o is not None))
        done += 1
        if time.perf_counter() - t0 >= seconds:
            break
    out_q.put((stream_idx, row_lo, row_hi, pu, done, t0, time.perf_counter()))


def _run_oracle_pool(jobs, n_frames, seconds, rho, augmented):
    """Run the oracle jobs [(workload, stream, row_lo, row_hi)] in parallel host processes that
    start their timed loops together; returns (pixel-updates, wall seconds, per-job results)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")   # fresh interpreters: nothing of this process's GPU state
    barrier = ctx.Barrier(len(jobs))
    q = ctx.Queue()
    procs = [ctx.Process(target=_oracle_worker, args=(*job, n_frames, seconds, rho, augmented, barrier, q))
             for job in jobs]
    for p in procs:
        p.start()
    res = [q.get() for _ in procs]
    for p in procs:
        p.join()
    if any(p.exitcode != 0 for p in procs):
        raise RuntimeError("an oracle worker failed")
    pu = sum(r[3] for r in res)
    wall = max(r[6] for r in res) - min(r[5] for r in res)
    return pu, wall, res


def cpu_baseline(wl_name: str, seconds: float, rho: str = "alpha", augmented: bool = False,
                 n_frames: int = 2):
    """The FP64 oracle timed on the host: one core, then every core of the process's share (at
    most MAX_POOL), each process stepping its own part of the workload."""
    from paper_2110_14934_amd.synth import workload
    wl = workload(wl_name)
    P = max(1, min(MAX_POOL, host_cores()))
    streams = wl.streams
    if len(streams) == 1:
        # one stream: the processes take row blocks of it
        sp = streams[0]
        edges = [sp.height * i // P for i in range(P + 1)]
        jobs = [(wl_name, 0, edges[i], edges[i + 1]) for i in range(P) if edges[i + 1] > edges[i]]
        one = [(wl_name, 0, 0, sp.height)]
        what = f"row blocks of the {sp.width}x{sp.height} stream"
    else:
        # streams spread evenly over the workload's list (which is grouped by kind), so the
        # sample keeps the mix's proportions of shapes and modalities
        picks = sorted({len(streams) * i // P for i in range(P)})
        jobs = [(wl_name, s, 0, streams[s].height) for s in picks]
        # one core: the most common shape of the mix
        shapes = [(s.width, s.height, s.rgb, s.depth) for s in streams]
        common = max(set(shapes), key=shapes.count)
        one = [(wl_name, shapes.index(common), 0, common[1])]
        kinds = {}
        for s in picks:
            sp = streams[s]
            k = f"{sp.width}x{sp.height} {'rgb+d' if sp.rgb and sp.depth else ('rgb' if sp.rgb else 'depth')}"
            kinds[k] = kinds.get(k, 0) + 1
        what = "streams " + ", ".join(f"{v} x {k}" for k, v in kinds.items())
    pu1, wall1, _ = _run_oracle_pool(one, n_frames, seconds, rho, augmented)
    pun, walln, _ = _run_oracle_pool(jobs, n_frames, seconds, rho, augmented)
    model = "four-channel mixture" if augmented else "colour and/or depth mixture + fusion"
    return {"value": pun / walln, "unit": "pixel-updates/s", "cores": len(jobs), "kind": "oracle",
            "sample": f"{len(jobs)} host processes, one per part: {what} of {wl_name}, whole parts, "
                      f"frames 0-{n_frames - 1} cycled, {model}, rho={rho}, float64 NumPy, one thread "
                      f"each, {walln:.1f} s wall",
            "one_core": {"value": pu1 / wall1, "cores": 1,
                         "sample": f"one {streams[one[0][1]].width}x{streams[one[0][1]].height} stream "
                                   f"of {wl_name}, {wall1:.1f} s"},
            "host_cpus": os.cpu_count(), "host_cores_available": host_cores(), "cpu_model": cpu_model()}


# ---- timed replay of a prepared step sequence ------------------------------------------------

def _capture(torch, stream, launches):
    """A hipGraph of the given launch callables, in order, on `stream` (captures execute nothing)."""
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for f in launches:
            f(torch.cuda.current_stream())
    torch.cuda.synchronize()
    return g


def _graph_plan(torch, stream, step_fn, W, K, F, max_nodes=1024):
    """Graphs that replay steps W .. W+K-1 (step i plays clip frame clip_frame(i, F)). The frame
    sequence is periodic with period 2F-2, so one graph of a whole period (or of K steps, when
    K is small) is replayed whole, and one more graph holds the remainder."""
    period = max(1, 2 * F - 2)
    if K <= max_nodes:
        return [(_capture(torch, stream, [lambda s, i=i: step_fn(W + i, s) for i in range(K)]), 1)]
    plan = []
    full, rem = divmod(K, period)
    if full:
        plan.append((_capture(torch, stream, [lambda s, i=i: step_fn(W + i, s) for i in range(period)]), full))
    if rem:
        plan.append((_capture(torch, stream, [lambda s, i=i: step_fn(W + i, s) for i in range(rem)]), 1))
    return plan


def _replay(torch, stream, plan):
    with torch.cuda.stream(stream):
        for g, reps in plan:
            for _ in range(reps):
                g.replay()


def _traffic(wl_name: str, kind: str):
    path = PROFILE_TRAFFIC.get(wl_name)
    if path is None or not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    if rec.get("kernel_source_digest") != kernel_source_digest(kind):
        return None, rec
    return rec.get("hbm_bytes_per_launch"), rec


# ---- batched workloads -------------------------------------------------------------------------

def _frames_file_layout(wl):
    """Byte layout of one frame-set of the workload in a frames file: per stream, the colour
    frame (H*W*3 bytes) then the depth frame (H*W*2 bytes), for the modalities present."""
    lay, off = [], 0
    for sp in wl.streams:
        r = (off, sp.npix * 3) if sp.rgb else None
        off += sp.npix * 3 if sp.rgb else 0
        d = (off, sp.npix * 2) if sp.depth else None
        off += sp.npix * 2 if sp.depth else 0
        lay.append((r, d))
    return lay, off


def bench_batch(args) -> int:
    """Many streams, one persistent launch per frame-set, replayed from captured hipGraphs."""
    import numpy as np
    import torch
    from paper_2110_14934_amd import _abi, Segmenter, Batch, GMM_RGB, GMM_DEPTH
    from paper_2110_14934_amd.synth import Stream, workload

    wl = workload(args.workload)
    dtype = args.state_dtype or wl.state_dtype
    esize = 4 if dtype == "f32" else 2
    M = wl.mix.M
    K, W = args.steps, args.warmup
    F = args.clip or wl.frames
    # the clip frames the run plays: warm-up, timed steps (and their replay with the record on)
    used = sorted({clip_frame(i, F) for i in range(W + K)})
    streams = [Stream(sp) for sp in wl.streams]
    lay, fs_bytes = _frames_file_layout(wl)

    if args.save_frames:
        # frames of every used clip frame, generated on the host, one file per frame-set
        os.makedirs(args.save_frames, exist_ok=True)
        for t in used:
            buf = np.empty(fs_bytes, dtype=np.uint8)
            for st, (r, d) in zip(streams, lay):
                if r:
                    buf[r[0]:r[0] + r[1]] = st.rgb(t, device=args.gen_device).cpu().numpy().reshape(-1)
                if d:
                    buf[d[0]:d[0] + d[1]] = st.depth(t, device=args.gen_device).cpu().numpy().reshape(-1).view(np.uint8)
            np.save(os.path.join(args.save_frames, f"frames_{t:04d}.npy"), buf)
            print(f"[bench] saved frame-set {t}", file=sys.stderr, flush=True)
        return 0

    if torch.cuda.device_count() < 1:   # counts devices without initialising them
        print("no GPU visible", file=sys.stderr)
        return 1
    if not os.path.exists(_abi.LIB_PATH):
        raise SystemExit("libgmm.so is not built: run __graft_entry__.build() first")

    cpu = None
    if not args.no_cpu_baseline:
        # before any GPU work: the oracle runs in fresh interpreters started by this process
        cpu = cpu_baseline(args.workload, args.cpu_seconds)
        print(f"[bench] oracle on the host: {cpu['value']:.4g} pu/s on {cpu['cores']} processes",
              file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    frames, holes = {}, {}
    for n_done, t in enumerate(used):
        fs, hs = [], []
        if args.load_frames:
            buf = np.load(os.path.join(args.load_frames, f"frames_{t:04d}.npy"), mmap_mode="r")
        for st, (r, d) in zip(streams, lay):
            sp = st.spec
            if args.load_frames:
                rgb = (torch.from_numpy(np.array(buf[r[0]:r[0] + r[1]])).reshape(sp.height, sp.width, 3).to(dev)
                       if r else None)
                dh = np.array(buf[d[0]:d[0] + d[1]]).view(np.uint16) if d else None
                dep = torch.from_numpy(dh).reshape(sp.height, sp.width).to(dev) if d else None
                hs.append(float((dh == 0).sum()) if d else 0.0)   # counted on the host
            else:
                rgb = st.rgb(t, device=dev) if sp.rgb else None
                dep = st.depth(t, device=dev) if sp.depth else None
                hs.append((dep == 0).sum() if dep is not None else torch.zeros((), device=dev, dtype=torch.int64))
            fs.append((rgb, dep))
        frames[t] = fs
        holes[t] = hs if args.load_frames else torch.stack(hs)
        if n_done % 20 == 19:
            print(f"[bench] {n_done + 1}/{len(used)} frame-sets resident", file=sys.stderr, flush=True)
    holes = {t: (np.asarray(h, dtype=np.float64) if args.load_frames else h.to(torch.float64).cpu().numpy())
             for t, h in holes.items()}
    torch.cuda.synchronize()
    print(f"[bench] {len(streams)} streams x {len(used)} frame-sets resident on {torch.cuda.get_device_name(0)}",
          file=sys.stderr, flush=True)

    segs = []
    for sp in wl.streams:
        mods = (GMM_RGB if sp.rgb else 0) | (GMM_DEPTH if sp.depth else 0)
        segs.append(Segmenter(sp.width, sp.height, mods, M, state_dtype=dtype))
    slot_of = {t: k for k, t in enumerate(used)}
    batch = Batch(segs, n_slots=len(used))
    stream = torch.cuda.Stream()
    for t in used:
        batch.set_frames(slot_of[t], frames[t], stream=stream)
    stream.synchronize()

    def step(i, s):
        batch.run(slot_of[clip_frame(i, F)], s)

    with torch.cuda.stream(stream):
        for i in range(W):
            step(i, stream)
    stream.synchronize()
    tune_ms = None
    if args.tuning:
        batch.set_tuning(*args.tuning)
    elif not args.no_autotune:
        # trial launches on the next frame-sets from the current state, which is restored after
        best, tune_ms = batch.autotune(slot_of[clip_frame(W, F)], stream)
        print(f"[bench] autotuned {best}: {tune_ms:.3f} ms per launch", file=sys.stderr, flush=True)

    plan = _graph_plan(torch, stream, step, W, K, F)
    if args.calibrate_copy:
        from paper_2110_14934_amd import gmm_device_copy
        nb = args.calibrate_copy << 20
        src = torch.empty(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        gmm_device_copy(dst, src, nb, stream)   # reads and writes MIB MiB each
        torch.cuda.synchronize()
        del src, dst
    # the state before the timed steps, to replay them with the traffic record on
    snaps = [torch.empty(sg.state_bytes(), dtype=torch.uint8, device=dev) for sg in segs]
    for sg, sn in zip(segs, snaps):
        sg.save_state(sn, stream)
    torch.cuda.synchronize()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    _replay(torch, stream, plan)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / K
    print(f"[bench] timed {K} steps: {ms_total:.3f} ms", file=sys.stderr, flush=True)

    # the same K steps from the same state with the per-wave traffic records attached (the
    # descriptor slots carry the record pointers, so they are prepared again)
    records = [torch.from_numpy(np.zeros((sg.npix + 63) // 64, dtype=np.int64)).to(dev) for sg in segs]
    for sg, rec in zip(segs, records):
        _abi.gmm_set_traffic_record(sg.handle, rec)
    for sg, sn in zip(segs, snaps):
        sg.restore_state(sn, stream)
    for t in used:
        batch.set_frames(slot_of[t], frames[t], stream=stream)
    # captured again: a launch picks the counting kernel from the descriptors prepared before it
    plan_rec = _graph_plan(torch, stream, step, W, K, F)
    _replay(torch, stream, plan_rec)
    torch.cuda.synchronize()
    del plan_rec
    for sg in segs:
        _abi.gmm_set_traffic_record(sg.handle, None)
    for t in used:   # the descriptors again without the records
        batch.set_frames(slot_of[t], frames[t], stream=stream)
    stream.synchronize()

    pu_step = sum(sp.npix * (int(sp.rgb) + int(sp.depth)) for sp in wl.streams)
    value = pu_step * K / (ms_total / 1e3)
    timed = [clip_frame(W + i, F) for i in range(K)]
    mean_holes = np.mean([holes[t] for t in timed], axis=0)
    full = sum(stream_bytes(sp, float(mean_holes[i]), M, esize, sp.rgb and sp.depth)
               for i, sp in enumerate(wl.streams))
    state = float(sum(int(r.sum().item()) for r in records)) / K
    alg = state + sum(io_bytes_per_frame(sp.npix, sp.rgb, sp.depth, sp.rgb and sp.depth, dtype == "f32")
                      for sp in wl.streams)
    achieved = alg / (ms_step / 1e3) / 1e9
    copy_gbs = device_copy_gbs(alg, stream, reps=20)
    traffic, trec = _traffic(args.workload, "batch") if dtype == "f32" else (None, None)
    out = {
        "metric": "RGBD GMM pixel-updates/s", "value": value, "unit": "pixel-updates/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Kinect-shaped RGB-D streams; the paper's captures are not available)",
        "config": {"workload": args.workload, "streams": len(wl.streams), "M": M, "state_dtype": dtype,
                   "clip_frames": F, "timed_clip_frames": f"{timed[0]}..{timed[-1]} (steps {W}..{W + K - 1}, "
                                                          f"clip played forwards then backwards)",
                   "launch": "graph", "tuning": list(batch.tuning()), "autotune_ms": tune_ms},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"rgbd::batch_kernel<{M}, {dtype}, {batch.tuning()[0]}, false>",
                     "algorithmic_bytes_per_launch": alg, "full_rewrite_bytes_per_launch": full,
                     "full_rewrite_frac": full / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "avg_launch_us": ms_step * 1e3,
                     "device_copy_same_bytes_gbs": copy_gbs,
                     "frac_of_device_copy": achieved / copy_gbs,
                     "traffic_record": None if trec is None else {
                         "digest_matches": traffic is not None, "workload_window": trec.get("dispatch_window"),
                         "algorithmic_bytes_same_run": trec.get("algorithmic_bytes_per_launch_same_run")}},
        "state_bytes": sum(sg.state_bytes() for sg in segs),
        "paper_context": {"value": 2 * 640 * 480 * 30, "unit": "pixel-updates/s",
                          "note": "30 fps VGA colour+depth end to end incl. transfers, unnamed GPU (Sec. V.B)"},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    batch.close()
    for sg in segs:
        sg.close()
    print(json.dumps(out), flush=True)
    return 0


def h2d_ceiling(pools, mix, n_streams: int, fps: float = 30.0, copy_streams: int = 4, reps: int = 3) -> dict:
    """Host->device rate of one frame of every stream of the serving mix (in the mix's
    proportions, n_streams in all), copied from the pinned frame pools over `copy_streams`
    streams as the executor copies them; beside it the rate that 30 frames per second of every
    stream need."""
    import torch
    total_w = sum(k.weight for k in mix)
    plan = []
    for k in mix:
        cnt = int(round(n_streams * k.weight / total_w))
        pool = pools[(k.width, k.height, k.modalities)]
        plan += [pool[i % len(pool)] for i in range(cnt)]
    nbytes = sum(sum(t.numel() * t.element_size() for t in f if t is not None) for f in plan)
    npu = sum(sum(t.shape[0] * t.shape[1] for t in f if t is not None) for f in plan)
    big = max(t.numel() * t.element_size() for f in plan for t in f if t is not None)
    dev = torch.device("cuda", 0)
    dst = [torch.empty(big, dtype=torch.uint8, device=dev) for _ in range(copy_streams)]
    streams = [torch.cuda.Stream() for _ in range(copy_streams)]
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        i = 0
        for f in plan:
            for t in f:
                if t is None:
                    continue
                j = i % copy_streams
                with torch.cuda.stream(streams[j]):
                    dst[j][:t.numel() * t.element_size()].copy_(t.reshape(-1).view(torch.uint8), non_blocking=True)
                i += 1
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    # the link itself: the same bytes as copy_streams large copies from pinned memory, one per
    # stream (no per-frame issue cost)
    part = (nbytes + copy_streams - 1) // copy_streams
    hsrc = [torch.empty(part, dtype=torch.uint8, pin_memory=True) for _ in range(copy_streams)]
    ddst = [torch.empty(part, dtype=torch.uint8, device=dev) for _ in range(copy_streams)]
    bulk = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(copy_streams):
            with torch.cuda.stream(streams[j]):
                ddst[j].copy_(hsrc[j], non_blocking=True)
        torch.cuda.synchronize()
        bulk = min(bulk, time.perf_counter() - t0)
    return {"per_frame_copies_gbs": nbytes / best / 1e9, "bulk_copies_gbs": copy_streams * part / bulk / 1e9,
            "demand_gbs": nbytes * fps / 1e9, "bytes_per_frame_set": nbytes, "pixel_updates_per_frame_set": npu,
            "streams": len(plan),
            "copy_streams": copy_streams,
            "note": "best of 3 rounds; per-frame: one async copy per frame of every stream from the pinned "
                    "pools, issued from Python; bulk: the same bytes in one copy per copy stream"}


def bench_serve(args) -> int:
    """The serving loop: jittered 30 fps arrivals on many resident streams, joins and leaves at
    1/s under a memory budget, continuous batching through the executor; p50/p99 latency."""
    import torch
    from paper_2110_14934_amd import _abi, GMM_RGB, GMM_DEPTH
    from paper_2110_14934_amd.serve import NativeExecutor, Server, run_load, SERVE_MIX
    from paper_2110_14934_amd.synth import Stream, StreamSpec

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    if not os.path.exists(_abi.LIB_PATH):
        raise SystemExit("libgmm.so is not built: run __graft_entry__.build() first")
    dtype = args.state_dtype or "f16"
    pools = {}
    for i, k in enumerate(SERVE_MIX):   # 8 distinct frames per stream kind, pinned host memory
        rgb, dep = bool(k.modalities & GMM_RGB), bool(k.modalities & GMM_DEPTH)
        st = Stream(StreamSpec(k.width, k.height, rgb=rgb, depth=dep, n_boxes=3, box_min=40, box_max=120,
                               speed_min=1, speed_max=4, hole_p=0.05, seed=211014938, index=i))
        pools[(k.width, k.height, k.modalities)] = [
            (st.rgb(t).contiguous().pin_memory() if rgb else None,
             st.depth(t).contiguous().pin_memory() if dep else None) for t in range(8)]
    h2d = h2d_ceiling(pools, SERVE_MIX, args.serve_streams)
    print(f"[serve] host->device: {h2d['bulk_copies_gbs']:.1f} GB/s in large copies, "
          f"{h2d['per_frame_copies_gbs']:.1f} GB/s frame by frame; demand at 30 fps "
          f"{h2d['demand_gbs']:.1f} GB/s", file=sys.stderr, flush=True)
    budget = int(args.serve_budget_gb * (1 << 30))
    ex = NativeExecutor(ring=4, state_dtype=dtype, tuning=(256, 1024, 4), arena_bytes=budget)
    srv = Server(ex, budget, max_queue=8)
    prog = lambda m: print("[serve] " + m, file=sys.stderr, flush=True)
    try:
        rep = run_load(srv, pools, n_streams=args.serve_streams, duration_s=args.serve_seconds,
                       churn_per_s=args.serve_churn, warmup_s=min(args.serve_warmup, args.serve_seconds / 4),
                       progress=prog)
    finally:
        srv.close()
        ex.close()
    # host->device bytes the served frames moved per second over the measured window
    pu_per_byte = h2d["pixel_updates_per_frame_set"] / h2d["bytes_per_frame_set"]
    h2d["served_gbs"] = rep["pixel_updates_per_s"] / pu_per_byte / 1e9
    out = {
        "metric": "RGBD GMM pixel-updates/s", "value": rep["pixel_updates_per_s"], "unit": "pixel-updates/s",
        "n_gpus": 1, "steps": rep["frames_completed"], "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Kinect-shaped streams replayed from pinned pools)",
        "config": {"workload": "serve-1024", "streams": args.serve_streams, "state_dtype": dtype,
                   "seconds": args.serve_seconds, "warmup_s": min(args.serve_warmup, args.serve_seconds / 4),
                   "budget_gb": args.serve_budget_gb, "churn_per_s": args.serve_churn},
        "latency_ms": {"p50": rep["p50_latency_ms"], "p99": rep["p99_latency_ms"], "max": rep["max_latency_ms"],
                       "p99_per_second_max_after_5s": max((e["p99_ms"] or 0.0) for e in rep["timeline"] if e["t"] >= 5)
                       if any(e["t"] >= 5 for e in rep["timeline"]) else None,
                       "p99_over_arrivals": rep["p99_latency_ms_arrivals"],
                       "dropped_in_window": rep["dropped_in_window"], "arrived_in_window": rep["arrived_in_window"]},
        "h2d": h2d,
        "serve": rep,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_plain(args) -> int:
    """One stream, one fused launch per frame (the single-stream comparison path)."""
    import numpy as np
    import torch
    from paper_2110_14934_amd import _abi, Segmenter, GMM_RGB, GMM_DEPTH
    from paper_2110_14934_amd.synth import Stream, workload

    if torch.cuda.device_count() < 1:
        print("no GPU visible", file=sys.stderr)
        return 1
    if not os.path.exists(_abi.LIB_PATH):
        raise SystemExit("libgmm.so is not built: run __graft_entry__.build() first")
    wl = workload(args.workload)
    spec, mix = wl.streams[0], wl.mix
    st = Stream(spec)
    F = args.clip or wl.frames
    n = spec.npix
    K, W = args.steps, args.warmup
    augmented = args.variant == "augmented"

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, args.cpu_seconds, args.rho, augmented)

    dev = torch.device("cuda", 0)
    used = sorted({clip_frame(i, F) for i in range(W + K)})
    if args.host_frames:   # built on the host: the GPU then runs little besides the path itself
        rgbs = {t: st.rgb(t).to(dev) for t in used}
        dh = {t: st.depth(t) for t in used}
        holes = {t: float((dh[t] == 0).sum()) for t in used}
        deps = {t: dh[t].to(dev) for t in used}
    else:
        rgbs = {t: st.rgb(t, device=dev) for t in used}
        deps = {t: st.depth(t, device=dev) for t in used}
        holes = {t: float((deps[t] == 0).sum().item()) for t in used}
    torch.cuda.synchronize()
    print(f"[bench] {len(used)} frames of {spec.width}x{spec.height} resident on {torch.cuda.get_device_name(0)}",
          file=sys.stderr, flush=True)

    seg = Segmenter(spec.width, spec.height, GMM_RGB | GMM_DEPTH, mix.M, state_dtype=wl.state_dtype,
                    rho=args.rho, augmented=augmented)

    def step(i, s):
        t = clip_frame(i, F)
        if augmented:
            seg.apply_augmented(rgbs[t], deps[t], s)
        else:
            seg.apply_fused(rgbs[t], deps[t], s)

    record = torch.from_numpy(np.zeros((n + 63) // 64, dtype=np.int64)).to(dev)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for i in range(W):
            step(i, stream)
    stream.synchronize()

    def plan_with(rec):
        # kernel arguments (the record pointer among them) are fixed at capture
        _abi.gmm_set_traffic_record(seg.handle, rec)
        p = _graph_plan(torch, stream, step, W, K, F)
        _abi.gmm_set_traffic_record(seg.handle, None)
        return p

    def run_steps(plan, rec):
        if plan is not None:
            _replay(torch, stream, plan)
        else:
            _abi.gmm_set_traffic_record(seg.handle, rec)
            with torch.cuda.stream(stream):
                for i in range(K):
                    step(W + i, stream)
            _abi.gmm_set_traffic_record(seg.handle, None)

    plan = plan_rec = None
    if args.mode == "graph":
        plan = plan_with(None)
        plan_rec = plan_with(record)

    if args.calibrate_copy:
        from paper_2110_14934_amd import gmm_device_copy
        nb = args.calibrate_copy << 20
        src = torch.empty(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        gmm_device_copy(dst, src, nb, stream)   # reads and writes MIB MiB each
        torch.cuda.synchronize()
        del src, dst

    snap = torch.empty(seg.state_bytes(), dtype=torch.uint8, device=dev)
    seg.save_state(snap, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    run_steps(plan, None)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / K
    print(f"[bench] timed {K} steps: {ms_total:.2f} ms", file=sys.stderr, flush=True)

    # the same K steps again from the same state, recording the state traffic of every launch
    seg.restore_state(snap, stream)
    run_steps(plan_rec, record)
    torch.cuda.synchronize()

    pu_step = (1 if augmented else 2) * n
    value = pu_step * K / (ms_total / 1e3)
    timed = [clip_frame(W + i, F) for i in range(K)]
    mean_holes = float(np.mean([holes[t] for t in timed]))
    esize = 4 if wl.state_dtype == "f32" else 2
    sorted_bytes = bytes_per_frame(n, mean_holes, mix.M, esize)
    state_bytes = float(record.sum().item()) / K
    # augmented: colour and depth inputs, one mask, no fusion state
    alg_bytes = state_bytes + (n * (3 + 2 + 1 / 8) if augmented else io_bytes_per_frame(n))
    achieved = alg_bytes / (ms_step / 1e3) / 1e9
    copy_gbs = device_copy_gbs(alg_bytes, stream, reps=200)
    traffic = None
    if not augmented and args.rho == "alpha":
        traffic, _ = _traffic(args.workload, "frame")

    out = {
        "metric": "RGBD GMM pixel-updates/s", "value": value, "unit": "pixel-updates/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Kinect-shaped RGB-D stream; the paper's captures are not available)",
        "config": {"workload": args.workload, "streams": 1, "width": spec.width, "height": spec.height,
                   "M": mix.M, "modalities": "rgb+depth (one 4-channel mixture)" if augmented else "rgb+depth+fusion",
                   "state_dtype": wl.state_dtype, "clip_frames": F,
                   "timed_clip_frames": f"{timed[0]}..{timed[-1]} (steps {W}..{W + K - 1}, clip played forwards "
                                        f"then backwards)",
                   "launch": args.mode, "rho": args.rho, "variant": args.variant},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     # the single-stream kernel streams its rows and frames (cache policy 2) for
                     # a state of 128 MiB or more, else keeps the default policy (0)
                     "kernel": f"rgbd::frame_kernel<5, float, {8 if augmented else 7}, "
                               f"{2 if seg.state_bytes() >= 128 << 20 else 0}>",
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "full_rewrite_bytes_per_launch": None if augmented else sorted_bytes,
                     "full_rewrite_frac": None if augmented else sorted_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "avg_launch_us": ms_step * 1e3,
                     "device_copy_same_bytes_gbs": copy_gbs},
        "frames_per_s": 1e3 / ms_step,
        "paper_context": {"value": 2 * 640 * 480 * 30, "unit": "pixel-updates/s",
                          "note": "30 fps VGA colour+depth end to end incl. transfers, unnamed GPU (Sec. V.B)"},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    seg.close()
    print(json.dumps(out), flush=True)
    return 0


def _tuning(s: str):
    parts = tuple(int(v) for v in s.split(","))
    if len(parts) != 3:
        raise argparse.ArgumentTypeError("--tuning takes block_threads,tile_pixels,blocks_per_cu")
    return parts


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=240)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batch-64",
                    choices=("batch-64", "plain-640x480", "precision-256", "serve-1024"))
    ap.add_argument("--mode", choices=("graph", "eager"), default="graph",
                    help="plain workload - graph: replay captured hipGraphs; eager: one launch per call")
    ap.add_argument("--state-dtype", choices=("f32", "f16", "bf16"), default=None,
                    help="override the workload's mixture-state storage type (batched workloads)")
    ap.add_argument("--clip", type=int, default=0, help="clip length in frames (default: the workload's)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning", type=_tuning, default=None, metavar="B,T,C",
                    help="batched workloads: fixed launch shape instead of the autotuner's")
    ap.add_argument("--save-frames", default=None, metavar="DIR",
                    help="batched workloads: write the frame-sets the run would play to DIR and exit")
    ap.add_argument("--load-frames", default=None, metavar="DIR",
                    help="batched workloads: read the frame-sets from DIR (written by --save-frames) instead "
                         "of generating them on the GPU (few GPU dispatches besides the path: counter runs)")
    ap.add_argument("--gen-device", default="cpu", help="device that generates frames for --save-frames")
    ap.add_argument("--serve-seconds", type=float, default=20.0, help="serving run length")
    ap.add_argument("--serve-streams", type=int, default=1024, help="resident streams at the start")
    ap.add_argument("--serve-budget-gb", type=float, default=48.0, help="device memory budget for admission")
    ap.add_argument("--serve-churn", type=float, default=1.0, help="streams leaving (and joining) per second")
    ap.add_argument("--serve-warmup", type=float, default=2.0,
                    help="seconds before the measured window (every initial stream joins at the start, and "
                         "the first frame of a stream takes the general path at every pixel)")
    ap.add_argument("--rho", choices=("alpha", "density"), default="alpha",
                    help="rate of the mean and variance updates (plain workload)")
    ap.add_argument("--variant", choices=("separate", "augmented"), default="separate",
                    help="separate colour and depth models + List 1 (the method), or one four-channel model")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="oracle work per leg (one core, then all cores) of the host baseline")
    ap.add_argument("--host-frames", action="store_true",
                    help="plain workload: build the frames on the host (few GPU dispatches besides the path)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one library copy of MIB MiB (counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: there is no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        return 2
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        return 2
    if args.workload in ("batch-64", "precision-256"):
        return bench_batch(args)
    if args.workload == "serve-1024":
        return bench_serve(args)
    return bench_plain(args)


if __name__ == "__main__":
    sys.exit(main())

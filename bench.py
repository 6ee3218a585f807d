#!/usr/bin/env python
"""Benchmark of the point-rasterization hot path on one MI355X.

Default workload: 2,000,000,000 points of the seeded terrain generator,
Morton-sorted into batches of 10,240, rendered as a stereo pair of
2 x 2016 x 2240 (one launch per eye, adaptive 10/20/30-bit precision, batch
frustum culling).  One step = one stereo frame = for each eye: clear, render,
resolve.  Inputs are resident in HBM before the timed region; the load-time
build (Morton sort, batch boxes, Eq. 1 split) is timed separately.

Metric (paper's convention, Sec. 4.1): processed points / frame time, where
processed points are the points of batches that were not culled (Table 2).

Prints ONE JSON line.  Also reports the render kernel against the HBM roofline
(algorithmic bytes per launch / measured launch duration) and the CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpoints/s rendered + achieved HBM GB/s; p50/p99 frame latency in served mode"
HBM_PEAK_GBS = 8000.0
# plain (unpacked) VALU issue: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per SIMD every 4 cycles
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name: str, n_override: int | None):
    import synth

    if name == "c3":
        n = n_override or 2_000_000_000
        cams = synth.stereo_cameras(synth.C3_SEED)
        # morton 2 = PR_ORDER_MORTON_SPREAD: the Morton batches, each stored in the spread order
        return dict(name="terrain_2e9_stereo_2x2016x2240", seed=synth.C3_SEED, n=n, morton=2, order=0,
                    cams=cams, desc=f"terrain {n} points, Morton-sorted 10240-point batches (each stored in the "
                                    f"spread order), stereo pair 2x2016x2240, one launch per eye, adaptive "
                                    f"precision, culling on")
    if name == "c2":
        n = n_override or 100_000_000
        cams = [synth.orbit_camera(f) for f in range(0, 60, 15)]
        return dict(name="terrain_1e8_orbit_1920x1080", seed=synth.C2_SEED, n=n, morton=2, order=1, cams=cams,
                    desc=f"terrain {n} points, Morton batches in the spread order, orbit frames 0/15/30/45 at "
                         f"1920x1080")
    if name == "c1":
        n = n_override or 1_000_000
        return dict(name="primitives_1e6_1280x720", seed=synth.C1_SEED, n=n, morton=False, order=0,
                    cams=[synth.c1_camera()], desc=f"8 primitives {n} points, 1280x720")
    raise SystemExit(f"unknown workload {name}")


def _wait(pending):
    if pending is not None and hasattr(pending, "result"):
        pending.result()


def load_cloud(ctx, wl, chunk=64_000_000, on_chunk=None):
    """Generate the cloud on the host in chunks (pinned, double-buffered) and stream it to HBM.

    on_chunk(lo, hi, xyz, rgba), if given, sees every generated chunk (numpy views of points [lo, hi) in input
    order) before it is uploaded; if it returns an object with .result(), that is waited for before the chunk's
    host buffer is reused."""
    import numpy as np
    import torch
    import paper_2204_01287_amd as pr
    import synth

    n, S, morton = wl["n"], wl.get("batch_size", 10240), wl["morton"]
    sizes = pr.pr_cloud_sizes(n, S, morton)
    dev = torch.device("cuda", 0)
    mem = {f: torch.empty(max(getattr(sizes, f), 256), dtype=torch.uint8, device=dev) for f in pr.DeviceCloud.FIELDS}
    bufs = pr.CloudBufs(*[mem[f].data_ptr() for f in pr.DeviceCloud.FIELDS], sizes)
    t0 = time.perf_counter()
    if wl["name"].startswith("primitives"):
        xyz, rgba = synth.primitives(wl["seed"], n)
        if on_chunk:
            _wait(on_chunk(0, n, xyz, rgba))
        mem["xyz"][: 12 * n].copy_(torch.from_numpy(xyz.view(np.uint8).reshape(-1)))
        mem["rgba"][: 4 * n].copy_(torch.from_numpy(rgba.view(np.uint8)))
    elif wl["order"] == 1:
        xyz, rgba = synth.terrain(wl["seed"], n, order=1)
        if on_chunk:
            _wait(on_chunk(0, n, xyz, rgba))
        mem["xyz"][: 12 * n].copy_(torch.from_numpy(xyz.view(np.uint8).reshape(-1)))
        mem["rgba"][: 4 * n].copy_(torch.from_numpy(rgba.view(np.uint8)))
        del xyz, rgba
    else:
        chunk = min(chunk, n)
        host = [(torch.empty(12 * chunk, dtype=torch.uint8, pin_memory=True),
                 torch.empty(4 * chunk, dtype=torch.uint8, pin_memory=True)) for _ in range(2)]
        done = [None, None]
        seen = [None, None]
        side = torch.cuda.Stream(dev)
        for ci, lo in enumerate(range(0, n, chunk)):
            hi = min(lo + chunk, n)
            hx, hc = host[ci % 2]
            if done[ci % 2] is not None:
                done[ci % 2].synchronize()
            _wait(seen[ci % 2])
            synth.terrain_range(wl["seed"], n, lo, hi, hx.data_ptr(), hc.data_ptr())
            if on_chunk:
                seen[ci % 2] = on_chunk(lo, hi, hx[: 12 * (hi - lo)].numpy().view(np.float32).reshape(-1, 3),
                                        hc[: 4 * (hi - lo)].numpy().view(np.uint32))
            with torch.cuda.stream(side):
                mem["xyz"][12 * lo: 12 * hi].copy_(hx[: 12 * (hi - lo)], non_blocking=True)
                mem["rgba"][4 * lo: 4 * hi].copy_(hc[: 4 * (hi - lo)], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(side)
            done[ci % 2] = ev
            if ci % 8 == 0:
                log(f"generated {hi / 1e6:.0f}M / {n / 1e6:.0f}M points ({time.perf_counter() - t0:.1f} s)")
        side.synchronize()
        for w in seen:
            _wait(w)
        del host
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    log(f"cloud resident in HBM after {t_gen:.1f} s")
    handle = pr.pr_load_points(ctx.handle, mem["xyz"], mem["rgba"], n, True, bufs)
    # A 100k-point build first (untimed): the build kernels' first launches and an idle GPU's clock ramp are not
    # part of building the big cloud (that build measured 0.32 s cold and 0.29 s after this warm-up).
    wx, wc = synth.terrain(wl["seed"] + 1000, 100_000)
    warm = pr.DeviceCloud(ctx, wx, wc, batch_size=S, morton=morton)
    torch.cuda.synchronize()
    del warm
    t1 = time.perf_counter()
    pr.pr_build_batches(ctx.handle, handle, S, morton)
    t_build = time.perf_counter() - t1
    nb = pr.pr_cloud_info(handle)[1]
    log(f"build (finite check{', Morton sort' if morton else ''}, boxes, Eq. 1 split): {t_build:.2f} s, {nb} batches")
    return dict(handle=handle, mem=mem, bufs=bufs, n=n, nb=nb, t_gen=t_gen, t_build=t_build)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads for the host legs: the CPUs this process may run on, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(wl, sample_n: int, seconds: float):
    """The oracle, as it stands, on a bounded sample of the same workload: frames rendered concurrently on the
    host's threads (one whole single-threaded oracle frame per thread at a time; frames are independent), and,
    beside it, on one thread."""
    import numpy as np
    import oracle
    import synth
    from concurrent.futures import ThreadPoolExecutor

    t0 = time.perf_counter()
    if wl["name"].startswith("primitives"):
        xyz, rgba = synth.primitives(wl["seed"], sample_n)
    else:
        xyz, rgba = synth.terrain(wl["seed"], sample_n, order=wl["order"])
    B = oracle.build_cloud(xyz, rgba, 10240, morton=wl["morton"])
    del xyz, rgba
    t_build = time.perf_counter() - t0
    nb = len(B.batches)
    cams = wl["cams"]

    def frame(i):
        cam = cams[i % len(cams)]
        vb, st = oracle.render(B, cam.view, cam.proj, cam.width, cam.height)
        return st["points"], int(np.count_nonzero(vb != oracle.EMPTY))

    # one thread first (at least one frame per camera, about a third of the time budget)
    pts1, secs1, frames1, cover = 0, 0.0, 0, []
    while secs1 < seconds / 3 or frames1 < len(cams):
        t = time.perf_counter()
        p, c = frame(frames1)
        secs1 += time.perf_counter() - t
        pts1 += p
        cover.append(c)
        frames1 += 1
    threads = host_threads()
    per_round = 2 * threads
    pts, frames, secs = 0, 0, 0.0
    with ThreadPoolExecutor(threads) as ex:
        while secs < seconds:
            t = time.perf_counter()
            res = list(ex.map(frame, range(frames, frames + per_round)))
            secs += time.perf_counter() - t
            for k, (p, c) in enumerate(res):
                pts += p
                assert c == cover[(frames + k) % len(cams)], "oracle frames differ between runs"
            frames += per_round
    label = wl["name"].split("_")[0]
    return dict(value=round(pts / secs / 1e9, 6), unit="Gpoints/s", cores=threads, kind="oracle",
                cpu_model=cpu_model(),
                sample=f"{label} generator at {sample_n} points (Morton={wl['morton']}, {nb} batches of 10240), "
                       f"same cameras and resolution; {frames} whole oracle frames rendered concurrently on "
                       f"{threads} threads, {pts} processed points in {secs:.1f} s; oracle build {t_build:.1f} s "
                       f"not included",
                single_thread={"value": round(pts1 / secs1 / 1e9, 6), "unit": "Gpoints/s", "frames": frames1,
                               "seconds": round(secs1, 2)})


def cpu_single_c1(seconds: float = 1.0) -> dict:
    """The oracle on one thread over the C1 workload (the 8 primitives, 1e6 points, 1280x720): its frame time, as the
    host's reference for the small configuration."""
    import oracle
    import synth

    wl = workload("c1", None)
    xyz, rgba = synth.primitives(wl["seed"], wl["n"])
    B = oracle.build_cloud(xyz, rgba, 10240, morton=wl["morton"])
    cam = wl["cams"][0]
    pts, secs, frames = 0, 0.0, 0
    while secs < seconds or frames < 3:
        t = time.perf_counter()
        _, st = oracle.render(B, cam.view, cam.proj, cam.width, cam.height)
        secs += time.perf_counter() - t
        pts += st["points"]
        frames += 1
    return {"workload": wl["name"], "ms_per_frame": round(secs / frames * 1e3, 3),
            "value": round(pts / secs / 1e9, 6), "unit": "Gpoints/s", "frames": frames, "threads": 1}


def profile_counters(kernel_src_hash: str, workload_name: str) -> dict:
    """Counters of the render kernel (HBM bytes, VALU instructions per launch) from the committed rocprofv3 --pmc
    summary, if it was taken on these kernel sources; else {}."""
    path = os.path.join(ROOT, "profiles", f"render_{workload_name}_counters.json")
    if not os.path.exists(path):
        return {}
    try:
        d = json.load(open(path))
    except Exception:
        return {}
    if d.get("kernel_src_sha256") != kernel_src_hash:
        return {}
    return d


def measure_stream(pr, ctx, nbytes: int = 4 << 30, reps: int = 10) -> dict:
    """Streaming ceiling of this device, from the library's own probe kernels: GB/s of a read-only pass over
    2 x nbytes and of a copy of nbytes (read + write counted), mean over reps launches each after two untimed."""
    import torch

    a = torch.ones(2 * nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    out = {}
    for name, src, dst, moved in (("read", a, None, 2 * nbytes), ("copy", a, b, 2 * nbytes)):
        nb = 2 * nbytes if dst is None else nbytes
        for _ in range(2):
            pr.pr_stream_probe(ctx.handle, src, dst, nb)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            pr.pr_stream_probe(ctx.handle, src, dst, nb)
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = round(moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def roofline(alg_bytes: float, ms: float, what: str, bytes_note: str) -> dict:
    """HBM roofline of a timed call: algorithmic bytes over its event-timed span, against 8 TB/s."""
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": what, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": int(alg_bytes), "bytes": bytes_note,
            "span_ms": round(ms, 4)}


def render_bytes(st: dict) -> int:
    """Algorithmic bytes of the point loop of a frame: its coordinate words plus one 80-byte render record per live
    (batch, view)."""
    return st["words_bytes"] + 80 * sum(st["level_batches"])


def timed_ms(fn, steps: int, warmup: int) -> float:
    """Mean span of fn() over steps calls, HIP events on the current stream, after warmup untimed calls."""
    import numpy as np
    import torch

    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def kernel_hash():
    import hashlib

    h = hashlib.sha256()
    for f in ("raster_core.h", "kern_raster.hip", "kern_render.hip", "internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2204_01287_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def multiview_and_graphs(pr, ctx, cloud, cams, vbs, fbs, frame, processed, plain_ms, steps, warmup):
    """The same stereo step with both eyes in one multi-view launch, and both forms replayed from HIP graphs."""
    import numpy as np
    import torch

    stream = torch.cuda.current_stream()
    need = pr.pr_views_work_bytes(cloud["handle"], len(cams))
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    vlist = [(c.view, c.proj, c.width, c.height, vb) for c, vb in zip(cams, vbs)]

    def frame_views():
        pr.pr_render_views(ctx.handle, cloud["handle"], vlist, None, work, need)
        for c, vb, fb in zip(cams, vbs, fbs):
            pr.pr_resolve(ctx.handle, cloud["handle"], vb, c.width, c.height, 0xFF000000, fb)

    def timed(fn):
        for _ in range(warmup):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        pr.pr_sync(ctx.handle)
        return [a.elapsed_time(b) for a, b in ev]

    mv = timed(frame_views)
    pr.pr_render_views(ctx.handle, cloud["handle"], vlist, pr.RenderOpts.make(counters=1), work, need)
    st = pr.pr_get_stats(ctx.handle)
    rv_ms = timed_ms(lambda: pr.pr_render_views(ctx.handle, cloud["handle"], vlist, None, work, need), steps, warmup)
    # the render kernel alone: the library's event pair around its launch
    pr.pr_time_kernels(ctx.handle, steps)
    for _ in range(steps):
        pr.pr_render_views(ctx.handle, cloud["handle"], vlist, None, work, need)
    torch.cuda.synchronize()
    kv_ms = float(np.mean(pr.pr_kernel_times(ctx.handle)))
    pr.pr_time_kernels(ctx.handle, 0)
    words_note = ("coordinate words streamed once per batch at the highest level among its live views + 80 B per "
                  "live (batch, view) record")
    res = {"launches": "one clear, one classify, one render launch for both eyes; resolve per eye",
           "roofline": roofline(render_bytes(st), rv_ms, "pr_render_views (clear, classify, render of both eyes)",
                                words_note),
           "roofline_kernel": roofline(render_bytes(st), kv_ms, "k_render_views (the render launch of "
                                       "pr_render_views, timed by HIP events around it: pr_time_kernels)",
                                       words_note),
           "ms_per_step": round(float(np.mean(mv)), 4),
           "gpts": round(processed / (float(np.mean(mv)) * 1e-3) / 1e9, 3),
           "frame_ms_p50": round(float(np.percentile(mv, 50)), 4),
           "frame_ms_p99": round(float(np.percentile(mv, 99)), 4),
           "speedup_vs_plain": round(plain_ms / float(np.mean(mv)), 4)}
    log(f"multi-view: {res}")
    graphs = {}
    for name, fn in (("plain", frame), ("multiview", frame_views)):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            fn()
        t = timed(g.replay)
        graphs[name] = {"ms_per_step": round(float(np.mean(t)), 4),
                        "gpts": round(processed / (float(np.mean(t)) * 1e-3) / 1e9, 3)}
        del g
    res["hip_graph"] = graphs
    log(f"graphs: {graphs}")
    return res


def order_leg(pr, ctx, cloud, cams, vbs, fbs, frame, processed, steps, warmup, order):
    """The headline cloud rebuilt in place in another point order (PR_ORDER_MORTON: the same Morton batches with
    their points in plain Morton order): the plain step and the multi-view step again."""
    import numpy as np
    import torch

    stream = torch.cuda.current_stream()
    mem, n = cloud["mem"], cloud["n"]
    # the xyz buffer holds the built order; the colours in that order become the build's input colours
    mem["rgba"][: 4 * n].copy_(mem["colors"][: 4 * n])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pr.pr_build_batches(ctx.handle, cloud["handle"], 10240, order)
    t_build = time.perf_counter() - t0
    need = pr.pr_views_work_bytes(cloud["handle"], len(cams))
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    vlist = [(c.view, c.proj, c.width, c.height, vb) for c, vb in zip(cams, vbs)]

    def frame_views():
        pr.pr_render_views(ctx.handle, cloud["handle"], vlist, None, work, need)
        for c, vb, fb in zip(cams, vbs, fbs):
            pr.pr_resolve(ctx.handle, cloud["handle"], vb, c.width, c.height, 0xFF000000, fb)

    def timed(fn):
        for _ in range(warmup):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        pr.pr_sync(ctx.handle)
        return float(np.mean([a.elapsed_time(b) for a, b in ev]))

    plain = timed(frame)
    mv = timed(frame_views)
    rv = timed_ms(lambda: pr.pr_render_views(ctx.handle, cloud["handle"], vlist, None, work, need), steps, warmup)
    c = cams[0]
    res_ms = timed_ms(lambda: pr.pr_resolve(ctx.handle, cloud["handle"], vbs[0], c.width, c.height, 0xFF000000,
                                            fbs[0]), steps, warmup)
    res = {"build_s": round(t_build, 3),
           "plain": {"ms_per_step": round(plain, 4), "gpts": round(processed / (plain * 1e-3) / 1e9, 3)},
           "multiview": {"ms_per_step": round(mv, 4), "gpts": round(processed / (mv * 1e-3) / 1e9, 3),
                         "render_views_ms": round(rv, 4)},
           "resolve_ms": round(res_ms, 4)}
    log(f"order {order}: {res}")
    return res


def hqs_leg(pr, ctx, cloud, cams, processed, steps, warmup, window=1.01):
    """The stereo step with high-quality shading (Sec. 3.6) instead of the plain resolve: per eye, the render,
    the shading pass (colour sums within the depth window) and the averaging resolve."""
    import numpy as np
    import torch

    stream = torch.cuda.current_stream()
    bufs = [(torch.empty(c.width * c.height, dtype=torch.int64, device="cuda"),
             torch.empty(2 * c.width * c.height, dtype=torch.int64, device="cuda"),
             torch.empty(c.width * c.height, dtype=torch.int32, device="cuda")) for c in cams]

    def step():
        for c, (vb, acc, fb) in zip(cams, bufs):
            pr.pr_render_hqs(ctx.handle, cloud["handle"], c.view, c.proj, c.width, c.height, None, window, vb, acc,
                             0xFF000000, fb)

    for _ in range(warmup):
        step()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    pr.pr_sync(ctx.handle)
    t = [a.elapsed_time(b) for a, b in ev]
    alg = 0
    for c, (vb, acc, fb) in zip(cams, bufs):
        pr.pr_render(ctx.handle, cloud["handle"], c.view, c.proj, c.width, c.height, pr.RenderOpts.make(counters=1),
                     vb)
        st = pr.pr_get_stats(ctx.handle)
        px = c.width * c.height
        # classify (32 B per batch, clear 8 B/px), render, zeroed sums (16 B/px), shading pass (words again,
        # 4 B colour per processed point, records, 8 B/px closest depths), averaging resolve (16 B/px + 4 B/px)
        alg += 32 * st["batches"] + 8 * px + render_bytes(st) + 16 * px + render_bytes(st) + 4 * st["points"] + \
            8 * px + 20 * px
    res = {"window": window, "ms_per_step": round(float(np.mean(t)), 4),
           "gpts": round(processed / (float(np.mean(t)) * 1e-3) / 1e9, 3),
           "roofline": roofline(alg, float(np.mean(t)), "pr_render_hqs of both eyes (render, shading pass, resolve)",
                                "classify 32 B/batch + clear 8 B/px, render words + 80 B/record, sums zeroed "
                                "16 B/px, shading words + 4 B colour per processed point + 80 B/record + 8 B/px "
                                "closest depths, resolve 20 B/px")}
    log(f"high-quality shading: {res}")
    return res


def lod_leg(pr, ctx, n: int, steps: int, warmup: int):
    """Level of detail (Sec. 3.5): the terrain as a layered point cloud (a seeded level per point, octree nodes,
    variable-size batches of at most 10,240 points), rendered with every node and with the nodes below the root
    culled under 100 px; the stereo pair and a 1920x1080 orbit overview."""
    import numpy as np
    import torch
    import synth

    t0 = time.perf_counter()
    xyz, rgba = synth.terrain(synth.C3_SEED, n, order=0)
    depth = synth.lpc_depth(n, 10240)
    xo, ro, spans, nodes = synth.lpc_layout(7, xyz, rgba, depth, 10240)
    del xyz, rgba
    dc = pr.DeviceCloud(ctx, xo, ro, spans=spans, nodes=nodes)
    del xo, ro
    log(f"lod: {n} points, depth {depth}, {len(spans)} batches, ready after {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream()
    views = {"stereo_2x2016x2240": synth.stereo_cameras(synth.C3_SEED),
             "orbit_1920x1080": [synth.orbit_camera(7)]}
    out = {"points": n, "depth": depth, "batches": len(spans), "cap": 10240}
    for vname, cams in views.items():
        vbs = [torch.empty(c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]
        fbs = [torch.empty(c.width * c.height, dtype=torch.int32, device="cuda") for c in cams]
        res = {}
        for lod_px in (0.0, 100.0):
            processed, alg = 0, 0
            for c, vb in zip(cams, vbs):
                pr.pr_render(ctx.handle, dc.handle, c.view, c.proj, c.width, c.height,
                             pr.RenderOpts.make(counters=1, lod_px=lod_px), vb)
                st = pr.pr_get_stats(ctx.handle)
                processed += st["points"]
                # classify 32 B/batch + clear 8 B/px, render, resolve 12 B/px
                alg += 32 * st["batches"] + 8 * c.width * c.height + render_bytes(st) + 12 * c.width * c.height
            o = pr.RenderOpts.make(lod_px=lod_px)

            def step():
                for c, vb, fb in zip(cams, vbs, fbs):
                    pr.pr_render(ctx.handle, dc.handle, c.view, c.proj, c.width, c.height, o, vb)
                    pr.pr_resolve(ctx.handle, dc.handle, vb, c.width, c.height, 0xFF000000, fb)

            for _ in range(warmup):
                step()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
            torch.cuda.synchronize()
            for a, b in ev:
                a.record(stream)
                step()
                b.record(stream)
            torch.cuda.synchronize()
            t = float(np.mean([a.elapsed_time(b) for a, b in ev]))
            res[f"lod_px_{int(lod_px)}"] = {"ms_per_frame": round(t, 4), "processed_points": processed,
                                            "gpts": round(processed / (t * 1e-3) / 1e9, 3),
                                            "all_points_rate_gpts": round(n * len(cams) / (t * 1e-3) / 1e9, 3),
                                            "roofline": roofline(alg, t, "pr_render + pr_resolve per view",
                                                                 "classify 32 B/batch + clear 8 B/px, render "
                                                                 "words + 80 B/record, resolve 12 B/px")}
        res["frame_speedup"] = round(res["lod_px_0"]["ms_per_frame"] / res["lod_px_100"]["ms_per_frame"], 3)
        # the autotuner on the LOD frame (lod_px 100): winner, then the same plain frame under it
        need = pr.pr_views_work_bytes(dc.handle, len(cams))
        work = torch.empty(need, dtype=torch.uint8, device="cuda")
        best, trials = pr.pr_autotune(ctx.handle, dc.handle, [(c.view, c.proj, c.width, c.height, vb)
                                                              for c, vb in zip(cams, vbs)],
                                      pr.RenderOpts.make(lod_px=100.0), work, need, 3)
        o = pr.RenderOpts.make(lod_px=100.0)
        for _ in range(warmup):
            step()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            step()
            b.record(stream)
        torch.cuda.synchronize()
        t = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        res["lod_px_100_tuned"] = {"tuning": best, "shape": pr.pr_raster_shapes(ctx.handle)[best["shape"]],
                                   "ms_per_frame": round(t, 4),
                                   "speedup_vs_default": round(res["lod_px_100"]["ms_per_frame"] / t, 3)}
        pr.pr_set_tuning(ctx.handle)
        del work
        # LOD with high-quality shading (window 1.01), the paper's VR combination, under the default tuning
        accs = [torch.empty(2 * c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]

        def step_hqs():
            for c, vb, acc, fb in zip(cams, vbs, accs, fbs):
                pr.pr_render_hqs(ctx.handle, dc.handle, c.view, c.proj, c.width, c.height, o, 1.01, vb, acc,
                                 0xFF000000, fb)

        for _ in range(warmup):
            step_hqs()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            step_hqs()
            b.record(stream)
        torch.cuda.synchronize()
        res["lod_px_100_hqs"] = {"window": 1.01,
                                 "ms_per_frame": round(float(np.mean([a.elapsed_time(b) for a, b in ev])), 4)}
        del accs
        out[vname] = res
        log(f"lod {vname}: {res}")
    pr.pr_sync(ctx.handle)
    dc.close()
    del dc
    torch.cuda.empty_cache()
    return out


def autotune_leg(pr, ctx, cloud, cams, vbs, frame, plain_ms, steps, warmup):
    """The autotuner on the headline workload: pr_autotune over the stereo pair (workgroup shape, tile bound,
    grid; the batch size stays 10,240), then the plain step timed again under the winner."""
    import numpy as np
    import torch

    need = pr.pr_views_work_bytes(cloud["handle"], len(cams))
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    views = [(c.view, c.proj, c.width, c.height, vb) for c, vb in zip(cams, vbs)]
    t0 = time.perf_counter()
    best, trials = pr.pr_autotune(ctx.handle, cloud["handle"], views, None, work, need, 3)
    t_tune = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        frame()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        frame()
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    pr.pr_set_tuning(ctx.handle)
    shapes = pr.pr_raster_shapes(ctx.handle)
    default_ms = next(m for t, m in trials if t == {"shape": 0, "tile_px": 0, "wg_per_cu": 0, "max_bands": 0})
    res = {"candidates": len(trials), "tune_s": round(t_tune, 2), "best": best, "best_shape": shapes[best["shape"]],
           "multiview_frame_ms": {"default": round(default_ms, 4), "best": round(min(m for _, m in trials), 4)},
           "plain_step_ms": {"default": round(plain_ms, 4), "tuned": round(ms, 4)},
           "top5": [{"tuning": t, "shape": shapes[t["shape"]], "ms": round(m, 4)}
                    for t, m in sorted(trials, key=lambda x: x[1])[:5]]}
    log(f"autotune (stereo): {res}")
    return res


class _BenchCloud:
    """A cloud loaded by load_cloud, with the handle/close interface the batch-size tuner expects."""

    def __init__(self, pr, c):
        self.pr, self.c, self.handle, self.nb = pr, c, c["handle"], c["nb"]

    def close(self):
        if self.handle:
            self.pr.pr_cloud_free(self.handle)
            self.handle = None
            self.c["mem"].clear()


def camera_array_leg(pr, ctx, n: int, steps: int, warmup: int, sizes=(5120, 10240, 20480)):
    """Camera array: 64 views of 1024x1024 at random cameras over an n-point terrain (seed 4, Morton batches).
    The autotuner sweeps batch size x workgroup shape x tile bound x grid on the 64-view frame; then 64
    single-view launches (pr_render + resolve each) against one multi-view launch (+ 64 resolves), under the
    default configuration (10,240, shape 0) and the tuned one.  Every configuration renders the same images."""
    import numpy as np
    import torch
    import synth
    from paper_2204_01287_amd.autotune import tune

    cams = synth.camera_array(4, 64, 1024, 1024)
    vbs = [torch.empty(c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]
    fbs = [torch.empty(c.width * c.height, dtype=torch.int32, device="cuda") for c in cams]
    stream = torch.cuda.current_stream()
    kept = {}

    def build(S):
        c = _BenchCloud(pr, load_cloud(ctx, dict(name=f"terrain_c4_S{S}", seed=4, n=n, morton=2, order=0,
                                                 batch_size=S)))
        kept[S] = c
        return _Keep(c)

    t0 = time.perf_counter()
    res = tune(ctx, build, sizes, cams, reps=2, log=log)
    t_tune = time.perf_counter() - t0
    best = res["best"]

    def timed(fn):
        for _ in range(warmup):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev]))

    out = {"points": n, "views": "64 x 1024x1024", "tune_s": round(t_tune, 1), "candidates": len(res["trials"]),
           "best": best, "best_shape": pr.pr_raster_shapes(ctx.handle)[best["tuning"]["shape"]]}
    configs = {"default": (10240, {"shape": 0, "tile_px": 0, "wg_per_cu": 0, "max_bands": 0}),
               "tuned": (best["batch_size"], best["tuning"])}
    for name, (S, t) in configs.items():
        c = kept[S]
        pr.pr_set_tuning(ctx.handle, **t)
        processed = 0
        for cam, vb in zip(cams, vbs):
            pr.pr_render(ctx.handle, c.handle, cam.view, cam.proj, cam.width, cam.height,
                         pr.RenderOpts.make(counters=1), vb)
            processed += pr.pr_get_stats(ctx.handle)["points"]
        need = pr.pr_views_work_bytes(c.handle, len(cams))
        work = torch.empty(need, dtype=torch.uint8, device="cuda")
        vlist = [(cam.view, cam.proj, cam.width, cam.height, vb) for cam, vb in zip(cams, vbs)]

        def plain():
            for cam, vb, fb in zip(cams, vbs, fbs):
                pr.pr_render(ctx.handle, c.handle, cam.view, cam.proj, cam.width, cam.height, None, vb)
                pr.pr_resolve(ctx.handle, c.handle, vb, cam.width, cam.height, 0xFF000000, fb)

        def multi():
            pr.pr_render_views(ctx.handle, c.handle, vlist, None, work, need)
            for cam, vb, fb in zip(cams, vbs, fbs):
                pr.pr_resolve(ctx.handle, c.handle, vb, cam.width, cam.height, 0xFF000000, fb)

        p_ms, m_ms = timed(plain), timed(multi)
        pr.pr_render_views(ctx.handle, c.handle, vlist, pr.RenderOpts.make(counters=1), work, need)
        st = pr.pr_get_stats(ctx.handle)
        npx = sum(cam.width * cam.height for cam in cams)
        chunks = (len(cams) + 15) // 16
        alg = 32 * c.nb * chunks + 8 * npx + render_bytes(st) + 12 * npx
        out[name] = {"batch_size": S, "tuning": t, "processed_points": processed,
                     "roofline_multiview": roofline(alg, m_ms, "pr_render_views of 64 views + 64 resolves",
                                                    "classify 32 B/batch per 16 views + clear 8 B/px, words once "
                                                    "per batch and classify launch + 80 B/record, resolve 12 B/px"),
                     "plain_64_launches_ms": round(p_ms, 3), "multiview_one_launch_ms": round(m_ms, 3),
                     "plain_gpts": round(processed / (p_ms * 1e-3) / 1e9, 2),
                     "multiview_gpts": round(processed / (m_ms * 1e-3) / 1e9, 2),
                     "multiview_speedup": round(p_ms / m_ms, 3)}
        log(f"camera array {name}: {out[name]}")
        del work
    out["tuned_vs_default_multiview"] = round(out["default"]["multiview_one_launch_ms"] /
                                              out["tuned"]["multiview_one_launch_ms"], 3)
    bys = {}
    for t in res["trials"]:
        bys[t["batch_size"]] = min(bys.get(t["batch_size"], 1e30), t["ms"])
    out["best_ms_by_batch_size"] = {str(k): round(v, 3) for k, v in bys.items()}
    pr.pr_set_tuning(ctx.handle)
    pr.pr_sync(ctx.handle)
    for c in kept.values():
        c.close()
    kept.clear()
    torch.cuda.empty_cache()
    return out


class _Keep:
    """Hands a cloud to the tuner without letting it free the cloud (the leg times it again afterwards)."""

    def __init__(self, c):
        self.handle = c.handle

    def close(self):
        pass


def c2_leg(pr, ctx, steps: int, warmup: int, n: int = 100_000_000):
    """The paper's bandwidth and ordering comparisons on the 1e8-point terrain, over the 60-frame orbit at
    1920x1080 (per frame: pr_render + pr_resolve): adaptive precision (4/8/12-byte loads, Sec. 3.3) against fixed
    12-byte loads (PR_FORCE30), Morton order against the generation order (10 m tiles in serpentine strips) and
    against the generator's index order (spatially incoherent, Sec. 4.2), and the default prefetch depth against
    one group in flight per wave (Sec. 3.4).  Every variant
    renders the same points; only what each frame loads, in which order, and how far ahead, differs."""
    import numpy as np
    import torch
    import synth

    cams = [synth.orbit_camera(f) for f in range(60)]
    stream = torch.cuda.current_stream()
    shapes = pr.pr_raster_shapes(ctx.handle)
    d1 = next(i for i, sh in enumerate(shapes) if sh["depth"] == 1 and sh["waves"] == shapes[0]["waves"] and
              sh["tile_px"] == shapes[0]["tile_px"])
    clouds = {}
    t0 = time.perf_counter()
    # generation order: 10 m tiles in serpentine strips (aerial-strip-like, already compact batches); index order:
    # the generator's points by index, spatially incoherent (like the paper's scan order of laser scans)
    for order, morton, gen in (("morton", 1, 1), ("morton_spread", 2, 1), ("generation", 0, 1), ("index", 0, 0)):
        clouds[order] = load_cloud(ctx, dict(name=f"terrain_1e8_{order}", seed=synth.C2_SEED, n=n, morton=morton,
                                             order=gen))
    log(f"c2: four 1e8-point builds in {time.perf_counter() - t0:.1f} s")
    w, h = cams[0].width, cams[0].height
    vb = torch.empty(w * h, dtype=torch.int64, device="cuda")
    fb = torch.empty(w * h, dtype=torch.int32, device="cuda")
    variants = {"morton_adaptive": ("morton", pr.PR_ADAPTIVE, 0),
                "morton_force30": ("morton", pr.PR_FORCE30, 0),
                "morton_spread_adaptive": ("morton_spread", pr.PR_ADAPTIVE, 0),
                "generation_adaptive": ("generation", pr.PR_ADAPTIVE, 0),
                "index_order_adaptive": ("index", pr.PR_ADAPTIVE, 0),
                "morton_adaptive_prefetch1": ("morton", pr.PR_ADAPTIVE, d1)}
    out = {"points": n, "frames": 60, "view": f"{w}x{h}", "prefetch1_shape": shapes[d1]}
    for name, (order, prec, shape) in variants.items():
        c = clouds[order]
        pr.pr_set_tuning(ctx.handle, shape=shape)
        processed, alg = 0, 0
        for cam in cams:  # counters pass: processed points and loaded words of every frame
            pr.pr_render(ctx.handle, c["handle"], cam.view, cam.proj, w, h,
                         pr.RenderOpts.make(precision=prec, counters=1), vb)
            st = pr.pr_get_stats(ctx.handle)
            processed += st["points"]
            lp = st["level_points"]
            alg += 4 * lp[0] + 8 * lp[1] + 12 * lp[2] + 80 * (st["batches"] - st["culled"])
        o = pr.RenderOpts.make(precision=prec)

        def orbit():
            for cam in cams:
                pr.pr_render(ctx.handle, c["handle"], cam.view, cam.proj, w, h, o, vb)
                pr.pr_resolve(ctx.handle, c["handle"], vb, w, h, 0xFF000000, fb)

        for _ in range(max(1, warmup)):
            orbit()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            orbit()
            b.record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev])) / len(cams)
        out[name] = {"ms_per_frame": round(ms, 4), "processed_points_per_frame": processed // len(cams),
                     "gpts": round(processed / len(cams) / (ms * 1e-3) / 1e9, 2),
                     "algorithmic_gb_per_frame": round(alg / len(cams) / 1e9, 4),
                     "algorithmic_gbs": round(alg / len(cams) / (ms * 1e-3) / 1e9, 1)}
        log(f"c2 {name}: {out[name]}")
    pr.pr_set_tuning(ctx.handle)
    base = out["morton_adaptive"]["ms_per_frame"]
    out["speedup_adaptive_vs_force30"] = round(out["morton_force30"]["ms_per_frame"] / base, 3)
    out["speedup_morton_vs_generation"] = round(out["generation_adaptive"]["ms_per_frame"] / base, 3)
    out["speedup_morton_vs_index_order"] = round(out["index_order_adaptive"]["ms_per_frame"] / base, 3)
    out["speedup_prefetch_vs_depth1"] = round(out["morton_adaptive_prefetch1"]["ms_per_frame"] / base, 3)
    out["speedup_spread_vs_morton"] = round(base / out["morton_spread_adaptive"]["ms_per_frame"], 3)
    pr.pr_sync(ctx.handle)
    for c in clouds.values():
        pr.pr_cloud_free(c["handle"])
        c["mem"].clear()
    torch.cuda.empty_cache()
    return out


def served_leg(pr, ctx, nreq: int, rates, budget: int):
    """Served workload: 8 resident terrain clouds (3.41e9 points), seeded Poisson request streams with random
    cameras and image sizes 640x480 / 1920x1080 / 3840x2160, admission by device bytes (visibility + frame buffers
    and the work-area share).  Continuous batching (grouped multi-view launches on 4 streams) against one view per
    launch on the same 4 streams (only the grouping differs), and against one view per launch with every request
    queued on one stream as soon as it is admitted: latency at each offered rate, and capacity with every request
    arriving at once."""
    import numpy as np
    import torch
    import synth
    from paper_2204_01287_amd.serve import Request, Server

    t0 = time.perf_counter()
    clouds = []
    for seed, n in synth.SERVED_CLOUDS:
        c = load_cloud(ctx, dict(name=f"served_{seed}", seed=seed, n=n, morton=2, order=0))
        pr.pr_cloud_drop_load_buffers(c["handle"])
        pr.pr_sync(ctx.handle)
        for f in ("xyz", "rgba", "perm", "scratch"):
            c["mem"][f] = None
        torch.cuda.empty_cache()
        clouds.append(c)
    t_load = time.perf_counter() - t0
    resident = sum(t.numel() for c in clouds for t in c["mem"].values() if t is not None)
    log(f"served: {len(clouds)} clouds resident ({resident / 1e9:.1f} GB) after {t_load:.1f} s")
    seeds = [s for s, _ in synth.SERVED_CLOUDS]
    streams = {r: synth.request_stream(5, nreq, r, seeds) for r in rates}
    handles = [c["handle"] for c in clouds]
    # processed points of every request (Table 2 definition), counted solo once (the same requests at every rate)
    first = streams[rates[0]]
    for r in rates[1:]:
        assert [(ci, cam.width) for _, ci, cam in streams[r]] == [(ci, cam.width) for _, ci, cam in first]
    pts = []
    need = max(pr.pr_views_work_bytes(h, 1) for h in handles)
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    vbmax = torch.empty(max(cam.width * cam.height for _, _, cam in first), dtype=torch.int64, device="cuda")
    for a, ci, cam in first:
        vb = vbmax[: cam.width * cam.height]
        pr.pr_render_views(ctx.handle, handles[ci], [(cam.view, cam.proj, cam.width, cam.height, vb)],
                           pr.RenderOpts.make(counters=1), work, need)
        pts.append(pr.pr_get_stats(ctx.handle)["points"])
    del work, vbmax
    total_pts = float(sum(pts))
    out = {"workload": "8 terrain clouds 1e7..1e9 (3.41e9 points), Poisson requests, 640x480/1920x1080/3840x2160",
           "requests": nreq, "rates_per_s": list(rates), "budget_bytes": budget,
           "resident_gb": round(resident / 1e9, 2), "load_s": round(t_load, 1),
           "mean_processed_points": round(total_pts / nreq)}
    modes = {"batched": dict(nstreams=4, max_group=64),
             "one_view_per_launch": dict(nstreams=4, max_group=1),
             "one_view_per_launch_1stream_queued": dict(nstreams=1, max_group=1, depth=1 << 30)}
    loads = [(f"offered_{int(r)}", r) for r in rates] + [("saturated", None)]
    for name, kw in modes.items():
        for load, rate in loads:
            if name.endswith("queued") and rate is not None:
                continue  # capacity only
            src = streams[rate if rate is not None else rates[0]]
            reqs = [Request(i, ci, cam, a if rate is not None else 0.0) for i, (a, ci, cam) in enumerate(src)]
            srv = Server(handles, budget_bytes=budget, **kw)
            done = srv.run(reqs)
            peak = srv.peak_bytes
            srv.close()
            lat = np.array([d.latency for d in done]) * 1e3
            span = max(d.completed for d in done) - min(r.arrival for r in reqs)
            out[f"{name}_{load}"] = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                                     "p99_ms": round(float(np.percentile(lat, 99)), 3),
                                     "gpts": round(total_pts / span / 1e9, 2), "span_s": round(span, 3),
                                     "mean_group": round(float(np.mean([d.group for d in done])), 2),
                                     "peak_admitted_bytes": int(peak)}
            log(f"served {name} {load}: {out[f'{name}_{load}']}")
    out["capacity_speedup_same_streams"] = round(out["batched_saturated"]["gpts"] /
                                                 out["one_view_per_launch_saturated"]["gpts"], 3)
    out["capacity_speedup_vs_1stream_queued"] = round(out["batched_saturated"]["gpts"] /
                                                      out["one_view_per_launch_1stream_queued_saturated"]["gpts"], 3)
    for c in clouds:
        pr.pr_cloud_free(c["handle"])
        c["mem"].clear()
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--preheat-s", type=float, default=0.3,
                    help="seconds of untimed frames before the warmup steps (GPU clocks reach their steady state)")
    ap.add_argument("--workload", choices=["c1", "c2", "c3"], default="c3")
    ap.add_argument("--n", type=int, default=None, help="override the point count (smaller test runs)")
    ap.add_argument("--cpu-sample", type=int, default=32_000_000)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-served", action="store_true", help="skip the served-mode leg")
    ap.add_argument("--no-c2", action="store_true", help="skip the 1e8-point precision / order / prefetch leg")
    ap.add_argument("--lod-points", type=int, default=500_000_000, help="points of the LOD leg (0: skip)")
    ap.add_argument("--array-points", type=int, default=500_000_000,
                    help="points of the 64-camera array leg with the batch-size autotuner (0: skip)")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner leg on the headline workload")
    ap.add_argument("--no-order-leg", action="store_true",
                    help="skip the headline cloud rebuilt in plain Morton order (PR_ORDER_MORTON) for comparison")
    ap.add_argument("--served-requests", type=int, default=10000)
    ap.add_argument("--served-rates", type=str, default="500,4000",
                    help="offered request rates per second (comma-separated)")
    ap.add_argument("--served-budget", type=int, default=4 << 30, help="bytes of visibility + frame buffers in flight")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB read + 1 GiB write kernel (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library renders on one GPU (sharding across GPUs is designed, not implemented); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2204_01287_amd as pr

    if args.calib_copy:
        ctx = pr.Context(0)
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            pr.pr_stream_probe(ctx.handle, a, b, a.numel() * 4)
        pr.pr_sync(ctx.handle)
        print(json.dumps({"calib_copy_kernel": "k_stream_copy", "calib_copy_bytes_read": a.numel() * 4,
                          "calib_copy_bytes_written": b.numel() * 4, "launches": 5}))
        ctx.close()
        return

    wl = workload(args.workload, args.n)
    # everything runs on one side stream, so that frames can be captured into HIP graphs
    main_stream = torch.cuda.Stream()
    torch.cuda.set_stream(main_stream)
    ctx = pr.Context(0, stream=main_stream)
    cloud = load_cloud(ctx, wl)
    cams = wl["cams"]
    vbs = [torch.empty(c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]
    fbs = [torch.empty(c.width * c.height, dtype=torch.int32, device="cuda") for c in cams]

    # Counters frame (untimed): processed points and precision levels per view.
    per_view = []
    for c, vb in zip(cams, vbs):
        pr.pr_render(ctx.handle, cloud["handle"], c.view, c.proj, c.width, c.height,
                     pr.RenderOpts.make(counters=1), vb)
        per_view.append(pr.pr_get_stats(ctx.handle))
    processed = sum(s["points"] for s in per_view)
    alg_bytes = [render_bytes(s) for s in per_view]  # k_render: words of live batches + 80 B per live record
    log(f"per-view counters: {per_view}")

    stream = torch.cuda.current_stream()
    ev = [[[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in cams] for _ in range(args.steps)]

    def frame(step_events=None):
        # per eye: pr_render (its classify launch also clears the visibility buffer), then pr_resolve
        for vi, (c, vb, fb) in enumerate(zip(cams, vbs, fbs)):
            e = step_events[vi] if step_events else None
            if e:
                e[0].record(stream)
            pr.pr_render(ctx.handle, cloud["handle"], c.view, c.proj, c.width, c.height, None, vb)
            if e:
                e[1].record(stream)
            pr.pr_resolve(ctx.handle, cloud["handle"], vb, c.width, c.height, 0xFF000000, fb)
            if e:
                e[2].record(stream)

    # The clocks of an idle GPU ramp up over the first tens of milliseconds of work: untimed frames until
    # preheat_s has passed, then the warmup steps, then the timed steps.
    preheat_frames = 0
    t_pre = time.perf_counter()
    while time.perf_counter() - t_pre < args.preheat_s:
        for _ in range(10):
            frame()
        torch.cuda.synchronize()
        preheat_frames += 10
    log(f"preheat: {preheat_frames} untimed frames in {time.perf_counter() - t_pre:.3f} s")
    for _ in range(args.warmup):
        frame()
    torch.cuda.synchronize()
    # The timed steps: one event pair per step (events between the launches add their own stream markers).
    step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in step_ev:
        a.record(stream)
        frame()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # The same steps again with events around every call, and the library's own event pair around each render
    # kernel launch (pr_time_kernels): the render kernel's duration for the roofline, without the header reset
    # and the classify launch that pr_render enqueues before it.
    pr.pr_time_kernels(ctx.handle, args.steps * len(cams))
    for s in range(args.steps):
        frame(ev[s])
    torch.cuda.synchronize()
    pr.pr_sync(ctx.handle)
    kernel_ms = pr.pr_kernel_times(ctx.handle)
    pr.pr_time_kernels(ctx.handle, 0)
    assert len(kernel_ms) == args.steps * len(cams), kernel_ms

    step_ms = [a.elapsed_time(b) for a, b in step_ev]
    step_ms_instrumented = [ev[s][0][0].elapsed_time(ev[s][-1][2]) for s in range(args.steps)]
    call_ms = [[ev[s][v][0].elapsed_time(ev[s][v][1]) for s in range(args.steps)] for v in range(len(cams))]
    render_ms = [[kernel_ms[s * len(cams) + v] for s in range(args.steps)] for v in range(len(cams))]
    resolve_ms = [ev[s][v][1].elapsed_time(ev[s][v][2]) for s in range(args.steps) for v in range(len(cams))]
    ms_per_step = float(np.mean(step_ms))
    value = processed / (ms_per_step * 1e-3) / 1e9
    mean_render = [float(np.mean(r)) for r in render_ms]
    mean_call = [float(np.mean(r)) for r in call_ms]
    achieved = sum(alg_bytes) / (sum(mean_render) * 1e-3) / 1e9  # GB/s over the render kernel launches
    stream_peak = measure_stream(pr, ctx)  # after the frames: clocks as in the timed region
    log(f"streaming probe: {stream_peak}")
    prof = profile_counters(kernel_hash(), wl["name"])
    traffic = prof.get("hbm_bytes_per_launch")
    log(f"wall {wall:.3f} s for {args.steps} steps; events {ms_per_step:.3f} ms/step; render {mean_render} ms; "
        f"resolve {np.mean(resolve_ms):.4f} ms")

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpoints/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["name"], "points": wl["n"], "batches": cloud["nb"], "batch_size": 10240,
                   "views": [f"{c.width}x{c.height}" for c in cams], "precision": "adaptive 10/20/30-bit",
                   "keys": "u64 depth|index",
                   "point_order": {0: "input", 1: "Morton", 2: "Morton batches, spread order inside"}[int(wl["morton"])],
                   "description": wl["desc"]},
        "processed_points_per_step": processed,
        "all_points_rate_gpts": round(wl["n"] * len(cams) / (ms_per_step * 1e-3) / 1e9, 3),
        "render_kernel_ms": [round(m, 4) for m in mean_render],
        "render_call_ms": [round(m, 4) for m in mean_call],
        "render_only_gpts": round(processed / (sum(mean_render) * 1e-3) / 1e9, 3),
        "frame": "per eye: pr_render (frame header reset, classify with the buffer clear, render) + pr_resolve",
        "resolve_ms": round(float(np.mean(resolve_ms)), 4),
        "frame_ms_p50": round(float(np.percentile(step_ms, 50)), 4),
        "frame_ms_p99": round(float(np.percentile(step_ms, 99)), 4),
        "wall_s_timed": round(wall, 4),
        "ms_per_step_with_launch_events": round(float(np.mean(step_ms_instrumented)), 4),
        "preheat": {"seconds": args.preheat_s, "frames": preheat_frames},
        "level_points": [sum(s["level_points"][i] for s in per_view) for i in range(3)],
        "culled_batches": [s["culled"] for s in per_view],
        "atomics": [s["atomics"] for s in per_view],
        "load": {"generate_and_upload_s": round(cloud["t_gen"], 2), "build_s": round(cloud["t_build"], 3),
                 "build_gpts": round(wl["n"] / cloud["t_build"] / 1e9, 3)},
        "roofline": {"bound": "hbm", "kernel": "k_render (the render launch of pr_render, timed by HIP events "
                                                "around that launch: pr_time_kernels)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes_per_launch": [int(b) for b in alg_bytes],
                     "traffic": traffic,
                     "measured_stream_gbs": stream_peak,
                     "frac_of_measured_read": round(achieved / stream_peak["read"], 4)},
    }
    if prof.get("valu_insts_per_launch"):
        # VALU issue beside HBM: wave64 VALU instructions of one render launch (SQ_INSTS_VALU, committed
        # profile of these sources) over the launch's mean duration
        rate = prof["valu_insts_per_launch"] / (float(np.mean(mean_render)) * 1e-3)
        out["valu_roofline"] = {"bound": "alu", "kernel": "render", "achieved": round(rate * 64 / 1e12, 2),
                                "peak": round(VALU_PEAK_WAVE_INSTS * 64 / 1e12, 2),
                                "unit": "T lane-ops/s (wave64 VALU instructions x 64)",
                                "frac": round(rate / VALU_PEAK_WAVE_INSTS, 4),
                                "valu_insts_per_launch": prof["valu_insts_per_launch"]}
    # the same ceiling against the method's own operation count per processed point (unpack 3, convert 3,
    # FMA 9, w test 1, two exact floors, two bounds checks, one 64-bit compare: 20)
    alg_ops = 20 * processed / len(cams) / (float(np.mean(mean_render)) * 1e-3)
    out.setdefault("valu_roofline", {"bound": "alu", "kernel": "render",
                                     "peak": round(VALU_PEAK_WAVE_INSTS * 64 / 1e12, 2)})
    out["valu_roofline"]["algorithmic_ops_per_point"] = 20
    out["valu_roofline"]["algorithmic_achieved"] = round(alg_ops / 1e12, 2)
    out["valu_roofline"]["algorithmic_frac"] = round(alg_ops / (VALU_PEAK_WAVE_INSTS * 64), 4)
    out["multiview"] = multiview_and_graphs(pr, ctx, cloud, cams, vbs, fbs, frame, processed, ms_per_step,
                                            args.steps, args.warmup)
    out["hqs"] = hqs_leg(pr, ctx, cloud, cams, processed, args.steps, args.warmup)
    if not args.no_autotune:
        out["autotune"] = autotune_leg(pr, ctx, cloud, cams, vbs, frame, ms_per_step, args.steps, args.warmup)
    if not args.no_order_leg and wl["morton"] == pr.PR_ORDER_MORTON_SPREAD:
        out["plain_morton_order"] = order_leg(pr, ctx, cloud, cams, vbs, fbs, frame, processed, args.steps,
                                              args.warmup, pr.PR_ORDER_MORTON)
    pr.pr_cloud_free(cloud["handle"])
    cloud["mem"].clear()
    torch.cuda.empty_cache()
    if not args.no_c2:
        out["c2"] = c2_leg(pr, ctx, min(args.steps, 10), args.warmup)
    if args.lod_points:
        out["lod"] = lod_leg(pr, ctx, args.lod_points, args.steps, args.warmup)
    if args.array_points:
        out["camera_array"] = camera_array_leg(pr, ctx, args.array_points, min(args.steps, 10), min(args.warmup, 2))
    if not args.no_served:
        out["served"] = served_leg(pr, ctx, args.served_requests,
                                   [float(r) for r in args.served_rates.split(",")], args.served_budget)
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(wl, min(args.cpu_sample, wl["n"]), args.cpu_seconds)
        out["cpu_baseline"]["single_thread_c1"] = cpu_single_c1()
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

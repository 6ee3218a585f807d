"""Served mode: resident clouds, a stream of render requests, continuous batching.

A request names a resident cloud, a camera and an image size, and arrives at some time.  The scheduler loop:

  * admits arrived requests in arrival order while the bytes of their visibility buffer and framebuffer
    (12 bytes per pixel) fit the memory budget (a request larger than the whole budget runs alone);
  * keeps the admitted requests that are not yet on the GPU per cloud, and whenever a HIP stream has fewer than
    `depth` groups in flight, launches the cloud with the oldest waiting request as one group on it: one
    pr_render_views launch for up to PR_MAX_VIEWS of that cloud's waiting requests (the batches' coordinate words
    are streamed once for the whole group) followed by one resolve per view;
  * runs several streams (one library context each), so that groups of different clouds overlap on the device;
    requests that arrive while the streams are busy wait and join larger groups, and at low load a stream is
    always free, so a request is launched as soon as it is admitted;
  * retires a group when its event has passed: hands each result to the caller's callback, frees its memory.

Latency = completion (host clock when the group's event is seen complete) - arrival.  Every result equals the
solo render of its request: the multi-view render equals the single-view render view by view.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass

from . import _binding as B


@dataclass
class Request:
    rid: int
    cloud: int     # index into the server's clouds
    cam: object    # .view, .proj (float32 4x4), .width, .height
    arrival: float  # seconds after the start of the run


@dataclass
class Done:
    rid: int
    cloud: int
    arrival: float
    launched: float
    completed: float
    group: int     # number of views in the launch that carried it
    stream: int

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


class Server:
    """Renders requests against resident, built clouds (DeviceCloud or handles) on one device."""

    def __init__(self, clouds, device: int = 0, nstreams: int = 4, budget_bytes: int = 4 << 30,
                 max_group: int = B.PR_MAX_VIEWS, clear_rgba: int = 0xFF000000, on_result=None, depth: int = 1):
        import torch

        if not 1 <= max_group <= B.PR_MAX_VIEWS:
            raise ValueError("max_group must be in 1..PR_MAX_VIEWS")
        if depth < 1:
            raise ValueError("depth must be >= 1")
        self.depth = depth  # groups in flight per stream
        self.torch = torch
        self.device = device
        self.handles = [getattr(c, "handle", c) for c in clouds]
        self.streams = [torch.cuda.Stream(device) for _ in range(nstreams)]
        self.ctxs = [B.Context(device, stream=s) for s in self.streams]
        self.budget = int(budget_bytes)
        self.max_group = max_group
        self.clear_rgba = clear_rgba
        self.on_result = on_result  # callable(request, vb, fb): runs before the buffers are released
        self.peak_bytes = 0

    @staticmethod
    def request_bytes(r: Request) -> int:
        return 12 * r.cam.width * r.cam.height

    def _launch(self, si: int, cloud: int, group):
        torch = self.torch
        ctx, stream = self.ctxs[si], self.streams[si]
        h = self.handles[cloud]
        with torch.cuda.stream(stream):
            dev = torch.device("cuda", self.device)
            vbs = [torch.empty(r.cam.width * r.cam.height, dtype=torch.int64, device=dev) for r in group]
            fbs = [torch.empty(r.cam.width * r.cam.height, dtype=torch.int32, device=dev) for r in group]
            need = B.pr_views_work_bytes(h, len(group))
            work = torch.empty(need, dtype=torch.uint8, device=dev)
            B.pr_render_views(ctx.handle, h, [(r.cam.view, r.cam.proj, r.cam.width, r.cam.height, vb)
                                              for r, vb in zip(group, vbs)], None, work, need)
            for r, vb, fb in zip(group, vbs, fbs):
                B.pr_resolve(ctx.handle, h, vb, r.cam.width, r.cam.height, self.clear_rgba, fb)
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev, vbs, fbs, work

    def run(self, requests, idle_sleep: float = 0.0):
        """Serve every request (arrival times relative to the call); returns a list of Done in completion order."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending: deque = deque()  # arrived, not admitted
        waiting = {}  # cloud -> deque of admitted requests not yet on the GPU
        inflight = []  # [event, stream, group, vbs, fbs, work, bytes, launched]
        load = [0] * len(self.streams)
        done = []
        used = 0
        nxt = 0
        t0 = time.perf_counter()
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                pending.append(reqs[nxt])
                nxt += 1
            retired = False
            still = []
            for g in inflight:
                if g[0].query():
                    tdone = time.perf_counter() - t0
                    for r, vb, fb in zip(g[2], g[3], g[4]):
                        if self.on_result is not None:
                            self.on_result(r, vb, fb)
                        done.append(Done(r.rid, r.cloud, r.arrival, g[7], tdone, len(g[2]), g[1]))
                    used -= g[6]
                    load[g[1]] -= 1
                    retired = True
                else:
                    still.append(g)
            inflight = still
            admitted = []
            while pending:
                nbytes = self.request_bytes(pending[0])
                if used + nbytes > self.budget and (inflight or admitted or waiting):
                    break
                used += nbytes
                admitted.append(pending.popleft())
            self.peak_bytes = max(self.peak_bytes, used)
            for r in admitted:
                waiting.setdefault(r.cloud, deque()).append(r)
            launched_any = False
            while waiting:
                si = min(range(len(self.streams)), key=lambda i: load[i])
                if load[si] >= self.depth:
                    break
                cloud = min(waiting, key=lambda c: waiting[c][0].arrival)
                q = waiting[cloud]
                group = [q.popleft() for _ in range(min(self.max_group, len(q)))]
                if not q:
                    del waiting[cloud]
                launched = time.perf_counter() - t0
                ev, vbs, fbs, work = self._launch(si, cloud, group)
                inflight.append([ev, si, group, vbs, fbs, work, sum(self.request_bytes(r) for r in group), launched])
                load[si] += 1
                launched_any = True
            if not admitted and not retired and not launched_any:
                if idle_sleep:
                    time.sleep(idle_sleep)
        for ctx in self.ctxs:
            B.pr_sync(ctx.handle)
        return done

    def close(self):
        for ctx in self.ctxs:
            ctx.close()

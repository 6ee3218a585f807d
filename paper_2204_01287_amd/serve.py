"""Served mode: resident clouds, a stream of render requests, continuous batching.

A request names a resident cloud, a camera and an image size, and arrives at some time.  The scheduler loop:

  * admits arrived requests in arrival order while their device bytes fit the memory budget (a request larger
    than the whole budget runs alone): its visibility buffer and framebuffer (12 bytes per pixel) and its share of
    the multi-view work area of the group that will carry it (pr_views_work_bytes of one view of its cloud, which
    bounds the share: a group's work area is its header and runs plus 80 bytes per batch and view);
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

Scheduler holds the policy and no device state (launch, completion and the clock are callbacks), so that it can
be exercised on the host alone; Server drives it with HIP streams, events and the library's launches.
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


class Scheduler:
    """Admission, grouping and stream assignment of the served mode, without device state.

    run() calls launch(stream, cloud, group) -> token for each group it starts, is_done(token) -> bool to poll a
    group, retire(token, group) when a polled group is complete, and now() for the clock (seconds since the run
    started)."""

    def __init__(self, nstreams: int = 4, budget_bytes: int = 4 << 30, max_group: int = B.PR_MAX_VIEWS,
                 depth: int = 1, request_bytes=None):
        if not 1 <= max_group <= B.PR_MAX_VIEWS:
            raise ValueError("max_group must be in 1..PR_MAX_VIEWS")
        if depth < 1 or nstreams < 1:
            raise ValueError("depth and nstreams must be >= 1")
        self.nstreams, self.budget, self.max_group, self.depth = nstreams, int(budget_bytes), max_group, depth
        self.request_bytes = request_bytes or (lambda r: 12 * r.cam.width * r.cam.height)
        self.peak_bytes = 0

    def run(self, requests, launch, is_done, retire, now, idle=None):
        """Serve every request (arrival times relative to the run); returns a list of Done in completion order."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending: deque = deque()  # arrived, not admitted
        waiting = {}  # cloud -> deque of admitted requests not yet on the GPU
        inflight = []  # [token, stream, group, bytes, launched]
        load = [0] * self.nstreams
        done = []
        used = 0
        nxt = 0
        while len(done) < len(reqs):
            t = now()
            while nxt < len(reqs) and reqs[nxt].arrival <= t:
                pending.append(reqs[nxt])
                nxt += 1
            retired = False
            still = []
            for g in inflight:
                if is_done(g[0]):
                    tdone = now()
                    retire(g[0], g[2])
                    for r in g[2]:
                        done.append(Done(r.rid, r.cloud, r.arrival, g[4], tdone, len(g[2]), g[1]))
                    used -= g[3]
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
                si = min(range(self.nstreams), key=lambda i: load[i])
                if load[si] >= self.depth:
                    break
                cloud = min(waiting, key=lambda c: waiting[c][0].arrival)
                q = waiting[cloud]
                group = [q.popleft() for _ in range(min(self.max_group, len(q)))]
                if not q:
                    del waiting[cloud]
                launched = now()
                token = launch(si, cloud, group)
                inflight.append([token, si, group, sum(self.request_bytes(r) for r in group), launched])
                load[si] += 1
                launched_any = True
            if not admitted and not retired and not launched_any and idle is not None:
                idle()
        return done


class Server:
    """Renders requests against resident, built clouds (DeviceCloud or handles) on one device."""

    def __init__(self, clouds, device: int = 0, nstreams: int = 4, budget_bytes: int = 4 << 30,
                 max_group: int = B.PR_MAX_VIEWS, clear_rgba: int = 0xFF000000, on_result=None, depth: int = 1):
        import torch

        self.torch = torch
        self.device = device
        self.handles = [getattr(c, "handle", c) for c in clouds]
        # a request's bound on its share of the work area of a pr_render_views group over its cloud
        self.work_share = [B.pr_views_work_bytes(h, 1) for h in self.handles]
        self.scheduler = Scheduler(nstreams, budget_bytes, max_group, depth, self.request_bytes)
        self.streams = [torch.cuda.Stream(device) for _ in range(nstreams)]
        self.ctxs = [B.Context(device, stream=s) for s in self.streams]
        self.clear_rgba = clear_rgba
        self.on_result = on_result  # callable(request, vb, fb): runs before the buffers are released

    @property
    def peak_bytes(self) -> int:
        return self.scheduler.peak_bytes

    def request_bytes(self, r: Request) -> int:
        """Device bytes a request holds while admitted: visibility buffer + framebuffer + its work-area share."""
        return 12 * r.cam.width * r.cam.height + self.work_share[r.cloud]

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
        t0 = time.perf_counter()

        def retire(token, group):
            _, vbs, fbs, _ = token
            if self.on_result is not None:
                for r, vb, fb in zip(group, vbs, fbs):
                    self.on_result(r, vb, fb)

        done = self.scheduler.run(requests, launch=self._launch, is_done=lambda tok: tok[0].query(),
                                  retire=retire, now=lambda: time.perf_counter() - t0,
                                  idle=(lambda: time.sleep(idle_sleep)) if idle_sleep else None)
        for ctx in self.ctxs:
            B.pr_sync(ctx.handle)
        return done

    def close(self):
        for ctx in self.ctxs:
            ctx.close()

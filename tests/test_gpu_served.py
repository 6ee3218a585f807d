"""Served mode: continuous batching over resident clouds gives every request its solo render.

Three terrain clouds are built and reduced to their render buffers (pr_cloud_drop_load_buffers).  A seeded
request stream (mixed image sizes, cameras over each cloud's terrain) starts with a burst of simultaneous
requests, so that several requests share a multi-view launch, and runs under a small memory budget, so that
admission has to wait for retirements, on three streams.  Every result must equal the request's solo render
(one view per launch, on another context) and, for the cloud the oracle also built, the oracle; every request
completes once, after it arrived; the bytes in flight never exceed the budget (or one oversize request).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_vb_equal, say

pytestmark = pytest.mark.gpu

CLEAR = 0xFF000000


def test_served_results_equal_solo_renders():
    import torch
    import paper_2204_01287_amd as pr
    from paper_2204_01287_amd.serve import Request, Server

    ctx = pr.Context(0)
    specs = [(11, 400_000), (12, 1_000_000), (13, 2_000_000)]
    clouds = []
    B = None
    for seed, n in specs:
        xyz, rgba = synth.terrain(seed, n, order=1)
        say(f"served: build cloud seed={seed} n={n}")
        dc = pr.DeviceCloud(ctx, xyz, rgba, batch_size=10240, morton=True)
        if B is None:
            B = oracle.build_cloud(xyz, rgba, 10240, morton=True)
        dc.drop_load_buffers()
        clouds.append(dc)
    torch.cuda.empty_cache()
    sizes = [(160, 120), (320, 240), (97, 61), (640, 360)]
    stream = synth.request_stream(21, 60, 3000.0, [s for s, _ in specs], sizes=sizes)
    reqs = [Request(i, c, cam, 0.0 if i < 24 else a) for i, (a, c, cam) in enumerate(stream)]
    got = {}

    def keep(r, vb, fb):
        got[r.rid] = (vb.cpu().numpy().view(np.uint64).copy(), fb.cpu().numpy().view(np.uint32).copy())

    budget = 2_000_000
    srv = Server(clouds, nstreams=3, budget_bytes=budget, on_result=keep)
    say("served: run 60 requests")
    done = srv.run(reqs)
    srv.close()
    assert sorted(d.rid for d in done) == list(range(len(reqs)))
    assert max(d.group for d in done) > 1, "no request shared a launch"
    assert srv.peak_bytes <= max(budget, max(srv.request_bytes(r) for r in reqs))
    assert all(d.completed >= d.launched >= d.arrival - 1e-6 for d in done)
    assert len({d.stream for d in done}) > 1

    say("served: solo renders")
    solo = pr.Context(0)
    for r in reqs:
        c, h = r.cam, clouds[r.cloud].handle
        vb = torch.empty(c.width * c.height, dtype=torch.int64, device="cuda")
        fb = torch.empty(c.width * c.height, dtype=torch.int32, device="cuda")
        need = pr.pr_views_work_bytes(h, 1)
        work = torch.empty(need, dtype=torch.uint8, device="cuda")
        pr.pr_render_views(solo.handle, h, [(c.view, c.proj, c.width, c.height, vb)], None, work, need)
        pr.pr_resolve(solo.handle, h, vb, c.width, c.height, CLEAR, fb)
        pr.pr_sync(solo.handle)
        v = vb.cpu().numpy().view(np.uint64)
        assert np.array_equal(got[r.rid][0], v), f"request {r.rid}: visibility buffer differs from its solo render"
        assert np.array_equal(got[r.rid][1], fb.cpu().numpy().view(np.uint32))
        if r.cloud == 0:
            ref, _ = oracle.render(B, c.view, c.proj, c.width, c.height)
            assert_vb_equal(v, ref, c.width)
    # the dropped scratch is not used again: single-view renders are refused
    cam = reqs[0].cam
    vb = torch.empty(cam.width * cam.height, dtype=torch.int64, device="cuda")
    with pytest.raises(pr.PrError, match="PR_ESTATE"):
        pr.pr_render(solo.handle, clouds[0].handle, cam.view, cam.proj, cam.width, cam.height, None, vb)
    solo.close()
    for dc in clouds:
        dc.close()
    ctx.close()

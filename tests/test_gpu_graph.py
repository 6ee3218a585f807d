"""Frames captured into HIP graphs (torch.cuda.CUDAGraph over the library's launches) and replayed.

The stereo frame of a 2M-point Morton terrain is captured twice: one launch sequence per eye (eye 0: render, which
clears the buffer in its classify launch, and resolve; eye 1: clear, accumulating render, resolve) and both eyes
through pr_render_views.  Each graph is replayed three times with the program's own eager
renders and synchronisations in between, and with the output buffers overwritten before each replay; every replay
must reproduce the eager frame bit for bit, and the eager frame equals the oracle.  The captured work is kernels
only (the clears are kernels, no memset nodes).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_vb_equal, say

pytestmark = pytest.mark.gpu

CLEAR = 0xFF000000


def test_graph_replays_match_eager():
    import torch
    import paper_2204_01287_amd as pr

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = pr.Context(0, stream=s)
        xyz, rgba = synth.terrain(synth.C2_SEED, 2_000_000, order=1)
        say("graph: build 2M terrain")
        dc = pr.DeviceCloud(ctx, xyz, rgba, batch_size=10240, morton=True)
        B = oracle.build_cloud(xyz, rgba, 10240, morton=True)
        cams = synth.stereo_cameras(synth.C2_SEED, 504, 560)
        npx = [c.width * c.height for c in cams]
        vb_a = [torch.empty(n, dtype=torch.int64, device="cuda") for n in npx]
        fb_a = [torch.empty(n, dtype=torch.int32, device="cuda") for n in npx]
        vb_b = [torch.empty(n, dtype=torch.int64, device="cuda") for n in npx]
        fb_b = [torch.empty(n, dtype=torch.int32, device="cuda") for n in npx]
        need = pr.pr_views_work_bytes(dc.handle, len(cams))
        work = torch.empty(need, dtype=torch.uint8, device="cuda")
        acc = pr.RenderOpts.make(accumulate=1)

        def plain():
            # eye 0 as bench.py renders it (pr_render clears in its classify launch), eye 1 through pr_clear and an
            # accumulating render
            for i, (c, vb, fb) in enumerate(zip(cams, vb_a, fb_a)):
                if i == 0:
                    pr.pr_render(ctx.handle, dc.handle, c.view, c.proj, c.width, c.height, None, vb)
                else:
                    pr.pr_clear(ctx.handle, vb, c.width, c.height)
                    pr.pr_render(ctx.handle, dc.handle, c.view, c.proj, c.width, c.height, acc, vb)
                pr.pr_resolve(ctx.handle, dc.handle, vb, c.width, c.height, CLEAR, fb)

        def views():
            pr.pr_render_views(ctx.handle, dc.handle, [(c.view, c.proj, c.width, c.height, vb) for c, vb in
                                                       zip(cams, vb_b)], None, work, need)
            for c, vb, fb in zip(cams, vb_b, fb_b):
                pr.pr_resolve(ctx.handle, dc.handle, vb, c.width, c.height, CLEAR, fb)

        def host(ts):
            return [t.cpu().numpy().copy() for t in ts]

        say("graph: eager frames")
        plain()
        views()
        torch.cuda.synchronize()
        ref = (host(vb_a), host(fb_a), host(vb_b), host(fb_b))
        for c, v, f in zip(cams, ref[0], ref[1]):
            o, _ = oracle.render(B, c.view, c.proj, c.width, c.height)
            assert_vb_equal(v.view(np.uint64), o, c.width)
            assert np.array_equal(f.view(np.uint32), oracle.resolve(o, B.colors, CLEAR))
        for a, b in zip(ref[0] + ref[1], ref[2] + ref[3]):
            assert np.array_equal(a, b)

        say("graph: capture")
        g_plain, g_views = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
        with torch.cuda.graph(g_plain, stream=s):
            plain()
        with torch.cuda.graph(g_views, stream=s):
            views()
        other = synth.orbit_camera(17, width=320, height=200)
        scratch = torch.empty(other.width * other.height, dtype=torch.int64, device="cuda")
        for rep in range(3):
            say(f"graph: replay {rep}")
            for t in vb_a + fb_a + vb_b + fb_b:
                t.fill_(rep + 1)
            torch.cuda.synchronize()
            g_plain.replay()
            torch.cuda.synchronize()
            assert all(np.array_equal(a, b) for a, b in zip(host(vb_a) + host(fb_a), ref[0] + ref[1]))
            # the program's own eager work between replays
            pr.pr_render(ctx.handle, dc.handle, other.view, other.proj, other.width, other.height, None, scratch)
            pr.pr_sync(ctx.handle)
            g_views.replay()
            torch.cuda.synchronize()
            assert all(np.array_equal(a, b) for a, b in zip(host(vb_b) + host(fb_b), ref[2] + ref[3]))
        o, _ = oracle.render(B, other.view, other.proj, other.width, other.height)
        assert_vb_equal(scratch.cpu().numpy().view(np.uint64), o, other.width)
        del g_plain, g_views
        dc.close()
        ctx.close()

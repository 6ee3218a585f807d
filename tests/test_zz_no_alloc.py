"""pr_render_views_static (the frame of pr_render_views with its work area in the library's static device array,
for callers that cannot allocate) against pr_render_views with a caller-owned work buffer.

Two calls in a row, the second with a smaller input (a cloud with fewer batches and fewer, smaller views), so the
second frame runs over what the first left in the shared array: each call's visibility buffers and counters must
equal those of pr_render_views on the same views bit for bit, and one view of each equals the oracle.  A frame that
needs more than the static area is refused with PR_ERANGE before anything is enqueued.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_vb_equal, gpu_build, oracle_stats_match, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2204_01287_amd as pr

    assert torch.cuda.is_available()
    c = pr.Context(0)
    yield c
    c.close()


def _frames(ctx, dc, cams, counters):
    """The same frame through pr_render_views (work buffer) and pr_render_views_static; host copies of both."""
    import torch
    import paper_2204_01287_amd as pr

    o = pr.RenderOpts.make(counters=counters)
    vbs_w = [torch.empty(c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]
    vbs_s = [torch.full((c.width * c.height,), 3, dtype=torch.int64, device="cuda") for c in cams]
    need = pr.pr_views_work_bytes(dc.handle, len(cams))
    assert need <= pr.PR_STATIC_WORK_BYTES
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    say(f"pr_render_views n={dc.n} nb={dc.nb} views={len(cams)}")
    pr.pr_render_views(ctx.handle, dc.handle, [(c.view, c.proj, c.width, c.height, vb) for c, vb in zip(cams, vbs_w)],
                       o, work, need)
    st_w = pr.pr_get_stats(ctx.handle) if counters else None
    pr.pr_sync(ctx.handle)
    say(f"pr_render_views_static n={dc.n} nb={dc.nb} views={len(cams)}")
    pr.pr_render_views_static(ctx.handle, dc.handle,
                              [(c.view, c.proj, c.width, c.height, vb) for c, vb in zip(cams, vbs_s)], o)
    st_s = pr.pr_get_stats(ctx.handle) if counters else None
    pr.pr_sync(ctx.handle)
    got_w = [v.cpu().numpy().view(np.uint64).copy() for v in vbs_w]
    got_s = [v.cpu().numpy().view(np.uint64).copy() for v in vbs_s]
    return got_w, got_s, st_w, st_s


def test_static_work_two_calls_second_smaller(ctx):
    # first call: a 2M-point Morton terrain (196 batches), a stereo pair and an orbit view
    xyz, rgba = synth.terrain(synth.C2_SEED, 2_000_000, order=1)
    dc1 = gpu_build(ctx, xyz, rgba, 10240, True)
    B1 = oracle.build_cloud(xyz, rgba, 10240, morton=True)
    cams1 = list(synth.stereo_cameras(synth.C3_SEED, width=640, height=720)) + [synth.orbit_camera(5, width=800, height=600)]
    w1, s1, stw1, sts1 = _frames(ctx, dc1, cams1, counters=1)
    for c, a, b in zip(cams1, w1, s1):
        assert_vb_equal(b, a, c.width)
    oracle_stats_match(sts1, stw1)  # the deterministic counters (the atomics count depends on timing)
    ref, _ = oracle.render(B1, cams1[2].view, cams1[2].proj, cams1[2].width, cams1[2].height)
    assert_vb_equal(s1[2], ref, cams1[2].width)
    assert np.count_nonzero(ref != oracle.EMPTY) > 0
    # second call, smaller: C1's 8 primitives at 300k points (30 batches, no Morton), one 320x200 view
    xyz2, rgba2 = synth.primitives(synth.C1_SEED, 300_000)
    dc2 = gpu_build(ctx, xyz2, rgba2, 10240, False)
    assert dc2.nb < dc1.nb
    B2 = oracle.build_cloud(xyz2, rgba2, 10240, morton=False)
    cam2 = synth.camera((50.0, -90.0, 120.0), (50.0, 50.0, 50.0), (0.0, 0.0, 1.0), 60.0, 320, 200, 0.5, 1000.0)
    w2, s2, stw2, sts2 = _frames(ctx, dc2, [cam2], counters=0)
    assert_vb_equal(s2[0], w2[0], cam2.width)
    ref2, _ = oracle.render(B2, cam2.view, cam2.proj, cam2.width, cam2.height)
    assert_vb_equal(s2[0], ref2, cam2.width)
    assert np.count_nonzero(ref2 != oracle.EMPTY) > 0
    dc1.close()
    dc2.close()


def test_static_work_too_large_is_refused(ctx):
    import torch
    import paper_2204_01287_amd as pr

    # 60,000 points in batches of 4: 15,000 batches; 64 views need 15,000 x 64 x 80 bytes > 64 MiB
    xyz, rgba = synth.primitives(synth.C1_SEED, 60_000)
    dc = gpu_build(ctx, xyz, rgba, 4, False)
    cam = synth.camera((50.0, -90.0, 120.0), (50.0, 50.0, 50.0), (0.0, 0.0, 1.0), 60.0, 64, 64, 0.5, 1000.0)
    vbs = [torch.full((64 * 64,), 9, dtype=torch.int64, device="cuda") for _ in range(64)]
    assert pr.pr_views_work_bytes(dc.handle, 64) > pr.PR_STATIC_WORK_BYTES
    say("pr_render_views_static beyond the static area (must be refused)")
    with pytest.raises(pr.PrError) as e:
        pr.pr_render_views_static(ctx.handle, dc.handle, [(cam.view, cam.proj, 64, 64, vb) for vb in vbs], None)
    assert e.value.name == "PR_ERANGE"
    assert "static area" in str(e.value)
    pr.pr_sync(ctx.handle)
    assert all(int(v.min()) == 9 and int(v.max()) == 9 for v in vbs)  # nothing was enqueued
    # within the limit the same cloud renders (one view) and equals pr_render_views
    w, s, _, _ = _frames(ctx, dc, [cam], counters=0)
    assert_vb_equal(s[0], w[0], 64)
    dc.close()

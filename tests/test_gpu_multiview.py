"""Several views in one launch (pr_render_views) against the oracle and against single-view renders.

Every view's visibility buffer must equal, bit for bit, the oracle's render of that view alone and the GPU's
pr_render of that view; the counters sum over all (batch, view) pairs.  Covered: stereo pairs, camera arrays of
mixed resolutions (more views than one classify launch takes), cameras inside the cloud and looking away, every
precision mode, accumulate, and the argument checks.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import MODES, assert_vb_equal, gpu_build, gpu_render, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2204_01287_amd as pr

    assert torch.cuda.is_available()
    c = pr.Context(0)
    yield c
    c.close()


def _cloud(ctx, xyz, rgba, S, morton):
    say(f"build n={len(xyz)} S={S} morton={morton}")
    return gpu_build(ctx, xyz, rgba, S, morton), oracle.build_cloud(xyz, rgba, S, morton=morton)


@pytest.fixture(scope="module")
def c1(ctx):
    xyz, rgba = synth.primitives(synth.C1_SEED, 1_000_000)
    return _cloud(ctx, xyz, rgba, 10240, False)


@pytest.fixture(scope="module")
def terrain(ctx):
    xyz, rgba = synth.terrain(synth.C2_SEED, 2_000_000, order=1)
    return _cloud(ctx, xyz, rgba, 10240, True)


def _render_views(ctx, dc, cams, counters=0, accumulate=0, vbs=None, **opt):
    import torch
    import paper_2204_01287_amd as pr

    if vbs is None:
        vbs = [torch.empty(c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]
    nbytes = pr.pr_views_work_bytes(dc.handle, len(cams))
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    o = pr.RenderOpts.make(counters=counters, accumulate=accumulate, **opt)
    say(f"render_views n={dc.n} views={len(cams)} opts={opt}")
    pr.pr_render_views(ctx.handle, dc.handle, [(c.view, c.proj, c.width, c.height, vb) for c, vb in zip(cams, vbs)], o,
                       work, nbytes)
    st = pr.pr_get_stats(ctx.handle) if counters else None
    pr.pr_sync(ctx.handle)
    return [vb.cpu().numpy().view(np.uint64) for vb in vbs], st


def _check(ctx, dc, B, cams, mode="adaptive"):
    opt = dict(MODES[mode])
    vbs, st = _render_views(ctx, dc, cams, counters=1, **opt)
    o = oracle.opts(precision=opt.get("precision", 0), cull=opt.get("cull", 1))
    tot = {"batches": 0, "culled": 0, "points": 0, "level_batches": [0, 0, 0], "level_points": [0, 0, 0]}
    for c, vb in zip(cams, vbs):
        ref, s = oracle.render(B, c.view, c.proj, c.width, c.height, o)
        assert_vb_equal(vb, ref, c.width)
        single, _, _ = gpu_render(ctx, dc, c.view, c.proj, c.width, c.height, counters=0, **opt)
        assert np.array_equal(single, vb)
        for k in ("batches", "culled", "points"):
            tot[k] += s[k]
        for k in ("level_batches", "level_points"):
            tot[k] = [a + b for a, b in zip(tot[k], s[k])]
    for k in tot:
        assert st[k] == tot[k], (k, st[k], tot[k])
    # coordinate words the frame streams: per batch and classify launch (16 views), at the highest level among
    # the batch's live views there (the oracle's per-batch decisions)
    words = 0
    count = B.batches["count"].astype(np.uint64)
    for c0 in range(0, len(cams), 16):
        lmax = np.zeros(len(B.batches), np.int64)
        for c in cams[c0:c0 + 16]:
            d = oracle.decide_all(B.batches, c.view, c.proj, c.width, c.height, o)
            lv = np.where(d["culled"] == 0, d["level"] // 10, 0)
            lmax = np.maximum(lmax, lv)
        words += int((4 * lmax.astype(np.uint64) * count).sum())
    assert st["words_bytes"] == words, (st["words_bytes"], words)
    _, _, s1 = gpu_render(ctx, dc, cams[0].view, cams[0].proj, cams[0].width, cams[0].height, counters=1, **opt)
    lp = s1["level_points"]
    assert s1["words_bytes"] == 4 * lp[0] + 8 * lp[1] + 12 * lp[2]
    return vbs


def _cams(seed, n, box, sizes, inside_every=0):
    rng = np.random.default_rng(seed)
    return [synth.random_camera(rng, *sizes[i % len(sizes)], inside=bool(inside_every and i % inside_every == 0),
                                box=box) for i in range(n)]


@pytest.mark.parametrize("mode", list(MODES))
def test_c1_view_set(ctx, c1, mode):
    dc, B = c1
    cams = [synth.c1_camera()] + _cams(7, 4, ((0, 0, 0), (100, 100, 100)), [(320, 200), (256, 256), (97, 61)], 3)
    _check(ctx, dc, B, cams, mode)


def test_stereo_pair(ctx, terrain):
    dc, B = terrain
    cams = synth.stereo_cameras(synth.C2_SEED, 504, 560)
    _check(ctx, dc, B, cams)


def test_stereo_pair_spread_order(ctx):
    """The two-view pass over a build in the spread order (PR_ORDER_MORTON_SPREAD), with a third view of another
    size in the same launch."""
    xyz, rgba = synth.terrain(synth.C2_SEED, 1_000_000, order=1)
    dc, B = _cloud(ctx, xyz, rgba, 10240, 2)
    cams = synth.stereo_cameras(synth.C2_SEED, 504, 560) + [synth.orbit_camera(7, width=640, height=360)]
    _check(ctx, dc, B, cams)


def test_more_views_than_one_classify_launch(ctx, terrain):
    """20 views of mixed sizes: two classify launches, runs of both in one render launch."""
    dc, B = terrain
    cams = _cams(11, 20, ((0, 0, -60), (1000, 1000, 120)), [(160, 120), (200, 200), (64, 48), (333, 77)], 6)
    cams.append(synth.orbit_camera(5, width=480, height=270))
    _check(ctx, dc, B, cams)


def test_view_looking_away_renders_nothing(ctx, c1):
    dc, B = c1
    away = synth.camera((50, 50, 300), (50, 50, 1000), (0, 1, 0), 40.0, 128, 96, 0.5, 1000.0)
    vbs = _check(ctx, dc, B, [synth.c1_camera(), away])
    assert np.all(vbs[1] == oracle.EMPTY) and np.any(vbs[0] != oracle.EMPTY)


def test_accumulate_combines_by_minimum(ctx, c1):
    import torch

    dc, B = c1
    cams = _cams(3, 3, ((0, 0, 0), (100, 100, 100)), [(200, 150)])
    first, _ = _render_views(ctx, dc, cams)
    other = _cams(4, 3, ((0, 0, 0), (100, 100, 100)), [(200, 150)])
    # render the second camera set on top of the first images
    vbs = [torch.from_numpy(v.view(np.int64).copy()).cuda() for v in first]
    both, _ = _render_views(ctx, dc, other, accumulate=1, vbs=vbs)
    for o, f, b in zip(other, first, both):
        ref, _ = oracle.render(B, o.view, o.proj, o.width, o.height)
        assert np.array_equal(b, np.minimum(f, ref))


def test_argument_checks(ctx, c1):
    import torch
    import paper_2204_01287_amd as pr

    dc, _ = c1
    cam = synth.c1_camera()
    vb = torch.empty(cam.width * cam.height, dtype=torch.int64, device="cuda")
    with pytest.raises(pr.PrError, match="PR_ERANGE"):
        pr.pr_views_work_bytes(dc.handle, 0)
    with pytest.raises(pr.PrError, match="PR_ERANGE"):
        pr.pr_views_work_bytes(dc.handle, pr.PR_MAX_VIEWS + 1)
    need = pr.pr_views_work_bytes(dc.handle, 1)
    work = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    views = [(cam.view, cam.proj, cam.width, cam.height, vb)]
    with pytest.raises(pr.PrError, match="PR_EINVAL"):
        pr.pr_render_views(ctx.handle, dc.handle, views, None, work, 64)
    with pytest.raises(pr.PrError, match="PR_EINVAL"):
        pr.pr_render_views(ctx.handle, dc.handle, views, None, work.data_ptr() + 16, need)
    with pytest.raises(pr.PrError, match="PR_ERANGE"):
        pr.pr_render_views(ctx.handle, dc.handle, [(cam.view, cam.proj, 0, 5, vb)], None, work, need)
    bad = np.array(cam.view, copy=True)
    bad[0, 0] = np.nan
    with pytest.raises(pr.PrError, match="PR_ENONFINITE"):
        pr.pr_render_views(ctx.handle, dc.handle, [(bad, cam.proj, cam.width, cam.height, vb)], None, work, need)
    pr.pr_sync(ctx.handle)

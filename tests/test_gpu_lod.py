"""Level-of-detail layouts (Sec. 3.5): variable-size batches and node culling on the GPU against the oracle.

A 1M-point terrain and the 1M-point primitives are converted to layered-point-cloud layouts (synth.lpc_layout),
built with pr_build_batches_spans and rendered with lod_px = 0 (every node), 100 (the paper's suggestion) and 400;
visibility buffers, framebuffers and counters must equal the oracle's bit for bit, also through pr_render_views and
pr_render_hqs; the build's batch records and Eq. 1 words equal the oracle's inside every span.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_vb_equal, gpu_render, oracle_stats_match, say

pytestmark = pytest.mark.gpu

CAP = 4096


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2204_01287_amd as pr

    assert torch.cuda.is_available()
    c = pr.Context(0)
    yield c
    c.close()


def _lpc(ctx, xyz, rgba, seed):
    import paper_2204_01287_amd as pr

    xo, ro, spans, nodes = synth.lpc_layout(seed, xyz, rgba, synth.lpc_depth(len(xyz), CAP), CAP)
    say(f"lod: build {len(spans)} batches over {len(xo)} slots")
    dc = pr.DeviceCloud(ctx, xo, ro, spans=spans, nodes=nodes)
    B = oracle.build_cloud_spans(xo, ro, spans, nodes)
    return dc, B, spans


@pytest.fixture(scope="module")
def terrain(ctx):
    xyz, rgba = synth.terrain(synth.C2_SEED, 1_000_000, order=1)
    return _lpc(ctx, xyz, rgba, 31)


@pytest.fixture(scope="module")
def prims(ctx):
    xyz, rgba = synth.primitives(synth.C1_SEED, 1_000_000)
    return _lpc(ctx, xyz, rgba, 32)


def test_build(terrain):
    import torch

    dc, B, spans = terrain
    assert dc.nb == len(spans)
    gb = dc.view("batches", torch.uint8, 32 * dc.nb).cpu().numpy()
    assert np.array_equal(gb, B.batches.view(np.uint8))
    idx = np.concatenate([np.arange(f, f + c) for f, c in spans])
    for f in ("low", "med", "high"):
        g = dc.view(f, torch.int32, dc.n).cpu().numpy().view(np.uint32)
        assert np.array_equal(g[idx], getattr(B, f)[idx]), f
    assert np.array_equal(dc.view("colors", torch.int32, dc.n).cpu().numpy().view(np.uint32), B.colors)


def _check(ctx, dc, B, cam, lod_px, **opt):
    vb, fb, st = gpu_render(ctx, dc, cam.view, cam.proj, cam.width, cam.height, clear_rgba=0xFF000000, lod_px=lod_px,
                            **opt)
    o = oracle.opts(precision=opt.get("precision", 0), cull=opt.get("cull", 1), lod_px=lod_px)
    ref, st_ref = oracle.render(B, cam.view, cam.proj, cam.width, cam.height, o)
    assert_vb_equal(vb, ref, cam.width)
    assert np.array_equal(fb, oracle.resolve(ref, B.colors, 0xFF000000))
    oracle_stats_match(st, st_ref)
    return st


@pytest.mark.parametrize("lod_px", [0.0, 100.0, 400.0])
def test_terrain_views(ctx, terrain, lod_px):
    dc, B, _ = terrain
    cams = [synth.orbit_camera(3, width=960, height=540)] + synth.stereo_cameras(synth.C2_SEED, 504, 560)
    culled = [_check(ctx, dc, B, cam, lod_px)["culled"] for cam in cams]
    if lod_px >= 100.0:
        assert max(culled) > 0


def test_lod_culls_more_with_a_larger_threshold(ctx, terrain):
    dc, B, _ = terrain
    cam = synth.orbit_camera(11, width=640, height=360)
    pts = [_check(ctx, dc, B, cam, lod)["points"] for lod in (0.0, 50.0, 200.0, 800.0)]
    assert pts[0] >= pts[1] >= pts[2] >= pts[3] and pts[3] < pts[0]


def test_primitives_random_cameras(ctx, prims):
    dc, B, _ = prims
    rng = np.random.default_rng(8)
    for i in range(4):
        cam = synth.random_camera(rng, 320, 240, inside=(i == 0), box=((0, 0, 0), (100, 100, 100)))
        _check(ctx, dc, B, cam, 100.0)
        _check(ctx, dc, B, cam, 100.0, precision=30, cull=0)


def test_multiview_and_hqs_with_lod(ctx, terrain):
    import torch
    import paper_2204_01287_amd as pr

    dc, B, _ = terrain
    cams = synth.stereo_cameras(synth.C2_SEED, 504, 560) + [synth.orbit_camera(20, width=320, height=200)]
    o = oracle.opts(lod_px=100.0)
    vbs = [torch.empty(c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]
    need = pr.pr_views_work_bytes(dc.handle, len(cams))
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    pr.pr_render_views(ctx.handle, dc.handle, [(c.view, c.proj, c.width, c.height, vb) for c, vb in zip(cams, vbs)],
                       pr.RenderOpts.make(lod_px=100.0), work, need)
    pr.pr_sync(ctx.handle)
    for c, vb in zip(cams, vbs):
        ref, _ = oracle.render(B, c.view, c.proj, c.width, c.height, o)
        assert_vb_equal(vb.cpu().numpy().view(np.uint64), ref, c.width)
    c = cams[0]
    vb = torch.empty(c.width * c.height, dtype=torch.int64, device="cuda")
    acc = torch.empty(2 * c.width * c.height, dtype=torch.int64, device="cuda")
    fb = torch.empty(c.width * c.height, dtype=torch.int32, device="cuda")
    pr.pr_render_hqs(ctx.handle, dc.handle, c.view, c.proj, c.width, c.height, pr.RenderOpts.make(lod_px=100.0), 1.01,
                     vb, acc, 0, fb)
    pr.pr_sync(ctx.handle)
    ref, _ = oracle.render(B, c.view, c.proj, c.width, c.height, o)
    racc = oracle.accumulate(B, c.view, c.proj, c.width, c.height, ref, window=1.01, o=o)
    assert np.array_equal(acc.cpu().numpy().view(np.uint64), racc)


def test_argument_checks(ctx):
    import torch
    import paper_2204_01287_amd as pr

    xyz, rgba = synth.terrain(3, 4000, order=1)
    sizes = pr.pr_cloud_sizes_spans(4000, 2)
    mem = {f: torch.empty(max(getattr(sizes, f), 256), dtype=torch.uint8, device="cuda") for f in pr.BUFFER_FIELDS}
    bufs = pr.CloudBufs(*[mem[f].data_ptr() for f in pr.BUFFER_FIELDS], sizes)
    h = pr.pr_load_points(ctx.handle, xyz, rgba, 4000, False, bufs)
    for bad in ([[2, 10], [100, 10]], [[0, 10], [8, 10]], [[0, 10], [3996, 8]], [[0, 0], [16, 4]]):
        with pytest.raises(pr.PrError, match="PR_EINVAL"):
            pr.pr_build_batches_spans(ctx.handle, h, np.array(bad, np.uint32))
    pr.pr_build_batches_spans(ctx.handle, h, np.array([[0, 2000], [2000, 2000]], np.uint32))
    cam = synth.orbit_camera(0, width=64, height=48)
    vb = torch.empty(64 * 48, dtype=torch.int64, device="cuda")
    with pytest.raises(pr.PrError, match="PR_EINVAL"):
        pr.pr_render(ctx.handle, h, cam.view, cam.proj, 64, 48, pr.RenderOpts.make(lod_px=float("nan")), vb)
    pr.pr_render(ctx.handle, h, cam.view, cam.proj, 64, 48, pr.RenderOpts.make(lod_px=100.0), vb)  # no nodes: no LOD
    pr.pr_sync(ctx.handle)
    pr.pr_cloud_free(h)

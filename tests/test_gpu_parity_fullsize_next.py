"""Parity at the full sizes of the camera-array and level-of-detail workloads, in the configurations bench.py times.

C4 -- 500,000,000-point terrain (seed 4, index order, Morton build, 10,240 points per batch) and 64 cameras of
1024 x 1024 (synth.camera_array).  The device's Morton build is checked against the oracle chunk by chunk as for C3
(the permutation is proved to be the unique stable order; positions, colours, batch records and Eq. 1 words are
the oracle's).  The frame is bench.py's: pr_autotune over the 64-view frame, then all 64 views in one
pr_render_views launch under the winning tuning.  Every one of the 64 views equals the oracle's render pixel for
pixel (threaded oracle, interleaved batch sets merged by elementwise minimum), and also its single-view render under
the default tuning.

C6 -- the 500,000,000-point terrain (seed 3, index order) converted to a layered point cloud (seed 7, batches of at
most 10,240 points, 227,804 variable-size batches), as bench.py's LOD leg.  The spans build (batch records, Eq. 1
words inside every span) equals the oracle's; both eyes of the stereo pair at lod_px 100 (plain frames, default
tuning, and again under the autotuned tuning) and eye 0 at lod_px 0 equal the oracle's visibility buffers,
framebuffers and counters.
"""
from __future__ import annotations

import types
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
from fullsize_util import CLEAR, _t, _u32, check_morton_build, device_views, oracle_frame
from gpu_util import assert_vb_equal, oracle_stats_match, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 500_000_000
CAP = 10240


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2204_01287_amd as pr

    assert torch.cuda.is_available()
    c = pr.Context(0)
    yield c
    pr.pr_set_tuning(c.handle)
    c.close()


# =================================================================== C4: camera array
@pytest.fixture(scope="module")
def c4(ctx):
    import torch
    import bench

    wl = dict(name="terrain_c4", seed=4, n=N, morton=2, order=0, batch_size=10240)
    boxes = []
    pool = ThreadPoolExecutor(2)

    def box(lo, hi, xyz, rgba):
        f = pool.submit(oracle.cloud_aabb, xyz)
        boxes.append(f)
        return f

    say(f"C4: generate and build {N} points on the GPU")
    cloud = bench.load_cloud(ctx, wl, on_chunk=box)
    pool.shutdown()
    corners = np.array([c for f in boxes for c in f.result()], np.float32)
    ns = types.SimpleNamespace(wl=wl, cloud=cloud, n=N, nb=cloud["nb"], cloud_box=oracle.cloud_aabb(corners))
    ns.res, ns.built, ns.colors = check_morton_build(ns, "C4")
    yield ns
    import paper_2204_01287_amd as pr

    pr.pr_cloud_free(cloud["handle"])
    cloud.clear()
    torch.cuda.empty_cache()


def test_c4_build_full(c4):
    res = sorted(c4.res, key=lambda r: r["lo"])
    for r in res:
        for k in ("mono", "stable", "xyz", "colors", "low", "med", "high", "batches"):
            assert r[k], f"chunk at {r['lo']}: {k} check failed"
    for a, b in zip(res, res[1:]):
        assert a["tail"][0] <= b["head"][0], f"Morton order broken at {b['lo']}"
        if a["tail"][0] == b["head"][0]:
            assert a["tail"][1] < b["head"][1], f"stability broken at {b['lo']}"


def test_c4_camera_array_autotuned_one_launch(ctx, c4):
    import torch
    import paper_2204_01287_amd as pr

    cams = synth.camera_array(4, 64, 1024, 1024)
    h = c4.cloud["handle"]
    vbs = [torch.empty(c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]
    views = [(c.view, c.proj, c.width, c.height, vb) for c, vb in zip(cams, vbs)]
    need = pr.pr_views_work_bytes(h, len(cams))
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    say("C4: pr_autotune over the 64-view frame")
    best, trials = pr.pr_autotune(ctx.handle, h, views, None, work, need, 2)
    say(f"C4: winner {best} {pr.pr_raster_shapes(ctx.handle)[best['shape']]}; 64 views in one launch")
    pr.pr_render_views(ctx.handle, h, views, None, work, need)
    pr.pr_sync(ctx.handle)
    got = [vb.cpu().numpy().view(np.uint64).copy() for vb in vbs]
    covered = [int(np.count_nonzero(g != oracle.EMPTY)) for g in got]
    say(f"C4: all 64 views against the oracle (covered pixels: min {min(covered)}, max {max(covered)})")
    t0 = _t()
    seen = 0
    for i, cam in enumerate(cams):
        ref, _ = oracle_frame(c4.built, cam, c4.nb)
        assert_vb_equal(got[i], ref, cam.width)
        seen += int(np.count_nonzero(ref != oracle.EMPTY) > 0)
        if i % 8 == 7:
            say(f"C4: {i + 1} views equal the oracle ({_t() - t0:.1f} s)")
    assert seen >= 32, "most cameras of the array must see the terrain"
    pr.pr_set_tuning(ctx.handle)
    one = torch.empty(1024 * 1024, dtype=torch.int64, device="cuda")
    for i, c in enumerate(cams):
        pr.pr_render(ctx.handle, h, c.view, c.proj, c.width, c.height, None, one)
        pr.pr_sync(ctx.handle)
        assert np.array_equal(one.cpu().numpy().view(np.uint64), got[i]), f"view {i} differs from its single render"


# =================================================================== C6: LOD
@pytest.fixture(scope="module")
def c6(ctx):
    import torch
    import paper_2204_01287_amd as pr

    t0 = _t()
    say(f"C6: generate {N} points and convert them to a layered point cloud")
    xyz, rgba = synth.terrain(synth.C3_SEED, N, order=0)
    xo, ro, spans, nodes = synth.lpc_layout(7, xyz, rgba, synth.lpc_depth(N, CAP), CAP)
    del xyz, rgba
    say(f"C6: {len(spans)} batches over {len(xo)} slots ({_t() - t0:.1f} s); spans build on the GPU")
    dc = pr.DeviceCloud(ctx, xo, ro, spans=spans, nodes=nodes)
    say(f"C6: oracle spans build ({_t() - t0:.1f} s)")
    B = oracle.build_cloud_spans(xo, ro, spans, nodes)
    say(f"C6: ready ({_t() - t0:.1f} s)")
    yield types.SimpleNamespace(dc=dc, B=B, spans=spans, nb=len(spans))
    dc.close()
    del dc
    torch.cuda.empty_cache()


def test_c6_spans_build_full(c6):
    import torch

    dc, B, spans = c6.dc, c6.B, c6.spans
    assert np.array_equal(dc.view("batches", torch.uint8, 32 * c6.nb).cpu().numpy(), B.batches.view(np.uint8))
    inside = np.zeros(dc.n, bool)
    for f, c in spans:
        inside[f:f + c] = True
    step = 1 << 26
    for f in ("low", "med", "high"):
        g = getattr(B, f)
        for lo in range(0, dc.n, step):
            hi = min(dc.n, lo + step)
            got = _u32(dc.view(f, torch.int32, dc.n)[lo:hi])
            m = inside[lo:hi]
            assert np.array_equal(got[m], g[lo:hi][m]), f"{f} words differ in [{lo}, {hi})"
    colors = _u32(dc.view("colors", torch.int32, dc.n))
    assert np.array_equal(colors[inside], B.colors[inside])


def _lod_frame(ctx, dc, cam, lod_px):
    """One eye as bench.py's LOD leg times it (pr_render + pr_resolve), then its counters frame."""
    import torch
    import paper_2204_01287_amd as pr

    vb = torch.empty(cam.width * cam.height, dtype=torch.int64, device="cuda")
    fb = torch.empty(cam.width * cam.height, dtype=torch.int32, device="cuda")
    pr.pr_render(ctx.handle, dc.handle, cam.view, cam.proj, cam.width, cam.height, pr.RenderOpts.make(lod_px=lod_px),
                 vb)
    pr.pr_resolve(ctx.handle, dc.handle, vb, cam.width, cam.height, CLEAR, fb)
    pr.pr_sync(ctx.handle)
    out = vb.cpu().numpy().view(np.uint64).copy(), fb.cpu().numpy().view(np.uint32).copy()
    pr.pr_render(ctx.handle, dc.handle, cam.view, cam.proj, cam.width, cam.height,
                 pr.RenderOpts.make(lod_px=lod_px, counters=1), vb)
    st = pr.pr_get_stats(ctx.handle)
    return out[0], out[1], st


@pytest.mark.parametrize("lod_px,eyes", [(100.0, (0, 1)), (0.0, (0,))])
def test_c6_lod_stereo(ctx, c6, lod_px, eyes):
    import torch
    import paper_2204_01287_amd as pr

    cams = synth.stereo_cameras(synth.C3_SEED)
    o = oracle.opts(lod_px=lod_px)
    refs = {}
    for e in eyes:
        t0 = _t()
        say(f"C6: eye {e} at lod_px {lod_px}: GPU frame, then the oracle")
        vb, fb, st = _lod_frame(ctx, c6.dc, cams[e], lod_px)
        ref, st_ref = oracle_frame(c6.B, cams[e], c6.nb, o)
        say(f"C6: oracle done ({_t() - t0:.1f} s): {st_ref}")
        assert_vb_equal(vb, ref, cams[e].width)
        assert np.array_equal(fb, oracle.resolve(ref, c6.B.colors, CLEAR))
        oracle_stats_match(st, st_ref)
        if lod_px > 0:
            assert st_ref["culled"] > 0
        refs[e] = ref
    if lod_px > 0:
        vbs = [torch.empty(c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]
        need = pr.pr_views_work_bytes(c6.dc.handle, len(cams))
        work = torch.empty(need, dtype=torch.uint8, device="cuda")
        best, _ = pr.pr_autotune(ctx.handle, c6.dc.handle, [(c.view, c.proj, c.width, c.height, vb)
                                                            for c, vb in zip(cams, vbs)],
                                 pr.RenderOpts.make(lod_px=lod_px), work, need, 2)
        say(f"C6: autotuned {best}; plain frames again")
        for e in eyes:
            vb, fb, _ = _lod_frame(ctx, c6.dc, cams[e], lod_px)
            assert_vb_equal(vb, refs[e], cams[e].width)
        pr.pr_set_tuning(ctx.handle)

"""Workgroup shapes, tunings and the autotuner: every tuning renders the oracle's image, bit for bit.

Every compiled shape of the persistent render kernel, with its full tile, half its tile and a 256-pixel tile
bound, and with all or one workgroup per CU, renders C1 and a 2M-point Morton terrain (single view with counters,
and several views in one launch) equal to the oracle.  pr_autotune returns the fastest of its trials, keeps it on
the context and leaves the oracle's image in the views; the batch-size level (autotune.tune) rebuilds the cloud
per batch size.  High-quality shading and LOD layouts under other shapes; the argument checks.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_vb_equal, gpu_build, gpu_render, oracle_stats_match, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2204_01287_amd as pr

    assert torch.cuda.is_available()
    c = pr.Context(0)
    yield c
    pr.pr_set_tuning(c.handle)
    c.close()


@pytest.fixture(scope="module")
def shapes(ctx):
    import paper_2204_01287_amd as pr

    return pr.pr_raster_shapes(ctx.handle)


@pytest.fixture(scope="module")
def c1(ctx):
    xyz, rgba = synth.primitives(synth.C1_SEED, 1_000_000)
    say("autotune: build C1")
    return gpu_build(ctx, xyz, rgba, 10240, False), oracle.build_cloud(xyz, rgba, 10240, morton=False)


@pytest.fixture(scope="module")
def terrain(ctx):
    xyz, rgba = synth.terrain(synth.C2_SEED, 2_000_000, order=1)
    say("autotune: build terrain 2M")
    return gpu_build(ctx, xyz, rgba, 10240, True), oracle.build_cloud(xyz, rgba, 10240, morton=True)


def _views(ctx, dc, cams):
    import torch
    import paper_2204_01287_amd as pr

    vbs = [torch.empty(c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]
    need = pr.pr_views_work_bytes(dc.handle, len(cams))
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    pr.pr_render_views(ctx.handle, dc.handle, [(c.view, c.proj, c.width, c.height, vb) for c, vb in zip(cams, vbs)],
                       None, work, need)
    pr.pr_sync(ctx.handle)
    return [vb.cpu().numpy().view(np.uint64) for vb in vbs]


def test_shapes(shapes):
    assert len(shapes) >= 2
    assert (shapes[0]["waves"], shapes[0]["depth"], shapes[0]["tile_px"]) == (4, 5, 4992)
    assert shapes[0]["max_wg_per_cu"] == 4  # the 4992-pixel tile keeps four workgroups per CU
    assert all(s["max_wg_per_cu"] >= 1 for s in shapes)
    assert len({(s["waves"], s["depth"], s["tile_px"]) for s in shapes}) == len(shapes)


def test_every_tuning_renders_the_oracle_image(ctx, shapes, c1, terrain):
    import paper_2204_01287_amd as pr

    rng = np.random.default_rng(77)
    cases = [(c1, synth.c1_camera()),
             (c1, synth.random_camera(rng, 320, 240, inside=True)),
             (terrain, synth.orbit_camera(5, width=960, height=540))] + \
            [(terrain, c) for c in synth.stereo_cameras(synth.C2_SEED, 504, 560)]
    refs = [oracle.render(B, c.view, c.proj, c.width, c.height) for (_, B), c in cases]
    for i, s in enumerate(shapes):
        for tile, wg, bands in [(t, w, 0) for t in sorted({0, s["tile_px"] // 2, 256}) for w in (0, 1)] + \
                               [(256, 0, 1), (256, 0, 64), (0, 0, 16)]:
            say(f"autotune: shape {i} {s} tile_px={tile} wg_per_cu={wg} max_bands={bands}")
            pr.pr_set_tuning(ctx.handle, shape=i, tile_px=tile, wg_per_cu=wg, max_bands=bands)
            assert pr.pr_get_tuning(ctx.handle) == {"shape": i, "tile_px": tile, "wg_per_cu": wg, "max_bands": bands}
            for ((dc, _), c), (ref, st_ref) in zip(cases, refs):
                vb, fb, st = gpu_render(ctx, dc, c.view, c.proj, c.width, c.height)
                assert_vb_equal(vb, ref, c.width)
                oracle_stats_match(st, st_ref)
        pr.pr_set_tuning(ctx.handle, shape=i)
        cams = [c for (d, _), c in cases if d is terrain[0]]
        for vb, ((_, _), c), (ref, _) in zip(_views(ctx, terrain[0], cams), cases[2:], refs[2:]):
            assert_vb_equal(vb, ref, c.width)
    pr.pr_set_tuning(ctx.handle)


def test_tuning_argument_checks(ctx, shapes):
    import paper_2204_01287_amd as pr

    n = len(shapes)
    bad = [dict(shape=n), dict(shape=0, tile_px=shapes[0]["tile_px"] + 1), dict(shape=0, wg_per_cu=1000),
           dict(shape=0, max_bands=65)]
    pr.pr_set_tuning(ctx.handle, shape=n - 1, tile_px=128, wg_per_cu=1)
    for b in bad:
        with pytest.raises(pr.PrError, match="PR_EINVAL"):
            pr.pr_set_tuning(ctx.handle, **b)
    assert pr.pr_get_tuning(ctx.handle) == {"shape": n - 1, "tile_px": 128, "wg_per_cu": 1, "max_bands": 0}
    assert pr.lib.pr_set_tuning(ctx.handle, None) == 0
    assert pr.pr_get_tuning(ctx.handle) == {"shape": 0, "tile_px": 0, "wg_per_cu": 0, "max_bands": 0}


def test_autotune_keeps_the_fastest_and_the_image(ctx, shapes, terrain):
    import torch
    import paper_2204_01287_amd as pr

    dc, B = terrain
    cams = synth.stereo_cameras(synth.C2_SEED, 504, 560) + [synth.orbit_camera(12, width=640, height=360)]
    vbs = [torch.empty(c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]
    views = [(c.view, c.proj, c.width, c.height, vb) for c, vb in zip(cams, vbs)]
    need = pr.pr_views_work_bytes(dc.handle, len(cams))
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    pr.pr_set_tuning(ctx.handle, shape=1)
    with pytest.raises(pr.PrError, match="PR_EINVAL"):
        pr.pr_autotune(ctx.handle, dc.handle, views, pr.RenderOpts.make(counters=1), work, need)
    assert pr.pr_get_tuning(ctx.handle)["shape"] == 1  # an error leaves the tuning alone
    say("autotune: pr_autotune over 3 views")
    best, trials = pr.pr_autotune(ctx.handle, dc.handle, views, None, work, need, reps=2)
    assert 2 * len(shapes) + 4 <= len(trials) <= 4 * len(shapes) + 4
    assert {t["max_bands"] for t, _ in trials} == {0, 1, 2, 8, 16}
    assert {t["shape"] for t, _ in trials} == set(range(len(shapes)))
    assert all(ms > 0 for _, ms in trials)
    ms = [m for _, m in trials]
    assert best == trials[int(np.argmin(ms))][0]
    assert pr.pr_get_tuning(ctx.handle) == best
    for c, vb in zip(cams, vbs):
        ref, _ = oracle.render(B, c.view, c.proj, c.width, c.height)
        assert_vb_equal(vb.cpu().numpy().view(np.uint64), ref, c.width)
    pr.pr_set_tuning(ctx.handle)


def test_batch_size_sweep(ctx):
    import paper_2204_01287_amd as pr
    from paper_2204_01287_amd.autotune import tune

    xyz, rgba = synth.terrain(5, 1_000_000, order=1)
    cams = synth.camera_array(5, n=6, width=320, height=320)
    built = []

    def build(S):
        say(f"autotune: build S={S}")
        built.append(S)
        return pr.DeviceCloud(ctx, xyz, rgba, batch_size=S, morton=True)

    res = tune(ctx, build, [5120, 10240, 20480], cams, reps=1)
    assert built == [5120, 10240, 20480]
    best = res["best"]
    assert best["batch_size"] in built and best["ms"] == min(t["ms"] for t in res["trials"])
    assert pr.pr_get_tuning(ctx.handle) == best["tuning"]
    S = best["batch_size"]
    dc = build(S)
    B = oracle.build_cloud(xyz, rgba, S, morton=True)
    for c, vb in zip(cams, _views(ctx, dc, cams)):
        ref, _ = oracle.render(B, c.view, c.proj, c.width, c.height)
        assert_vb_equal(vb, ref, c.width)
    dc.close()
    pr.pr_set_tuning(ctx.handle)


def test_hqs_and_lod_under_other_shapes(ctx, shapes, terrain):
    import torch
    import paper_2204_01287_amd as pr

    dc, B = terrain
    cam = synth.stereo_cameras(synth.C2_SEED, 504, 560)[0]
    w, h = cam.width, cam.height
    ref, _ = oracle.render(B, cam.view, cam.proj, w, h)
    racc = oracle.accumulate(B, cam.view, cam.proj, w, h, ref, window=1.01)
    xyz, rgba = synth.terrain(synth.C2_SEED, 1_000_000, order=1)
    xo, ro, spans, nodes = synth.lpc_layout(31, xyz, rgba, synth.lpc_depth(len(xyz), 4096), 4096)
    lc = pr.DeviceCloud(ctx, xo, ro, spans=spans, nodes=nodes)
    LB = oracle.build_cloud_spans(xo, ro, spans, nodes)
    ocam = synth.orbit_camera(3, width=960, height=540)
    lref, _ = oracle.render(LB, ocam.view, ocam.proj, ocam.width, ocam.height, oracle.opts(lod_px=100.0))
    for i, s in enumerate(shapes):
        say(f"autotune: hqs + lod under shape {i} {s}")
        pr.pr_set_tuning(ctx.handle, shape=i, tile_px=s["tile_px"] // 2)
        vb = torch.empty(w * h, dtype=torch.int64, device="cuda")
        acc = torch.empty(2 * w * h, dtype=torch.int64, device="cuda")
        fb = torch.empty(w * h, dtype=torch.int32, device="cuda")
        pr.pr_render_hqs(ctx.handle, dc.handle, cam.view, cam.proj, w, h, None, 1.01, vb, acc, 0, fb)
        pr.pr_sync(ctx.handle)
        assert_vb_equal(vb.cpu().numpy().view(np.uint64), ref, w)
        assert np.array_equal(acc.cpu().numpy().view(np.uint64), racc)
        lvb, _, _ = gpu_render(ctx, lc, ocam.view, ocam.proj, ocam.width, ocam.height, lod_px=100.0, counters=0)
        assert_vb_equal(lvb, lref, ocam.width)
    lc.close()
    pr.pr_set_tuning(ctx.handle)

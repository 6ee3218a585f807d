"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by element.

Bit-exact everywhere: build outputs (positions in render order, colours,
permutation, batch records, low/med/high words), visibility buffers,
framebuffers and the deterministic counters.  The atomics counter depends on
timing and is only reported.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import (MODES, assert_build_equal, assert_vb_equal, gpu_build, gpu_build_outputs, gpu_render,
                      oracle_stats_match, say)

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2204_01287_amd as pr

    assert torch.cuda.is_available()
    c = pr.Context(0)
    yield c
    c.close()


def _both(ctx, xyz, rgba, S, morton):
    say(f"build n={len(xyz)} S={S} morton={morton}")
    dc = gpu_build(ctx, xyz, rgba, S, morton)
    B = oracle.build_cloud(xyz, rgba, S, morton=morton)
    return dc, B


def _check_frame(ctx, dc, B, cam_view, cam_proj, w, h, mode="adaptive", clear_rgba=0, **kw):
    opt = dict(MODES[mode])
    opt.update(kw)
    say(f"render {mode} {w}x{h} n={dc.n} opts={opt}")
    vb, fb, st = gpu_render(ctx, dc, cam_view, cam_proj, w, h, clear_rgba=clear_rgba, **opt)
    o = oracle.opts(precision=opt.get("precision", 0), cull=opt.get("cull", 1), t10=opt.get("t10", 500.0),
                    t20=opt.get("t20", 512000.0))
    ref, st_ref = oracle.render(B, cam_view, cam_proj, w, h, o)
    assert_vb_equal(vb, ref, w)
    assert np.array_equal(fb, oracle.resolve(ref, B.colors, clear_rgba))
    oracle_stats_match(st, st_ref)
    return vb, st


# ------------------------------------------------------------ worked example
def test_worked_example(ctx):
    g = json.load(open(GOLD))
    xyz = np.array(g["points"], np.float32)
    cols = np.array([int(c, 16) for c in g["colors"]], np.uint32)
    dc, B = _both(ctx, xyz, cols, g["batch_size"], False)
    assert_build_equal(gpu_build_outputs(dc), B)
    view, proj = np.array(g["view"], np.float32), np.array(g["proj"], np.float32)
    for cull in (1, 0):
        vb, fb, st = gpu_render(ctx, dc, view, proj, g["width"], g["height"], cull=cull)
        got = {int(p): int(vb[p]) for p in np.nonzero(vb != oracle.EMPTY)[0]}
        assert got == {int(k): int(v, 16) for k, v in g["expected_vb"].items()}
        assert st["culled"] == (2 if cull else 0)


# ------------------------------------------------------------------ config 1
@pytest.fixture(scope="module")
def c1(ctx):
    xyz, rgba = synth.primitives(synth.C1_SEED, 1_000_000)
    return _both(ctx, xyz, rgba, 10240, False)


def test_c1_build(c1):
    dc, B = c1
    assert_build_equal(gpu_build_outputs(dc), B)


@pytest.mark.parametrize("mode", list(MODES))
def test_c1_render(ctx, c1, mode):
    dc, B = c1
    cam = synth.c1_camera()
    _check_frame(ctx, dc, B, cam.view, cam.proj, cam.width, cam.height, mode, clear_rgba=0xFF202020)


def test_c1_random_cameras(ctx, c1):
    dc, B = c1
    rng = np.random.default_rng(7)
    for k in range(6):
        w, h = int(rng.integers(64, 1400)), int(rng.integers(64, 900))
        cam = synth.random_camera(rng, w, h, inside=bool(k % 2))
        _check_frame(ctx, dc, B, cam.view, cam.proj, w, h, "adaptive", t10=float(rng.choice([500.0, 60.0])),
                     t20=float(rng.choice([512000.0, 200.0])))


def test_consecutive_frames_and_determinism(ctx, c1):
    """A frame never sees the previous frame's values, and repeated frames agree."""
    import torch

    dc, B = c1
    cam = synth.c1_camera()
    rng = np.random.default_rng(3)
    other = synth.random_camera(rng, cam.width, cam.height)
    vb = torch.empty(cam.width * cam.height, dtype=torch.int64, device="cuda")
    fb = torch.empty(cam.width * cam.height, dtype=torch.int32, device="cuda")
    say("consecutive frames")
    first, _, _ = gpu_render(ctx, dc, other.view, other.proj, cam.width, cam.height, vb=vb, fb=fb)
    second, _, _ = gpu_render(ctx, dc, cam.view, cam.proj, cam.width, cam.height, vb=vb, fb=fb)
    third, _, _ = gpu_render(ctx, dc, cam.view, cam.proj, cam.width, cam.height, vb=vb, fb=fb)
    ref, _ = oracle.render(B, cam.view, cam.proj, cam.width, cam.height)
    assert_vb_equal(second, ref, cam.width)
    assert np.array_equal(second, third)


# ------------------------------------------------------ tiny random clouds
def _tiny(rng, n):
    kind = rng.integers(4)
    if kind == 0:
        pts = rng.uniform(0, 10, (n, 3))
    elif kind == 1:
        c = rng.uniform(0, 10, (4, 3))
        pts = c[rng.integers(0, 4, n)] + rng.normal(0, 0.3, (n, 3))
    elif kind == 2:
        pts = np.column_stack([rng.uniform(0, 10, n), rng.uniform(0, 10, n), np.full(n, 5.0)])
        pts[rng.integers(0, n, n // 8)] = pts[0]
    else:  # signed zeros and exact grid values
        pts = rng.integers(-4, 5, (n, 3)).astype(np.float64) * 0.5
        pts[rng.random((n, 3)) < 0.2] = -0.0
    return pts.astype(np.float32)


@pytest.mark.parametrize("seed", range(24))
def test_tiny_random_clouds(ctx, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 3000))
    S = int(rng.choice([4, 8, 64, 256, 1024]))
    xyz = _tiny(rng, n)
    rgba = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    dc, B = _both(ctx, xyz, rgba, S, bool(seed % 2))
    assert_build_equal(gpu_build_outputs(dc), B)
    w, h = int(rng.integers(1, 300)), int(rng.integers(1, 300))
    cam = synth.random_camera(rng, w, h, inside=bool(seed % 3 == 0), box=((-2, -2, -2), (10, 10, 10)))
    for mode in ("adaptive", "force10", "force20", "force30", "adaptive_nocull"):
        _check_frame(ctx, dc, B, cam.view, cam.proj, w, h, mode)
    _check_frame(ctx, dc, B, cam.view, cam.proj, w, h, "adaptive", t10=3.0, t20=9.0)


def test_exact_floor_edges(ctx):
    view = np.eye(4, dtype=np.float32)
    proj = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, -2, -3], [0, 0, -1, 0]], np.float32)
    pts = []
    for z in (-1.0, -3.0, -0.75, -1e-3, -2.5e-20):
        for px in range(-3, 12):
            x = np.float32((px / 4.0 - 1.0) * (-z))
            for xx in (x, np.nextafter(x, np.float32(-np.inf)), np.nextafter(x, np.float32(np.inf))):
                for yy in (np.float32(0.3 * -z), np.float32((2 / 4.0 - 1.0) * (-z))):
                    pts.append([xx, yy, z])
    xyz = np.array(pts, np.float32)
    rgba = np.arange(len(pts), dtype=np.uint32)
    for S in (4, 12):
        dc, B = _both(ctx, xyz, rgba, S, False)
        for mode in ("force10", "force20", "force30", "adaptive"):
            _check_frame(ctx, dc, B, view, proj, 8, 8, mode)


def test_camera_inside_and_behind(ctx):
    """Boxes that reach w <= 0 and points near the eye plane (the exact binary64 floor path)."""
    xyz, rgba = synth.terrain(11, 300_000, order=0)
    dc, B = _both(ctx, xyz, rgba, 1024, True)
    rng = np.random.default_rng(4)
    for k in range(4):
        eye = np.array([rng.uniform(100, 900), rng.uniform(100, 900), synth.terrain_height(11, 500, 500) + 2.0])
        tgt = eye + np.array([np.cos(k), np.sin(k), -0.2])
        cam = synth.camera(eye, tgt, (0, 0, 1), 90.0, 640, 480, 1e-3, 5000.0)
        _check_frame(ctx, dc, B, cam.view, cam.proj, 640, 480, "adaptive")
        _check_frame(ctx, dc, B, cam.view, cam.proj, 640, 480, "adaptive_nocull")


# ------------------------------------------------- terrain, Morton order
@pytest.fixture(scope="module")
def terrain_small(ctx):
    xyz, rgba = synth.terrain(synth.C2_SEED, 2_000_000, order=1)
    return _both(ctx, xyz, rgba, 10240, True)


def test_terrain_morton_build(terrain_small):
    dc, B = terrain_small
    assert_build_equal(gpu_build_outputs(dc), B)


@pytest.mark.parametrize("frame", [0, 13, 29, 44])
def test_terrain_orbit(ctx, terrain_small, frame):
    dc, B = terrain_small
    cam = synth.orbit_camera(frame)
    _check_frame(ctx, dc, B, cam.view, cam.proj, cam.width, cam.height, "adaptive")
    _check_frame(ctx, dc, B, cam.view, cam.proj, cam.width, cam.height, "force30")


def test_terrain_stereo_pair(ctx, terrain_small):
    dc, B = terrain_small
    for cam in synth.stereo_cameras(synth.C2_SEED, 504, 560):
        _check_frame(ctx, dc, B, cam.view, cam.proj, cam.width, cam.height, "adaptive")


@pytest.fixture(scope="module")
def terrain_spread(ctx):
    xyz, rgba = synth.terrain(synth.C2_SEED, 2_000_000, order=1)
    return _both(ctx, xyz, rgba, 10240, 2)


def test_terrain_spread_build_and_frames(ctx, terrain_spread):
    """The spread order (each Morton batch stored with a golden-ratio stride over its ranks): build outputs, orbit
    frames in both precision modes and the stereo pair equal the oracle's spread build."""
    dc, B = terrain_spread
    assert_build_equal(gpu_build_outputs(dc), B)
    for frame in (0, 29):
        cam = synth.orbit_camera(frame)
        _check_frame(ctx, dc, B, cam.view, cam.proj, cam.width, cam.height, "adaptive")
        _check_frame(ctx, dc, B, cam.view, cam.proj, cam.width, cam.height, "force30")
    for cam in synth.stereo_cameras(synth.C2_SEED, 504, 560):
        _check_frame(ctx, dc, B, cam.view, cam.proj, cam.width, cam.height, "adaptive")


def test_unknown_order_is_refused(ctx):
    import paper_2204_01287_amd as pr

    xyz, rgba = synth.primitives(5, 1000)
    with pytest.raises(pr.PrError) as e:
        gpu_build(ctx, xyz, rgba, 64, 3)
    assert e.value.name == "PR_EINVAL"


# ----------------------------------------------------------------- edges
@pytest.mark.parametrize("n,S", [(0, 64), (1, 4), (5, 4), (10241, 10240), (20480, 10240), (1003, 64), (50003, 1000),
                                 (600001, 262144)])
def test_ragged_and_empty(ctx, n, S):
    xyz, rgba = synth.primitives(5, max(n, 1))
    xyz, rgba = xyz[:n], rgba[:n]
    # odd n: Morton order, and every third case of those in the spread order (ragged last batches included)
    order = (2 if n % 3 == 2 else 1) if n % 2 == 1 else 0
    dc, B = _both(ctx, xyz, rgba, S, order)
    if n:
        assert_build_equal(gpu_build_outputs(dc), B)
    cam = synth.c1_camera()
    _check_frame(ctx, dc, B, cam.view, cam.proj, 320, 180, "adaptive")
    _check_frame(ctx, dc, B, cam.view, cam.proj, 1, 1, "force30")


def test_maximum_image_size(ctx, c1):
    dc, B = c1
    cam = synth.c1_camera()
    _check_frame(ctx, dc, B, cam.view, cam.proj, 8192, 8192, "adaptive")


@pytest.mark.parametrize("morton", [False, True])
def test_non_finite_inputs(ctx, morton):
    """A NaN or infinite coordinate fails the build (with the Morton order the check runs on the cloud box's
    loads); a bad view matrix or an empty image fails the render."""
    import paper_2204_01287_amd as pr

    xyz, rgba = synth.primitives(6, 5000)
    for bad_value, at in ((np.nan, (4321, 2)), (np.inf, (17, 0)), (-np.inf, (4999, 1))):
        xyz_bad = xyz.copy()
        xyz_bad[at] = bad_value
        with pytest.raises(pr.PrError) as e:
            gpu_build(ctx, xyz_bad, rgba, 64, morton)
        assert e.value.name == "PR_ENONFINITE"
    dc = gpu_build(ctx, xyz, rgba, 64, morton)
    cam = synth.c1_camera()
    bad = cam.view.copy()
    bad[1, 2] = np.inf
    import torch

    vb = torch.empty(64, dtype=torch.int64, device="cuda")
    with pytest.raises(pr.PrError) as e:
        pr.pr_render(ctx.handle, dc.handle, bad, cam.proj, 8, 8, None, vb)
    assert e.value.name == "PR_ENONFINITE"
    with pytest.raises(pr.PrError) as e:
        pr.pr_render(ctx.handle, dc.handle, cam.view, cam.proj, 0, 8, None, vb)
    assert e.value.name == "PR_ERANGE"


def test_clear_and_accumulate(ctx, c1):
    """pr_clear + accumulate render == plain render; two views accumulate to the elementwise minimum."""
    import torch
    import paper_2204_01287_amd as pr

    dc, B = c1
    cam = synth.c1_camera()
    other = synth.random_camera(np.random.default_rng(12), cam.width, cam.height)
    w, h = cam.width, cam.height
    vb = torch.empty(w * h, dtype=torch.int64, device="cuda")
    say("clear + accumulate")
    pr.pr_clear(ctx.handle, vb, w, h)
    acc = pr.RenderOpts.make(accumulate=1)
    pr.pr_render(ctx.handle, dc.handle, cam.view, cam.proj, w, h, acc, vb)
    pr.pr_sync(ctx.handle)
    one = vb.cpu().numpy().view(np.uint64).copy()
    ref_a, _ = oracle.render(B, cam.view, cam.proj, w, h)
    assert_vb_equal(one, ref_a, w)
    pr.pr_render(ctx.handle, dc.handle, other.view, other.proj, w, h, acc, vb)
    pr.pr_sync(ctx.handle)
    ref_b, _ = oracle.render(B, other.view, other.proj, w, h)
    assert_vb_equal(vb.cpu().numpy().view(np.uint64), np.minimum(ref_a, ref_b), w)


def test_kernel_timing_events(ctx, c1):
    """pr_time_kernels: the armed render launches (plain and multi-view) each time their kernel, the frames stay
    bit-equal to the oracle, later launches are not recorded, 0 disarms, and too many launches are refused."""
    import torch
    import paper_2204_01287_amd as pr

    dc, B = c1
    cam = synth.c1_camera()
    other = synth.random_camera(np.random.default_rng(21), cam.width, cam.height)
    w, h = cam.width, cam.height
    ref_a, _ = oracle.render(B, cam.view, cam.proj, w, h)
    ref_b, _ = oracle.render(B, other.view, other.proj, w, h)
    vb = torch.empty(w * h, dtype=torch.int64, device="cuda")
    vb2 = torch.empty(w * h, dtype=torch.int64, device="cuda")
    say("kernel timing: 3 armed launches, 4 made")
    pr.pr_time_kernels(ctx.handle, 3)
    assert pr.pr_kernel_times(ctx.handle) == []
    pr.pr_render(ctx.handle, dc.handle, cam.view, cam.proj, w, h, None, vb)
    need = pr.pr_views_work_bytes(dc.handle, 2)
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    views = [(cam.view, cam.proj, w, h, vb), (other.view, other.proj, w, h, vb2)]
    pr.pr_render_views(ctx.handle, dc.handle, views, None, work, need)
    pr.pr_render(ctx.handle, dc.handle, other.view, other.proj, w, h, None, vb2)
    pr.pr_render(ctx.handle, dc.handle, cam.view, cam.proj, w, h, None, vb)
    t = pr.pr_kernel_times(ctx.handle)
    assert len(t) == 3 and all(0.0 < x < 1000.0 for x in t), t
    assert pr.pr_kernel_times(ctx.handle, 2) == t[:2]
    assert_vb_equal(vb.cpu().numpy().view(np.uint64), ref_a, w)
    assert_vb_equal(vb2.cpu().numpy().view(np.uint64), ref_b, w)
    pr.pr_time_kernels(ctx.handle, 0)
    pr.pr_render(ctx.handle, dc.handle, cam.view, cam.proj, w, h, None, vb)
    assert pr.pr_kernel_times(ctx.handle) == []
    with pytest.raises(pr.PrError) as e:
        pr.pr_time_kernels(ctx.handle, pr.PR_MAX_TIMED_LAUNCHES + 1)
    assert e.value.name == "PR_EINVAL"
    pr.pr_sync(ctx.handle)

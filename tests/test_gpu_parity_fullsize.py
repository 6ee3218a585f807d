"""Parity at the full workload sizes, in the launch configuration that bench.py times.

Every GPU frame here is bench.py's: pr_render with default options (its classify launch also clears the
visibility buffer), then pr_resolve with the clear colour 0xFF000000, on the context's stream, with the persistent
render grid of pr_create.

C2 -- 100,000,000-point terrain (serpentine generation order, Morton build), orbit frames 0/15/30/45 at 1920x1080.
The oracle builds and renders the same cloud.  The whole build (positions in render order, colours, permutation,
batch records, low/med/high words), every visibility buffer, every framebuffer and the frame counters are compared
element by element.

C3 -- 2,000,000,000-point terrain (index generation order, Morton build), stereo pair 2 x 2016 x 2240, one launch
per eye and both eyes in one multi-view launch (pr_render_views).  The oracle
cannot sort 2e9 points in test time, so the device's Morton permutation is checked by the two properties that make
it unique:
  * it is a permutation of 0..n-1;
  * the oracle's Morton codes of the generator's points taken in that order (over the oracle's box of the
    generator's cloud) are non-decreasing, with equal codes in increasing input index.
A stable sort by code is the only order with both.  Everything else compared is the oracle's, computed from the
generator's points in that order: batch table, Eq. 1 words, colours, per-batch decisions and frame counters, and
the complete visibility buffer and framebuffer of each eye.  The oracle renders interleaved batch sets on worker
threads into private buffers that are merged by elementwise minimum; the minimum is associative and commutative,
so the merge is exact.
"""
from __future__ import annotations

import types
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from fullsize_util import CH, CLEAR, RENDER_WORKERS, S, _t, _u32, check_morton_build, device_views, oracle_frame
from gpu_util import assert_vb_equal, oracle_stats_match, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2204_01287_amd as pr

    assert torch.cuda.is_available()
    c = pr.Context(0)
    yield c
    c.close()


def _bench_frame(ctx, handle, cam, precision=0):
    """One eye exactly as bench.py times it; returns host copies of VB and FB and the frame counters."""
    import torch
    import paper_2204_01287_amd as pr

    dev = torch.device("cuda", 0)
    vb = torch.empty(cam.width * cam.height, dtype=torch.int64, device=dev)
    fb = torch.empty(cam.width * cam.height, dtype=torch.int32, device=dev)
    vb.fill_(7)  # stale contents: the frame must clear them
    o = pr.RenderOpts.make(precision=precision) if precision else None
    pr.pr_render(ctx.handle, handle, cam.view, cam.proj, cam.width, cam.height, o, vb)
    pr.pr_resolve(ctx.handle, handle, vb, cam.width, cam.height, CLEAR, fb)
    pr.pr_sync(ctx.handle)
    out_vb, out_fb = vb.cpu().numpy().view(np.uint64), fb.cpu().numpy().view(np.uint32)
    # the counters frame (bench.py's untimed first frame)
    pr.pr_render(ctx.handle, handle, cam.view, cam.proj, cam.width, cam.height,
                 pr.RenderOpts.make(precision=precision, counters=1), vb)
    st = pr.pr_get_stats(ctx.handle)
    assert np.array_equal(vb.cpu().numpy().view(np.uint64), out_vb), "counters frame differs from the timed frame"
    return out_vb, out_fb, st


def _check_eye(ctx, handle, built, colors, cam, nb, tag, precision=0):
    t0 = _t()
    say(f"{tag}: bench frame on the GPU ({cam.width}x{cam.height}, precision {precision or 'adaptive'})")
    vb, fb, st = _bench_frame(ctx, handle, cam, precision)
    say(f"{tag}: GPU frame done ({_t() - t0:.1f} s); oracle render of {nb} batches on {RENDER_WORKERS} threads")
    ref, st_ref = oracle_frame(built, cam, nb, oracle.opts(precision=precision))
    say(f"{tag}: oracle done ({_t() - t0:.1f} s): {st_ref}")
    assert_vb_equal(vb, ref, cam.width)
    assert np.array_equal(fb, oracle.resolve(ref, colors, CLEAR)), "framebuffer differs"
    oracle_stats_match(st, st_ref)
    assert st["points"] > 0 and np.count_nonzero(ref != oracle.EMPTY) > 0


# =================================================================== C2: 1e8
@pytest.fixture(scope="module")
def c2(ctx):
    import torch
    import bench

    wl = bench.workload("c2", None)
    seen = {}

    def keep(lo, hi, xyz, rgba):
        seen["xyz"], seen["rgba"] = xyz, rgba

    say(f"C2: generate and build {wl['n']} points on the GPU")
    cloud = bench.load_cloud(ctx, wl, on_chunk=keep)
    t0 = _t()
    say("C2: oracle build (Morton sort, batches, Eq. 1) of the same points")
    B = oracle.build_cloud(seen["xyz"], seen["rgba"], S, morton=wl["morton"])
    say(f"C2: oracle build done ({_t() - t0:.1f} s)")
    yield types.SimpleNamespace(wl=wl, cloud=cloud, B=B, n=wl["n"], nb=cloud["nb"])
    import paper_2204_01287_amd as pr

    pr.pr_cloud_free(cloud["handle"])
    cloud.clear()
    torch.cuda.empty_cache()


def test_c2_build_full(c2):
    n, nb, B = c2.n, c2.nb, c2.B
    assert nb == B.batches.shape[0]
    v = device_views(c2.cloud, n, nb)
    say("C2: compare every build output with the oracle")
    for f in ("perm", "colors", "low", "med", "high"):
        a = _u32(getattr(v, f))
        b = getattr(B, f)
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{f}: {len(bad)} mismatches, first at {bad[:5]}")
    assert np.array_equal(_u32(v.xyz), B.xyz.view(np.uint32).reshape(-1)), "positions in render order differ"
    assert np.array_equal(v.batches.cpu().numpy(), B.batches.view(np.uint8)), "batch records differ"


@pytest.mark.parametrize("frame", [0, 1, 2, 3])
def test_c2_orbit_frame(ctx, c2, frame):
    cam = c2.wl["cams"][frame]
    _check_eye(ctx, c2.cloud["handle"], c2.B, c2.B.colors, cam, c2.nb, f"C2 orbit view {frame}")


def test_c2_force30_frames(ctx, c2):
    """Fixed 12-byte loads (PR_FORCE30, Sec. 3.3's comparison), as bench.py's c2 leg renders them."""
    import synth

    for f in (0, 30):
        cam = synth.orbit_camera(f)
        _check_eye(ctx, c2.cloud["handle"], c2.B, c2.B.colors, cam, c2.nb, f"C2 orbit {f} FORCE30", precision=30)


@pytest.fixture(scope="module", params=[1, 0], ids=["generation", "index"])
def c2_generation(ctx, request):
    """The 1e8 points batched without a Morton sort, as bench.py's c2 leg builds them: in the generator's tile
    order (10 m tiles in serpentine strips) and in its index order (spatially incoherent)."""
    import torch
    import bench

    wl = dict(bench.workload("c2", None), morton=False, order=request.param, name=f"terrain_1e8_order{request.param}")
    n = wl["n"]
    xyz_all, rgba_all = np.empty((n, 3), np.float32), np.empty(n, np.uint32)

    def keep(lo, hi, xyz, rgba):  # the loader reuses its chunk buffers: copy
        xyz_all[lo:hi] = xyz
        rgba_all[lo:hi] = rgba

    say(f"C2 generator order {request.param}, no Morton sort: build on the GPU")
    cloud = bench.load_cloud(ctx, wl, on_chunk=keep)
    B = oracle.build_cloud(xyz_all, rgba_all, S, morton=False)
    del xyz_all, rgba_all
    yield types.SimpleNamespace(wl=wl, cloud=cloud, B=B, n=wl["n"], nb=cloud["nb"])
    import paper_2204_01287_amd as pr

    pr.pr_cloud_free(cloud["handle"])
    cloud.clear()
    torch.cuda.empty_cache()


def test_c2_generation_order(ctx, c2_generation):
    import synth

    g = c2_generation
    v = device_views(g.cloud, g.n, g.nb)
    for f in ("colors", "low", "med", "high"):
        assert np.array_equal(_u32(getattr(v, f)), getattr(g.B, f)), f"{f} differs"
    assert np.array_equal(v.batches.cpu().numpy(), g.B.batches.view(np.uint8)), "batch records differ"
    for f in (0, 45):
        _check_eye(ctx, g.cloud["handle"], g.B, g.B.colors, synth.orbit_camera(f), g.nb,
                   f"C2 order {g.wl['order']} frame {f}")


# =================================================================== C3: 2e9
@pytest.fixture(scope="module")
def c3(ctx):
    import torch
    import bench

    wl = bench.workload("c3", None)
    boxes = []
    pool = ThreadPoolExecutor(2)

    def box(lo, hi, xyz, rgba):
        f = pool.submit(oracle.cloud_aabb, xyz)
        boxes.append(f)
        return f

    say(f"C3: generate and build {wl['n']} points on the GPU")
    cloud = bench.load_cloud(ctx, wl, on_chunk=box)
    pool.shutdown()
    corners = np.array([c for f in boxes for c in f.result()], np.float32)
    ns = types.SimpleNamespace(wl=wl, cloud=cloud, n=wl["n"], nb=cloud["nb"], cloud_box=oracle.cloud_aabb(corners))
    ns.res, ns.built, ns.colors = check_morton_build(ns, "C3")
    yield ns
    import paper_2204_01287_amd as pr

    pr.pr_cloud_free(cloud["handle"])
    cloud.clear()
    torch.cuda.empty_cache()


def test_c3_build_full(c3):
    res = sorted(c3.res, key=lambda r: r["lo"])
    assert sum(1 for _ in range(0, c3.n, CH)) == len(res)
    for r in res:
        for k in ("mono", "stable", "xyz", "colors", "low", "med", "high", "batches"):
            assert r[k], f"chunk at {r['lo']}: {k} check failed"
    for a, b in zip(res, res[1:]):  # across chunk seams
        assert a["tail"][0] <= b["head"][0], f"Morton order broken at {b['lo']}"
        if a["tail"][0] == b["head"][0]:
            assert a["tail"][1] < b["head"][1], f"stability broken at {b['lo']}"


@pytest.mark.parametrize("eye", [0, 1])
def test_c3_stereo_eye(ctx, c3, eye):
    cam = c3.wl["cams"][eye]
    _check_eye(ctx, c3.cloud["handle"], c3.built, c3.colors, cam, c3.nb, f"C3 eye {eye}")


def test_c3_stereo_one_launch(ctx, c3):
    """Both eyes through pr_render_views (one persistent launch) equal the oracle's single-eye renders."""
    import torch
    import paper_2204_01287_amd as pr

    cams = c3.wl["cams"]
    vbs = [torch.empty(c.width * c.height, dtype=torch.int64, device="cuda") for c in cams]
    need = pr.pr_views_work_bytes(c3.cloud["handle"], len(cams))
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    say("C3: both eyes in one multi-view launch")
    pr.pr_render_views(ctx.handle, c3.cloud["handle"], [(c.view, c.proj, c.width, c.height, vb) for c, vb in
                                                         zip(cams, vbs)], pr.RenderOpts.make(counters=1), work, need)
    st = pr.pr_get_stats(ctx.handle)
    pr.pr_sync(ctx.handle)
    tot = None
    for c, vb in zip(cams, vbs):
        ref, s = oracle_frame(c3.built, c, c3.nb)
        assert_vb_equal(vb.cpu().numpy().view(np.uint64), ref, c.width)
        tot = s if tot is None else {k: (tot[k] + s[k] if not isinstance(s[k], list) else
                                         [a + b for a, b in zip(tot[k], s[k])]) for k in s}
    oracle_stats_match(st, tot)


@pytest.mark.parametrize("eye", [0, 1])
def test_c3_hqs(ctx, c3, eye):
    """High-quality shading of each eye, as bench.py's shading leg renders them: visibility buffer, sums and
    averaged framebuffer equal the oracle's (threads over interleaved batch sets, private sums added modulo 2^64,
    exact)."""
    import torch
    import paper_2204_01287_amd as pr

    cam = c3.wl["cams"][eye]
    w, h = cam.width, cam.height
    vb = torch.empty(w * h, dtype=torch.int64, device="cuda")
    acc = torch.empty(2 * w * h, dtype=torch.int64, device="cuda")
    fb = torch.empty(w * h, dtype=torch.int32, device="cuda")
    acc.fill_(5)  # stale sums: the frame must clear them
    say(f"C3: high-quality shading of eye {eye}")
    pr.pr_render_hqs(ctx.handle, c3.cloud["handle"], cam.view, cam.proj, w, h, None, 1.01, vb, acc, CLEAR, fb)
    pr.pr_sync(ctx.handle)
    ref, _ = oracle_frame(c3.built, cam, c3.nb)
    assert_vb_equal(vb.cpu().numpy().view(np.uint64), ref, w)
    groups = [np.arange(g, c3.nb, 4 * RENDER_WORKERS, dtype=np.uint64) for g in range(4 * RENDER_WORKERS)]

    def job(ids):
        return oracle.accumulate(c3.built, cam.view, cam.proj, w, h, ref, window=1.01, batch_ids=ids,
                                 colors=c3.colors)

    racc = np.zeros(2 * w * h, np.uint64)
    with ThreadPoolExecutor(RENDER_WORKERS) as ex:
        for part in ex.map(job, groups):
            racc += part
    assert np.count_nonzero(racc) > 0
    assert np.array_equal(acc.cpu().numpy().view(np.uint64), racc)
    assert np.array_equal(fb.cpu().numpy().view(np.uint32), oracle.resolve_hqs(racc, CLEAR))

"""The seeded generators: deterministic per (seed, index), independent of threading."""
import numpy as np
import pytest

import synth


def test_primitives_deterministic_and_thread_independent():
    a = synth.primitives(1, 50_000, threads=1)
    b = synth.primitives(1, 50_000, threads=7)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    c = synth.primitives(2, 50_000)
    assert not np.array_equal(a[0], c[0])
    assert np.isfinite(a[0]).all()
    assert (a[0] > -1).all() and (a[0] < 101).all()


def test_terrain_prefix_property_in_index_order():
    """Index order: point i depends only on (seed, i, n's category split)."""
    a = synth.terrain(3, 100_000, order=0, threads=2)
    b = synth.terrain(3, 100_000, order=0, threads=5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_terrain_tile_order_is_a_stable_serpentine_bucketing():
    xyz0, c0 = synth.terrain(4, 200_000, order=0)
    xyz1, c1 = synth.terrain(4, 200_000, order=1, threads=3)
    tx = np.clip(np.floor(xyz0[:, 0] / 10.0), 0, 99).astype(np.int64)
    ty = np.clip(np.floor(xyz0[:, 1] / 10.0), 0, 99).astype(np.int64)
    tile = ty * 100 + np.where(ty % 2 == 1, 99 - tx, tx)
    order = np.argsort(tile, kind="stable")
    assert np.array_equal(xyz1, xyz0[order]) and np.array_equal(c1, c0[order])


def test_terrain_category_mix():
    xyz, _ = synth.terrain(5, 100_000, order=0)
    assert np.isfinite(xyz).all()
    assert xyz[:, 0].min() > -1 and xyz[:, 0].max() < 1001
    # ground is 80 %: its z follows the height field (noise 1 cm)
    g = xyz[:80_000:997]
    h = np.array([synth.terrain_height(5, float(x), float(y)) for x, y, _ in g])
    assert np.abs(g[:, 2] - h).max() < 0.1


def test_terrain_range_matches_whole_cloud():
    n = 123_457
    xyz, rgba = synth.terrain(6, n, order=0)
    for lo, hi in ((0, 1000), (5000, 70001), (n - 17, n)):
        x = np.empty((hi - lo, 3), np.float32)
        c = np.empty(hi - lo, np.uint32)
        synth.terrain_range(6, n, lo, hi, x.ctypes.data, c.ctypes.data, threads=3)
        assert np.array_equal(x, xyz[lo:hi]) and np.array_equal(c, rgba[lo:hi])


def test_terrain_gather_matches_whole_cloud():
    n = 123_457
    xyz, rgba = synth.terrain(6, n, order=0)
    idx = np.random.default_rng(0).integers(0, n, 5000).astype(np.uint32)
    idx[:3] = (0, n - 1, 0)
    for t in (1, 5):
        x, c = synth.terrain_gather(6, n, idx, threads=t)
        assert np.array_equal(x, xyz[idx]) and np.array_equal(c, rgba[idx])
    with pytest.raises(RuntimeError):
        synth.terrain_gather(6, n, np.array([n], np.uint32))


def test_request_stream_is_seeded_and_poisson():
    a = synth.request_stream(3, 400, 500.0, [1, 2, 3])
    b = synth.request_stream(3, 400, 500.0, [1, 2, 3])
    assert [(x, c, cam.width) for x, c, cam in a] == [(x, c, cam.width) for x, c, cam in b]
    assert all(np.array_equal(p[2].view, q[2].view) for p, q in zip(a, b))
    t = np.array([x for x, _, _ in a])
    assert np.all(np.diff(t) > 0) and 0.6 < t[-1] < 1.0  # 400 arrivals at 500/s take about 0.8 s
    assert {cam.width for _, _, cam in a} == {640, 1920, 3840} and {c for _, c, _ in a} == {0, 1, 2}


def test_lpc_layout_properties():
    xyz, rgba = synth.terrain(7, 200_000, order=1)
    cap = 2048
    depth = synth.lpc_depth(len(xyz), cap)
    xo, ro, spans, nodes = synth.lpc_layout(3, xyz, rgba, depth, cap)
    again = synth.lpc_layout(3, xyz, rgba, depth, cap)
    assert all(np.array_equal(a, b) for a, b in zip((xo, ro, spans, nodes), again))
    first, count = spans[:, 0].astype(np.int64), spans[:, 1].astype(np.int64)
    assert np.all(first % 4 == 0) and np.all(count >= 1) and np.all(count <= cap)
    assert np.all(first[1:] >= first[:-1] + count[:-1])  # ordered, disjoint
    idx = np.concatenate([np.arange(f, f + c) for f, c in zip(first, count)])
    # every input point exactly once
    a = np.rec.fromarrays([xyz[:, 0], xyz[:, 1], xyz[:, 2], rgba])
    b = np.rec.fromarrays([xo[idx, 0], xo[idx, 1], xo[idx, 2], ro[idx]])
    assert np.array_equal(np.sort(a), np.sort(b))
    pad = np.setdiff1d(np.arange(len(xo)), idx)
    assert np.all(xo[pad] == 0) and np.all(ro[pad] == 0)
    # batches lie in their node's cube (up to one ulp of the grid), levels deepen in order
    for (f, c), nd in zip(spans[::7], nodes[::7]):
        p = xo[f:f + c].astype(np.float64)
        tol = 1e-6 * nd[3] + 1e-6
        assert np.all(p >= nd[:3] - tol) and np.all(p <= nd[:3] + nd[3] + tol)
    assert np.all(np.diff(nodes[:, 4]) >= 0) and nodes[0, 4] == 0
    pts = np.bincount(nodes[:, 4].astype(int), weights=count)
    assert np.all(pts[1:-1] / pts[:-2] > 3.0) and np.all(pts[1:-1] / pts[:-2] < 5.0)  # about 4x per level


def test_lpc_layout_spread_order_permutes_inside_batches():
    """The layout's default stores each batch in the spread order: the same spans and nodes as the plain (level,
    Morton) order, and inside a batch of c points slot t holds the plain order's point t * m mod c, for one step m
    coprime with c just above c / 4."""
    import math

    xyz, rgba = synth.terrain(7, 100_000, order=1)
    cap = 1024
    depth = synth.lpc_depth(len(xyz), cap)
    xs, rs, spans, nodes = synth.lpc_layout(3, xyz, rgba, depth, cap)
    xp, rp, spans_p, nodes_p = synth.lpc_layout(3, xyz, rgba, depth, cap, spread=False)
    assert np.array_equal(spans, spans_p) and np.array_equal(nodes, nodes_p)
    for f, c in spans[::5]:
        f, c = int(f), int(c)
        if c == 1:
            assert np.array_equal(xs[f], xp[f])
            continue
        m = next(k for k in range(c // 4 + 1, c + c // 4 + 2) if math.gcd(k, c) == 1)
        t = np.arange(c)
        assert np.array_equal(xs[f:f + c], xp[f + (t * m) % c]) and np.array_equal(rs[f:f + c], rp[f + (t * m) % c])


def test_stereo_eyes_share_the_y_and_w_rows():
    """The stereo pairs' eyes differ by a shift along the camera's x axis, so the pixel-space y and w rows of their
    frame matrices (and of every batch's folded matrix) are bit-equal: the two-view pass of the renderer then
    computes those chains once.  The x rows differ."""
    import oracle

    for seed, w, h in ((synth.C3_SEED, 2016, 2240), (synth.C2_SEED, 504, 560)):
        a, b = synth.stereo_cameras(seed, w, h)
        pa, pb = oracle.frame_matrix(a.view, a.proj, w, h), oracle.frame_matrix(b.view, b.proj, w, h)
        assert pa[1:].tobytes() == pb[1:].tobytes()
        assert not np.array_equal(pa[0], pb[0])

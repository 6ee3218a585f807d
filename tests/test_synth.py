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

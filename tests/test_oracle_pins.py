"""Pins for the CPU oracle against things other than itself.

- the hand-derived worked example in tests/golden/worked_example.json;
- an exact-rational, pixel-major brute force (tests/exact_ref.py) on tiny clouds;
- closed forms of Eq. 1 and the decode error bound;
- the textbook OpenGL pipeline in float64 (orientation, viewport, depth);
- Morton order against an independent comparator (Chan's most-significant-bit
  rule) and against Python's stable sort;
- invariants: culling never changes the image, culled batches draw nothing,
  batch order and subsets compose by minimum, resolve is index -> colour.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import exact_ref
import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def _gold():
    with open(GOLD) as f:
        return json.load(f)


def _hex(s):
    return int(s, 16)


# ------------------------------------------------------------ worked example
def test_worked_example_build():
    g = _gold()
    xyz = np.array(g["points"], np.float32)
    cols = np.array([_hex(c) for c in g["colors"]], np.uint32)
    B = oracle.build_cloud(xyz, cols, g["batch_size"], morton=False)
    assert [hex(v) for v in B.low[:8]] == [hex(_hex(v)) for v in g["expected_batch0_low"]]
    assert [hex(v) for v in B.med[:8]] == [hex(_hex(v)) for v in g["expected_batch0_med"]]
    assert [hex(v) for v in B.high[:8]] == [hex(_hex(v)) for v in g["expected_batch0_high"]]
    assert B.batches["first"].tolist() == [0, 8, 16]
    assert B.batches["count"].tolist() == [8, 8, 8]
    assert B.batches["min"][0].tolist() == [-2, -2, -6]
    assert B.batches["max"][0].tolist() == [2, 2, -2]


@pytest.mark.parametrize("cull", [1, 0])
def test_worked_example_render(cull):
    g = _gold()
    xyz = np.array(g["points"], np.float32)
    cols = np.array([_hex(c) for c in g["colors"]], np.uint32)
    B = oracle.build_cloud(xyz, cols, g["batch_size"], morton=False)
    view = np.array(g["view"], np.float32)
    proj = np.array(g["proj"], np.float32)
    w, h = g["width"], g["height"]
    o = oracle.opts(cull=cull)
    dec = oracle.decide_all(B.batches, view, proj, w, h, o)
    assert dec["level"].tolist() == g["expected_levels"]
    if cull:
        assert [bool(c) for c in dec["culled"]] == g["expected_culled"]
    else:
        assert not dec["culled"].any()
    vb, st = oracle.render(B, view, proj, w, h, o)
    expect = {int(k): _hex(v) for k, v in g["expected_vb"].items()}
    got = {int(p): int(vb[p]) for p in np.nonzero(vb != oracle.EMPTY)[0]}
    assert got == expect
    assert st["batches"] == 3
    assert st["culled"] == (2 if cull else 0)
    assert st["points"] == (8 if cull else 24)
    fb = oracle.resolve(vb, B.colors, _hex(g["clear_rgba"]))
    for p in range(w * h):
        want = _hex(g["expected_fb"][str(p)]) if str(p) in g["expected_fb"] else _hex(g["clear_rgba"])
        assert int(fb[p]) == want


def test_worked_example_exact_reference():
    g = _gold()
    pts = [[float(v) for v in p] for p in g["points"]]
    got, levels = exact_ref.brute_force(pts, g["batch_size"], g["view"], g["proj"], g["width"], g["height"])
    assert levels == g["expected_levels"]
    assert got == {int(k): _hex(v) for k, v in g["expected_vb"].items()}


# ------------------------------------------------------------------- Eq. 1
def test_eq1_closed_forms():
    assert oracle.eq1(-2.0, -2.0, 2.0) == 0
    assert oracle.eq1(2.0, -2.0, 2.0) == 2 ** 30 - 1  # x = max clamps
    assert oracle.eq1(0.0, -2.0, 2.0) == 2 ** 29  # midpoint
    assert oracle.eq1(-1.0, -2.0, 2.0) == 2 ** 28
    assert oracle.eq1(5.0, 5.0, 5.0) == 0  # empty extent
    assert oracle.eq1(1.0, 0.0, 3.0) == (2 ** 30) // 3  # floor(2^30 / 3)
    assert oracle.eq1(2.0, 0.0, 3.0) == (2 ** 31) // 3


def test_eq1_matches_exact_rationals():
    rng = np.random.default_rng(11)
    lo = rng.uniform(-1000, 1000, 4000).astype(np.float32)
    ext = (10.0 ** rng.uniform(-3, 3, 4000)).astype(np.float32)
    hi = (lo + ext).astype(np.float32)
    t = rng.uniform(0, 1, 4000)
    x = np.clip((lo + t * (hi - lo)).astype(np.float32), lo, hi)
    diff = 0
    for a, b, c in zip(x, lo, hi):
        e = exact_ref.eq1_exact(float(a), float(b), float(c))
        o = oracle.eq1(float(a), float(b), float(c))
        assert abs(e - o) <= 1
        diff += e != o
    assert diff <= 2  # binary64 rounds onto an integer only in rare cases


def test_split_recombines_and_pads():
    xyz, rgba = synth.terrain(5, 40000, order=0)
    B = oracle.build_cloud(xyz, rgba, 1024, morton=True)
    for a in range(3):
        lo = (B.low >> (10 * a)) & 1023
        md = (B.med >> (10 * a)) & 1023
        hi = (B.high >> (10 * a)) & 1023
        X30 = (lo.astype(np.int64) << 20) | (md.astype(np.int64) << 10) | hi
        # 30-bit fields reproduce Eq. 1 exactly (spot check against exact rationals)
        for i in range(0, B.n, 997):
            b = i // 1024
            e = exact_ref.eq1_exact(float(B.xyz[i, a]), float(B.batches["min"][b][a]),
                                    float(B.batches["max"][b][a]))
            assert abs(int(X30[i]) - e) <= 1
    for word in (B.low, B.med, B.high):
        assert not (word >> 30).any()  # the two pad bits are zero


@pytest.mark.parametrize("k", [10, 20, 30])
def test_decode_error_bound(k):
    """Lower-corner decode: 0 <= x - (min + F size 2^-k) <= size 2^-k per axis, exactly."""
    xyz, rgba = synth.primitives(7, 20480)
    B = oracle.build_cloud(xyz, rgba, 10240, morton=False)
    for i in range(0, B.n, 37):
        b = i // 10240
        for a in range(3):
            mn = Fraction(float(B.batches["min"][b][a]))
            mx = Fraction(float(B.batches["max"][b][a]))
            s = mx - mn
            lo = (int(B.low[i]) >> (10 * a)) & 1023
            md = (int(B.med[i]) >> (10 * a)) & 1023
            hi = (int(B.high[i]) >> (10 * a)) & 1023
            F = {10: lo, 20: (lo << 10) | md, 30: (lo << 20) | (md << 10) | hi}[k]
            dec = mn + F * s / 2 ** k
            x = Fraction(float(B.xyz[i, a]))
            err = x - dec
            assert err >= 0 or (k == 30 and -err <= s / 2 ** 30)  # binary64 Eq. 1 may round up by 1
            assert err <= s / 2 ** k * (1 + Fraction(1, 2 ** 20))


# ------------------------------------------------------ exact brute force
def _tiny_cloud(rng, n):
    kind = rng.integers(3)
    if kind == 0:
        pts = rng.uniform(0, 10, (n, 3))
    elif kind == 1:  # clustered, Morton-like compact batches
        c = rng.uniform(0, 10, (4, 3))
        pts = c[rng.integers(0, 4, n)] + rng.normal(0, 0.3, (n, 3))
    else:  # a plane with a few duplicates and a zero-extent axis
        pts = np.column_stack([rng.uniform(0, 10, n), rng.uniform(0, 10, n), np.full(n, 5.0)])
        pts[rng.integers(0, n, n // 8)] = pts[0]
    return pts.astype(np.float32)


@pytest.mark.parametrize("seed", range(16))
def test_oracle_equals_exact_bruteforce(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(60, 400))
    S = int(rng.choice([4, 8, 16, 32]))
    xyz = _tiny_cloud(rng, n)
    rgba = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    morton = bool(seed % 2)
    B = oracle.build_cloud(xyz, rgba, S, morton=morton)
    w, h = int(rng.integers(8, 40)), int(rng.integers(8, 40))
    cam = synth.random_camera(rng, w, h, inside=bool(seed % 3 == 0), box=((0, 0, 0), (10, 10, 10)))
    # thresholds scaled to tiny images so that all three levels occur
    for prec, t10, t20 in [(0, 3.0, 9.0), (0, 500.0, 512000.0), (10, 500.0, 512000.0),
                           (20, 500.0, 512000.0), (30, 500.0, 512000.0)]:
        o = oracle.opts(precision=prec, t10=t10, t20=t20)
        vb, st = oracle.render(B, cam.view, cam.proj, w, h, o)
        got = {int(p): int(vb[p]) for p in np.nonzero(vb != oracle.EMPTY)[0]}
        want, levels = exact_ref.brute_force(B.xyz.tolist(), S, cam.view.tolist(), cam.proj.tolist(), w, h,
                                             prec, t10, t20)
        dec = oracle.decide_all(B.batches, cam.view, cam.proj, w, h, o)
        assert dec["level"].tolist() == levels
        assert got == want


def test_exact_floor_on_pixel_edges():
    """Points whose hx/hw is exactly an integer, and their float neighbours on either side."""
    view = np.eye(4, dtype=np.float32)
    proj = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, -2, -3], [0, 0, -1, 0]], np.float32)
    pts = []
    for z in (-1.0, -3.0, -0.75):
        for px in range(-3, 12):  # hx/hw = 4(x/(-z) + 1) = px  ->  x = (px/4 - 1)(-z)
            x = np.float32((px / 4.0 - 1.0) * (-z))
            for xx in (x, np.nextafter(x, np.float32(-np.inf)), np.nextafter(x, np.float32(np.inf))):
                pts.append([xx, np.float32(0.3 * -z), z])
    xyz = np.array(pts, np.float32)
    rgba = np.arange(len(pts), dtype=np.uint32)
    B = oracle.build_cloud(xyz, rgba, 4, morton=False)
    for prec in (10, 20, 30):
        o = oracle.opts(precision=prec)
        vb, _ = oracle.render(B, view, proj, 8, 8, o)
        got = {int(p): int(vb[p]) for p in np.nonzero(vb != oracle.EMPTY)[0]}
        want, _ = exact_ref.brute_force(B.xyz.tolist(), 4, view.tolist(), proj.tolist(), 8, 8, prec)
        assert got == want


# ---------------------------------------------------------- level threshold
@pytest.mark.parametrize("extent,level", [(499.5, 10), (500.0, 20), (500.5, 20), (1.0, 10)])
def test_level_threshold_500px(extent, level):
    """A box at depth 1 whose projection is exactly `extent` pixels wide (W = 1024)."""
    view = np.eye(4, dtype=np.float32)
    proj = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, -2, -3], [0, 0, -1, 0]], np.float32)
    L = extent / 512.0  # hx/hw = 512 (x + 1) at z = -1
    xyz = np.array([[-0.5, -0.1, -1.0], [-0.5 + L, 0.1, -1.0]], np.float32)
    assert float(xyz[1, 0] - xyz[0, 0]) == L
    B = oracle.build_cloud(xyz, np.zeros(2, np.uint32), 4, morton=False)
    dec = oracle.decide_all(B.batches, view, proj, 1024, 1024, oracle.opts())
    assert int(dec["level"][0]) == level


def test_level_infinite_when_box_reaches_behind_eye():
    view = np.eye(4, dtype=np.float32)
    proj = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, -2, -3], [0, 0, -1, 0]], np.float32)
    xyz = np.array([[0.0, 0.0, -1.0], [0.001, 0.001, 0.5]], np.float32)  # tiny box crossing w = 0
    B = oracle.build_cloud(xyz, np.zeros(2, np.uint32), 4, morton=False)
    dec = oracle.decide_all(B.batches, view, proj, 64, 64, oracle.opts())
    assert int(dec["level"][0]) == 30 and int(dec["culled"][0]) == 0


# ------------------------------------------------------ textbook pipeline
def test_textbook_pipeline_agreement():
    """FORCE30 pixels and depths agree with the float64 OpenGL pipeline
    (clip = P V p, NDC = clip/w, window = (NDC + 1) size / 2, row 0 at the bottom)."""
    xyz, rgba = synth.primitives(3, 100_000)
    B = oracle.build_cloud(xyz, rgba, 10240, morton=False)
    cam = synth.c1_camera()
    W, H = cam.width, cam.height
    vb, _ = oracle.render(B, cam.view, cam.proj, W, H, oracle.opts(precision=30))
    M = cam.proj.astype(np.float64) @ cam.view.astype(np.float64)
    P4 = np.column_stack([B.xyz.astype(np.float64), np.ones(B.n)])
    clip = P4 @ M.T
    wx = (clip[:, 0] / clip[:, 3] + 1.0) * W / 2.0
    wy = (clip[:, 1] / clip[:, 3] + 1.0) * H / 2.0
    inview = (clip[:, 3] > 0) & (wx >= 0) & (wx < W) & (wy >= 0) & (wy < H)
    edge = (np.abs(wx - np.round(wx)) < 1e-3) | (np.abs(wy - np.round(wy)) < 1e-3)
    pix = np.floor(wy).astype(np.int64) * W + np.floor(wx).astype(np.int64)
    covered = np.nonzero(vb != oracle.EMPTY)[0]
    assert len(covered) > 1000
    win = (vb[covered] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    hw_bits = (vb[covered] >> np.uint64(32)).astype(np.uint32)
    hw = hw_bits.view(np.float32).astype(np.float64)
    ok = ~edge[win]
    assert (pix[win][ok] == covered[ok]).all()  # the winner's textbook pixel is this pixel
    assert inview[win].all()
    np.testing.assert_allclose(hw, clip[win, 3], rtol=1e-5)  # key depth is w_clip = -z_eye
    # every in-view point (away from edges) lands on a covered pixel whose winner is no farther
    sel = inview & ~edge
    vb_at = vb[pix[sel]]
    assert (vb_at != oracle.EMPTY).all()
    win_depth = (vb_at >> np.uint64(32)).astype(np.uint32).view(np.float32).astype(np.float64)
    assert (win_depth <= clip[sel, 3] * (1 + 1e-5)).all()


# ------------------------------------------------------------------ Morton
def _less_msb(a, b):
    return a < b and a < (a ^ b)


def _zorder_less(p, q):
    """Chan's comparator: compare along the axis whose XOR has the highest set bit;
    at equal bit positions z outranks y outranks x (code bit 3b + axis)."""
    j, x = None, 0
    for k in (2, 1, 0):
        y = p[k] ^ q[k]
        if _less_msb(x, y):
            j, x = k, y
    if j is None:
        return False
    return p[j] < q[j]


def test_morton_codes_order_matches_comparator():
    rng = np.random.default_rng(5)
    xyz = rng.uniform(-50, 50, (3000, 3)).astype(np.float32)
    mn, mx = oracle.cloud_aabb(xyz)
    codes = oracle.morton_codes(xyz, mn, mx)
    assert (codes < (1 << 63)).all()
    q = np.empty((3000, 3), np.int64)
    for i in range(3000):
        for a in range(3):
            r = (Fraction(float(xyz[i, a])) - Fraction(float(mn[a]))) * 2 ** 21 / (
                Fraction(float(mx[a])) - Fraction(float(mn[a])))
            q[i, a] = min(r.numerator // r.denominator, 2 ** 21 - 1)
    for _ in range(20000):
        i, j = rng.integers(0, 3000, 2)
        if i == j:
            continue
        assert (codes[i] < codes[j]) == _zorder_less(q[i], q[j])


def test_morton_grid_z_curve():
    # the 8 corners of a unit cube in z-order: x fastest, then y, then z
    g = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], np.float32)
    rng = np.random.default_rng(0)
    shuffled = g[rng.permutation(8)]
    mn, mx = oracle.cloud_aabb(shuffled)
    codes = oracle.morton_codes(shuffled, mn, mx)
    order = oracle.morton_order(codes)
    assert shuffled[order].tolist() == g.tolist()


@pytest.mark.parametrize("n,S", [(5003, 64), (10240 * 3 + 777, 10240), (7, 4), (1, 4)])
def test_spread_order_keeps_each_batch_and_steps_across_it(n, S):
    """The spread build (morton = 2) stores each batch of the Morton build in another order: the same points, the
    same batch records, and Eq. 1 words that follow the points; inside a batch of c points the Morton ranks advance
    by one fixed step coprime with c, just above c / 4, so that the four points of a quadruple lie in four quarters
    of the batch while the quadruples' j-th points are Morton neighbours."""
    rng = np.random.default_rng(n)
    xyz = rng.uniform(-20, 20, (n, 3)).astype(np.float32)
    rgba = rng.integers(0, 2**32, n, dtype=np.uint32)
    A = oracle.build_cloud(xyz, rgba, S, morton=1)
    B = oracle.build_cloud(xyz, rgba, S, morton=2)
    assert np.array_equal(A.batches, B.batches)
    pos_in_a = np.empty(n, np.int64)
    pos_in_a[A.perm] = np.arange(n)
    for b0 in range(0, n, S):
        c = min(S, n - b0)
        ranks = pos_in_a[B.perm[b0:b0 + c]] - b0  # Morton rank inside the batch of each spread position
        assert sorted(ranks.tolist()) == list(range(c))
        if c > 1:
            steps = np.unique((ranks[1:] - ranks[:-1]) % c)
            assert len(steps) == 1 and math.gcd(int(steps[0]), c) == 1
            assert c // 4 < int(steps[0]) <= c // 4 + 8
            if c % 4 == 0 and int(steps[0]) == c // 4 + 1:  # quadruple q, point j: rank 4q + j * step (mod c)
                q = np.arange(c // 4)
                for j in range(4):
                    assert np.array_equal(ranks[4 * q + j], (4 * q + j * int(steps[0])) % c)
        assert ranks[0] == 0
        src = A.perm[b0 + ranks]
        assert np.array_equal(B.perm[b0:b0 + c], src)
        assert np.array_equal(B.xyz[b0:b0 + c], A.xyz[b0 + ranks])
        assert np.array_equal(B.colors[b0:b0 + c], A.colors[b0 + ranks])
        for f in ("low", "med", "high"):
            assert np.array_equal(getattr(B, f)[b0:b0 + c], getattr(A, f)[b0 + ranks])


def test_morton_order_is_stable():
    rng = np.random.default_rng(9)
    base = rng.uniform(0, 1, (50, 3)).astype(np.float32)
    xyz = base[rng.integers(0, 50, 2000)]  # many exact duplicates
    mn, mx = oracle.cloud_aabb(xyz)
    codes = oracle.morton_codes(xyz, mn, mx)
    perm = oracle.morton_order(codes)
    ref = sorted(range(2000), key=lambda i: int(codes[i]))  # Python's sort is stable
    assert perm.tolist() == ref


# -------------------------------------------------------------- invariants
@pytest.mark.parametrize("seed", range(4))
def test_culling_never_changes_the_image(seed):
    rng = np.random.default_rng(seed)
    xyz, rgba = synth.terrain(seed + 20, 60000, order=0)
    B = oracle.build_cloud(xyz, rgba, 1024, morton=True)
    cam = synth.random_camera(rng, 320, 200, inside=bool(seed % 2), box=((0, 0, -50), (1000, 1000, 100)))
    on, st_on = oracle.render(B, cam.view, cam.proj, 320, 200, oracle.opts(cull=1))
    off, st_off = oracle.render(B, cam.view, cam.proj, 320, 200, oracle.opts(cull=0))
    assert np.array_equal(on, off)
    dec = oracle.decide_all(B.batches, cam.view, cam.proj, 320, 200, oracle.opts(cull=1))
    culled = np.nonzero(dec["culled"])[0]
    assert st_on["culled"] == len(culled)
    if len(culled):
        alone, _ = oracle.render(B, cam.view, cam.proj, 320, 200, oracle.opts(cull=0), batch_ids=culled)
        assert (alone == oracle.EMPTY).all()


def test_batch_subsets_compose_by_minimum():
    xyz, rgba = synth.primitives(4, 50000)
    B = oracle.build_cloud(xyz, rgba, 1024, morton=False)
    cam = synth.c1_camera()
    full, _ = oracle.render(B, cam.view, cam.proj, cam.width, cam.height)
    nb = B.batches.shape[0]
    ids = np.random.default_rng(1).permutation(nb)
    vb = np.full(cam.width * cam.height, oracle.EMPTY, np.uint64)
    oracle.render(B, cam.view, cam.proj, cam.width, cam.height, batch_ids=ids[: nb // 2], vb=vb)
    oracle.render(B, cam.view, cam.proj, cam.width, cam.height, batch_ids=ids[nb // 2:][::-1], vb=vb)
    assert np.array_equal(full, vb)


def test_resolve_identity():
    rng = np.random.default_rng(2)
    colors = rng.integers(0, 2 ** 32, 1000, dtype=np.uint64).astype(np.uint32)
    idx = rng.integers(0, 1000, 500)
    keys = (rng.integers(0x3F800000, 0x4F000000, 500).astype(np.uint64) << np.uint64(32)) | idx.astype(np.uint64)
    vb = np.full(700, oracle.EMPTY, np.uint64)
    vb[:500] = keys
    fb = oracle.resolve(vb, colors, 0xDEADBEEF)
    assert (fb[:500] == colors[idx]).all()
    assert (fb[500:] == 0xDEADBEEF).all()


def test_key_exact_in_numpy_and_torch():
    import torch

    keys = np.array([0, 1, 0x40C0000000000000, 0x7F7FFFFFFFFFFFFF, 0xFFFFFFFFFFFFFFFF], np.uint64)
    t = torch.from_numpy(keys.view(np.int64).copy())
    back = t.numpy().view(np.uint64)
    assert back.tolist() == keys.tolist()
    assert int(t[-1]) == -1  # EMPTY must never be compared as signed
    assert float(np.float64(0x40C0000000000001)) == float(np.float64(0x40C0000000000000))  # why keys never go through float


def test_validate_rejects_non_finite():
    xyz, rgba = synth.primitives(2, 1000)
    assert oracle.validate(xyz) == -1
    for bad in (np.nan, np.inf, -np.inf):
        x = xyz.copy()
        x[617, 1] = bad
        assert oracle.validate(x) == 617
        with pytest.raises(ValueError):
            oracle.build_cloud(x, rgba, 64)


def test_signed_zero_boxes_use_total_order():
    """-0 sorts below +0 in every box, whichever order the points come in."""
    for pts in ([[0.0, -0.0, 1.0], [-0.0, 0.0, 1.0]], [[-0.0, 0.0, 1.0], [0.0, -0.0, 1.0]]):
        xyz = np.array(pts, np.float32)
        B = oracle.build_cloud(xyz, np.zeros(2, np.uint32), 4, morton=False)
        mn = B.batches["min"][0].view(np.uint32).tolist()
        mx = B.batches["max"][0].view(np.uint32).tolist()
        assert mn[:2] == [0x80000000, 0x80000000] and mx[:2] == [0, 0]
        cmn, cmx = oracle.cloud_aabb(xyz)
        assert cmn.view(np.uint32).tolist()[:2] == [0x80000000] * 2
        assert cmx.view(np.uint32).tolist()[:2] == [0, 0]


def test_resolve_foreign_index_gives_clear():
    colors = np.arange(10, dtype=np.uint32) + 100
    vb = np.array([3, 10, 0xFFFFFFFF, (0x40000000 << 32) | 9], np.uint64)
    assert oracle.resolve(vb, colors, 7).tolist() == [103, 7, 7, 109]


# ------------------------------------------------------- high-quality shading (Sec. 3.6)
def _worked_built():
    g = _gold()
    xyz = np.array(g["points"], np.float32)
    cols = np.array([_hex(c) for c in g["colors"]], np.uint32)
    B = oracle.build_cloud(xyz, cols, g["batch_size"], morton=False)
    view, proj = np.array(g["view"], np.float32), np.array(g["proj"], np.float32)
    return g, B, view, proj


@pytest.mark.parametrize("window", ["1.01", "1.3"])
def test_hqs_worked_example(window):
    """Hand-derived sums and averages (tests/golden/worked_example.json, hqs)."""
    g, B, view, proj = _worked_built()
    w, h = g["width"], g["height"]
    vb, _ = oracle.render(B, view, proj, w, h)
    acc = oracle.accumulate(B, view, proj, w, h, vb, window=float(window))
    want = g["hqs"][window]
    covered = {int(p) for p in np.nonzero(acc[1::2] >> np.uint64(32))[0]}
    assert covered == {int(p) for p in want["acc"]}
    for p, (a0, a1) in want["acc"].items():
        assert (int(acc[2 * int(p)]), int(acc[2 * int(p) + 1])) == (a0, a1)
    fb = oracle.resolve_hqs(acc, 0)
    for p in range(w * h):
        assert int(fb[p]) == (_hex(want["fb"][str(p)]) if str(p) in want["fb"] else 0)


@pytest.mark.parametrize("seed", range(8))
def test_hqs_matches_exact_bruteforce(seed):
    """Exact-rational reference: every drawn point's hw, the window threshold rounded once to binary32, the
    packed sums modulo 2^64."""
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(60, 300))
    S = int(rng.choice([4, 8, 16]))
    xyz = _tiny_cloud(rng, n)
    rgba = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    B = oracle.build_cloud(xyz, rgba, S, morton=bool(seed % 2))
    w, h = int(rng.integers(8, 30)), int(rng.integers(8, 30))
    cam = synth.random_camera(rng, w, h, inside=bool(seed % 3 == 0), box=((0, 0, 0), (10, 10, 10)))
    for window, prec in [(1.0, 0), (1.01, 0), (1.2, 10), (3.0, 30)]:
        o = oracle.opts(precision=prec)
        vb, _ = oracle.render(B, cam.view, cam.proj, w, h, o)
        acc = oracle.accumulate(B, cam.view, cam.proj, w, h, vb, window=window, o=o)
        want = exact_ref.brute_force_hqs(B.xyz.tolist(), B.colors.tolist(), S, cam.view.tolist(), cam.proj.tolist(),
                                         w, h, window, prec)
        got = {p: (int(acc[2 * p]), int(acc[2 * p + 1])) for p in range(w * h) if acc[2 * p + 1] != 0}
        assert got == want


def test_hqs_window_one_keeps_the_ties_at_the_closest_depth():
    g, B, view, proj = _worked_built()
    vb, _ = oracle.render(B, view, proj, g["width"], g["height"])
    acc = oracle.accumulate(B, view, proj, g["width"], g["height"], vb, window=1.0)
    counts = {int(p): int(acc[2 * p + 1] >> np.uint64(32)) for p in np.nonzero(acc[1::2])[0]}
    assert counts == {18: 4, 20: 2, 63: 1}  # four points share depth 6, two share depth 4


def test_hqs_resolve_rounds_to_nearest():
    H = 1 << 32
    acc = np.array([3 + 5 * H, 7 + 2 * H,      # R 3/2 -> 2 (half up), G 5/2 -> 3, B 7/2 -> 4
                    0, 0,                       # nothing joined: clear colour
                    255 * 3 + 0 * H, 1 + 3 * H],  # R 255, G 0, B 1/3 -> 0
                   np.uint64)
    fb = oracle.resolve_hqs(acc, 0x12345678)
    assert fb.tolist() == [0xFF040302, 0x12345678, 0xFF0000FF]


# ------------------------------------------------------------------ LOD (Sec. 3.5)
def _lpc_cloud(seed, n, cap=64):
    rng = np.random.default_rng(seed)
    xyz = _tiny_cloud(rng, n)
    rgba = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    depth = synth.lpc_depth(n, cap)
    xo, ro, spans, nodes = synth.lpc_layout(seed, xyz, rgba, depth, cap)
    return rng, oracle.build_cloud_spans(xo, ro, spans, nodes), spans, nodes


@pytest.mark.parametrize("seed", range(6))
def test_lod_culling_matches_exact_cube_extent(seed):
    """A node below the root is culled iff its cube's exact projected extent is below lod_px (decisions within a
    relative 1e-9 of the threshold are not compared)."""
    rng, B, spans, nodes = _lpc_cloud(400 + seed, 3000)
    w, h = int(rng.integers(40, 200)), int(rng.integers(40, 200))
    for _ in range(20):  # a camera that sees some batch below the root
        cam = synth.random_camera(rng, w, h, box=((0, 0, 0), (10, 10, 10)))
        d = oracle.decide_all(B.batches, cam.view, cam.proj, w, h, oracle.opts(), nodes)
        if np.any((d["culled"] == 0) & (nodes[:, 4] >= 1)):
            break
    for lod_px in (2.0, 10.0, 40.0):
        d_lod = oracle.decide_all(B.batches, cam.view, cam.proj, w, h, oracle.opts(lod_px=lod_px), nodes)
        d_off = oracle.decide_all(B.batches, cam.view, cam.proj, w, h, oracle.opts(), nodes)
        compared = 0
        for b in range(len(spans)):
            if d_off["culled"][b]:
                assert d_lod["culled"][b]
                continue
            if nodes[b, 4] == 0:
                assert not d_lod["culled"][b]
                continue
            E = exact_ref.cube_extent(cam.view.tolist(), cam.proj.tolist(), w, h, nodes[b, :3], nodes[b, 3])
            if E is not None and abs(float(E) - lod_px) <= 1e-9 * lod_px:
                continue
            assert bool(d_lod["culled"][b]) == (E is not None and E < lod_px), (b, E, lod_px)
            compared += 1
        assert compared > 0


@pytest.mark.parametrize("seed", range(4))
def test_lod_off_equals_exact_bruteforce_over_spans(seed):
    rng, B, spans, nodes = _lpc_cloud(500 + seed, 400, cap=32)
    w, h = int(rng.integers(8, 30)), int(rng.integers(8, 30))
    cam = synth.random_camera(rng, w, h, inside=bool(seed % 2), box=((0, 0, 0), (10, 10, 10)))
    vb, _ = oracle.render(B, cam.view, cam.proj, w, h)
    got = {int(p): int(vb[p]) for p in np.nonzero(vb != oracle.EMPTY)[0]}
    assert got == exact_ref.brute_force_spans(B.xyz.tolist(), spans.tolist(), cam.view.tolist(), cam.proj.tolist(),
                                              w, h)


def test_lod_renders_exactly_the_surviving_batches_and_is_monotone():
    rng, B, spans, nodes = _lpc_cloud(600, 4000)
    cam = synth.random_camera(rng, 160, 120, box=((0, 0, 0), (10, 10, 10)))
    prev = None
    for lod_px in (0.0, 5.0, 20.0, 80.0, 1e6):
        o = oracle.opts(lod_px=lod_px)
        vb, st = oracle.render(B, cam.view, cam.proj, 160, 120, o)
        dec = oracle.decide_all(B.batches, cam.view, cam.proj, 160, 120, o, nodes)
        keep = np.nonzero(dec["culled"] == 0)[0].astype(np.uint64)
        B_plain = oracle.build_cloud_spans(B.xyz, B.colors, spans)  # no nodes: no LOD culling
        sub, _ = oracle.render(B_plain, cam.view, cam.proj, 160, 120, batch_ids=keep)
        assert np.array_equal(vb, sub)
        assert st["culled"] == int(np.count_nonzero(dec["culled"]))
        if prev is not None:
            assert np.all(dec["culled"] >= prev)  # a larger threshold never brings a node back
        prev = dec["culled"]
    assert not np.any(dec["culled"][nodes[:, 4] == 0] & (oracle.decide_all(
        B.batches, cam.view, cam.proj, 160, 120, oracle.opts(), nodes)["culled"] == 0))

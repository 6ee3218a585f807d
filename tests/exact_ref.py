"""Exact-rational brute force used to pin the CPU oracle (tiny inputs only).

Independent of ``oracle/``: nothing here calls or reads it.  Every binary32
rounding is performed explicitly from the IEEE 754 definition
(round-to-nearest, ties-to-even) on exact ``Fraction`` values, so a fused
multiply-add is ``round32(a*b + c)`` with no intermediate rounding, and the
pixel is the exact floor of the rational quotient.  The per-batch binary64
steps use Python floats (IEEE binary64, one rounding per operation, never
fused).

The brute force is pixel-major over *all* points: no culling, no early
depth test, no batch order -- only each point's own batch box and precision
level enter, as the method defines.
"""
from __future__ import annotations

import math
import struct
from fractions import Fraction

TWO30 = 1 << 30


# --------------------------------------------------------- binary32 rounding
def round32(x: Fraction) -> Fraction:
    """Round an exact rational to the nearest binary32 value (ties to even).
    Returns a Fraction, or +-inf as a float."""
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    a = -x if x < 0 else x
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)  # subnormal range shares the exponent of 2^-126
    q = 2 ** (e - 23)  # spacing of binary32 values in [2^e, 2^(e+1))
    m = a / Fraction(q)
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    r = Fraction(fl) * Fraction(q)
    if r >= Fraction(2) ** 128 - Fraction(2) ** 103:  # beyond max finite after rounding
        return float("inf") * sign
    return r * sign


def f32(x) -> Fraction:
    """Exact value of a Python float / int after rounding to binary32."""
    return round32(Fraction(x))


def fma32(a: Fraction, b: Fraction, c: Fraction) -> Fraction:
    return round32(a * b + c)


def f32_bits(x: Fraction) -> int:
    return struct.unpack("<I", struct.pack("<f", float(x)))[0]


# ------------------------------------------------------------------- Eq. 1
def eq1_exact(x: float, bmin: float, bmax: float) -> int:
    """X30 = min(floor(2^30 (x - min) / size), 2^30 - 1), exact rationals; 0 for size 0."""
    s = Fraction(bmax) - Fraction(bmin)
    if s == 0:
        return 0
    q = (Fraction(x) - Fraction(bmin)) * TWO30 / s
    return min(q.numerator // q.denominator, TWO30 - 1)


# ------------------------------------------------- per-batch steps (binary64)
def frame_matrix(view, proj, w, h):
    """Rows: hx = (W/2)(C0 + C3), hy = (H/2)(C1 + C3), hw = C3, C = proj view."""
    v = [[float(view[i][j]) for j in range(4)] for i in range(4)]
    p = [[float(proj[i][j]) for j in range(4)] for i in range(4)]
    C = [[((p[i][0] * v[0][j] + p[i][1] * v[1][j]) + p[i][2] * v[2][j]) + p[i][3] * v[3][j]
          for j in range(4)] for i in range(4)]
    return [[(0.5 * w) * (C[0][j] + C[3][j]) for j in range(4)],
            [(0.5 * h) * (C[1][j] + C[3][j]) for j in range(4)],
            [C[3][j] for j in range(4)]]


def batch_level_and_fold(Pm, bmin, bmax, w, h, precision=0, t10=500.0, t20=512000.0):
    """Precision level k and the folded fp32 matrix of one batch."""
    s = [float(bmax[a]) - float(bmin[a]) for a in range(3)]
    H = [[0.0] * 8 for _ in range(3)]
    for c in range(8):
        cx = float(bmax[0] if c & 1 else bmin[0])
        cy = float(bmax[1] if c & 2 else bmin[1])
        cz = float(bmax[2] if c & 4 else bmin[2])
        for r in range(3):
            H[r][c] = ((Pm[r][0] * cx + Pm[r][1] * cy) + Pm[r][2] * cz) + Pm[r][3]
    if precision in (10, 20, 30):
        k = precision
    else:
        if all(H[2][c] > 0.0 for c in range(8)):
            u = [H[0][c] / H[2][c] for c in range(8)]
            v = [H[1][c] / H[2][c] for c in range(8)]
            E = max(max(u) - min(u), max(v) - min(v))
        else:
            E = math.inf
        k = 10 if E < float(f32(t10)) else (20 if E < float(f32(t20)) else 30)
    scale = 2.0 ** -k
    P = [[f32(Pm[r][j] * (s[j] * scale)) for j in range(3)] for r in range(3)]
    t = [f32(((Pm[r][0] * float(bmin[0]) + Pm[r][1] * float(bmin[1])) + Pm[r][2] * float(bmin[2])) + Pm[r][3])
         for r in range(3)]
    return k, P, t


# --------------------------------------------------------------- brute force
def point_key(i, xyz_i, bmin, bmax, k, P, t, w, h):
    """(pixel, key) of one point, or None if it lands outside the image."""
    F = []
    for a in range(3):
        X30 = eq1_exact(float(xyz_i[a]), float(bmin[a]), float(bmax[a]))
        F.append(f32(X30 >> (30 - k)))
    hx = fma32(P[0][2], F[2], fma32(P[0][1], F[1], fma32(P[0][0], F[0], t[0])))
    hy = fma32(P[1][2], F[2], fma32(P[1][1], F[1], fma32(P[1][0], F[0], t[1])))
    hw = fma32(P[2][2], F[2], fma32(P[2][1], F[1], fma32(P[2][0], F[0], t[2])))
    if isinstance(hw, float) or isinstance(hx, float) or isinstance(hy, float):
        return None  # overflowed; never produced by the test inputs
    if not hw > 0:
        return None
    if not (0 <= hx < w * hw and 0 <= hy < h * hw):
        return None
    qx, qy = hx / hw, hy / hw
    px = qx.numerator // qx.denominator
    py = qy.numerator // qy.denominator
    return py * w + px, (f32_bits(hw) << 32) | i


def brute_force(xyz_sorted, batch_size, view, proj, w, h, precision=0, t10=500.0, t20=512000.0):
    """dict pixel -> min key over every point; points are in render order."""
    n = len(xyz_sorted)
    Pm = frame_matrix(view, proj, w, h)
    out = {}
    levels = []
    for b0 in range(0, n, batch_size):
        pts = xyz_sorted[b0:b0 + batch_size]
        bmin = [min(float(p[a]) for p in pts) for a in range(3)]
        bmax = [max(float(p[a]) for p in pts) for a in range(3)]
        # batch boxes are fp32 values already (min/max of fp32 inputs)
        k, P, t = batch_level_and_fold(Pm, bmin, bmax, w, h, precision, t10, t20)
        levels.append(k)
        for j, p in enumerate(pts):
            r = point_key(b0 + j, p, bmin, bmax, k, P, t, w, h)
            if r is None:
                continue
            pix, key = r
            if pix not in out or key < out[pix]:
                out[pix] = key
    return out, levels


def brute_force_hqs(xyz_sorted, colors, batch_size, view, proj, w, h, window, precision=0):
    """High-quality shading sums by definition: dict pixel -> (R + G*2^32, B + count*2^32) mod 2^64 over the
    points within round32(closest hw * round32(window)) of each pixel's closest point."""
    n = len(xyz_sorted)
    Pm = frame_matrix(view, proj, w, h)
    hits = {}
    for b0 in range(0, n, batch_size):
        pts = xyz_sorted[b0:b0 + batch_size]
        bmin = [min(float(p[a]) for p in pts) for a in range(3)]
        bmax = [max(float(p[a]) for p in pts) for a in range(3)]
        k, P, t = batch_level_and_fold(Pm, bmin, bmax, w, h, precision)
        for j, p in enumerate(pts):
            r = point_key(b0 + j, p, bmin, bmax, k, P, t, w, h)
            if r is None:
                continue
            pix, key = r
            hw = Fraction(struct.unpack("<f", struct.pack("<I", key >> 32))[0])
            hits.setdefault(pix, []).append((hw, int(colors[b0 + j])))
    win = f32(window)
    out = {}
    M = 1 << 64
    for pix, lst in hits.items():
        thr = round32(min(hw for hw, _ in lst) * win)
        a0 = a1 = 0
        for hw, c in lst:
            if hw <= thr:
                a0 = (a0 + (c & 255) + (((c >> 8) & 255) << 32)) % M
                a1 = (a1 + ((c >> 16) & 255) + (1 << 32)) % M
        out[pix] = (a0, a1)
    return out


def brute_force_spans(xyz, spans, view, proj, w, h, precision=0):
    """As brute_force, for variable-size batches given as (first, count) spans over xyz (render order)."""
    Pm = frame_matrix(view, proj, w, h)
    out = {}
    for first, count in spans:
        pts = xyz[first:first + count]
        bmin = [min(float(p[a]) for p in pts) for a in range(3)]
        bmax = [max(float(p[a]) for p in pts) for a in range(3)]
        k, P, t = batch_level_and_fold(Pm, bmin, bmax, w, h, precision)
        for j, p in enumerate(pts):
            r = point_key(first + j, p, bmin, bmax, k, P, t, w, h)
            if r is None:
                continue
            pix, key = r
            if pix not in out or key < out[pix]:
                out[pix] = key
    return out


def cube_extent(view, proj, w, h, origin, edge):
    """Projected extent of the cube [origin, origin + edge] in exact rationals: the larger side of the screen box
    of its 8 projected corners, or None if a corner has w <= 0."""
    Pm = [[Fraction(x) for x in row] for row in frame_matrix(view, proj, w, h)]
    us, vs = [], []
    for c in range(8):
        p = [Fraction(origin[a]) + (Fraction(edge) if (c >> a) & 1 else 0) for a in range(3)]
        hx, hy, hw = (sum(Pm[r][j] * p[j] for j in range(3)) + Pm[r][3] for r in range(3))
        if hw <= 0:
            return None
        us.append(hx / hw)
        vs.append(hy / hw)
    return max(max(us) - min(us), max(vs) - min(vs))

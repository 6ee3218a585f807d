"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Python (ctypes + numpy) access to ``ptoracle.c``, the plain single-threaded
reference of the rasterizer's build, render and resolve steps.  Only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package; the GPU library (``paper_2204_01287_amd``) never does, and the
two share no code.  Parity pins for every function are in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libptoracle.so")
_lib = None

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)

BATCH_DTYPE = np.dtype([("first", "<u4"), ("count", "<u4"), ("min", "<f4", (3,)), ("max", "<f4", (3,))])
assert BATCH_DTYPE.itemsize == 32
DECISION_DTYPE = np.dtype([("culled", "<i4"), ("level", "<i4"), ("P", "<f4", (3, 3)), ("t", "<f4", (3,))])


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("cull", ctypes.c_int), ("t10", ctypes.c_float),
                ("t20", ctypes.c_float), ("lod_px", ctypes.c_float)]


class Stats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("culled", ctypes.c_uint64), ("points", ctypes.c_uint64),
                ("level_batches", ctypes.c_uint64 * 3), ("level_points", ctypes.c_uint64 * 3)]

    def as_dict(self):
        return {"batches": self.batches, "culled": self.culled, "points": self.points,
                "level_batches": list(self.level_batches), "level_points": list(self.level_points)}


def build(force: bool = True) -> str:
    """Compile ptoracle.c (gcc, contraction off, no fast-math)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-frounding-math",
               "-o", _SO + ".tmp", os.path.join(_HERE, "ptoracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _lib_():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        P, U64, U32, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.or_validate.argtypes = [P, U64]
        L.or_validate.restype = ctypes.c_int64
        L.or_cloud_aabb.argtypes = [P, U64, P, P]
        L.or_morton_codes.argtypes = [P, U64, P, P, P]
        L.or_morton_order.argtypes = [P, U64, P]
        L.or_morton_order.restype = I
        L.or_batch_count.argtypes = [U64, U32]
        L.or_batch_count.restype = U64
        L.or_make_batches.argtypes = [P, U64, U32, P]
        L.or_eq1.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_float]
        L.or_eq1.restype = U32
        L.or_quantize.argtypes = [P, P, U64, P, P, P]
        L.or_build.argtypes = [P, P, U64, U32, I, P, P, P, P, P, P, P]
        L.or_build.restype = I
        L.or_spread_multiplier.argtypes = [U64]
        L.or_spread_multiplier.restype = U64
        L.or_frame_matrix.argtypes = [P, P, U32, U32, P]
        L.or_decide_all.argtypes = [P, P, U64, P, P, U32, U32, ctypes.POINTER(Opts), P]
        L.or_render.argtypes = [P, P, U64, P, U64, P, P, P, P, P, U32, U32, ctypes.POINTER(Opts), P,
                                ctypes.POINTER(Stats)]
        L.or_make_batches_spans.argtypes = [P, P, U64, P]
        L.or_resolve.argtypes = [P, U64, P, U64, U32, P]
        L.or_accumulate.argtypes = [P, P, U64, P, U64, P, P, P, P, P, P, U32, U32, ctypes.POINTER(Opts),
                                    ctypes.c_float, P, P]
        L.or_resolve_hqs.argtypes = [P, U64, U32, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None else None


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def opts(precision: int = 0, cull: int = 1, t10: float = 500.0, t20: float = 512000.0, lod_px: float = 0.0) -> Opts:
    return Opts(precision, cull, t10, t20, lod_px)


def validate(xyz) -> int:
    xyz = _c(xyz, np.float32)
    return int(_lib_().or_validate(_p(xyz), xyz.shape[0]))


def cloud_aabb(xyz):
    xyz = _c(xyz, np.float32)
    mn = np.empty(3, np.float32)
    mx = np.empty(3, np.float32)
    _lib_().or_cloud_aabb(_p(xyz), xyz.shape[0], _p(mn), _p(mx))
    return mn, mx


def morton_codes(xyz, mn, mx):
    xyz = _c(xyz, np.float32)
    mn = _c(mn, np.float32)
    mx = _c(mx, np.float32)
    out = np.empty(xyz.shape[0], np.uint64)
    _lib_().or_morton_codes(_p(xyz), xyz.shape[0], _p(mn), _p(mx), _p(out))
    return out


def morton_order(codes):
    codes = _c(codes, np.uint64)
    perm = np.empty(codes.shape[0], np.uint32)
    if _lib_().or_morton_order(_p(codes), codes.shape[0], _p(perm)) != 0:
        raise MemoryError("or_morton_order")
    return perm


def batch_count(n: int, S: int) -> int:
    return int(_lib_().or_batch_count(n, S))


def make_batches(xyz, S: int):
    xyz = _c(xyz, np.float32)
    out = np.empty(batch_count(xyz.shape[0], S), BATCH_DTYPE)
    _lib_().or_make_batches(_p(xyz), xyz.shape[0], S, _p(out))
    return out


def eq1(x: float, bmin: float, bmax: float) -> int:
    return int(_lib_().or_eq1(x, bmin, bmax))


def quantize(xyz, batches):
    xyz = _c(xyz, np.float32)
    n = xyz.shape[0]
    low, med, high = (np.zeros(n, np.uint32) for _ in range(3))
    _lib_().or_quantize(_p(xyz), _p(batches), batches.shape[0], _p(low), _p(med), _p(high))
    return low, med, high


class Built:
    """Output of the oracle's load-time build, all in render order."""

    def __init__(self, n, S):
        self.n, self.S = n, S
        self.xyz = np.empty((n, 3), np.float32)
        self.colors = np.empty(n, np.uint32)
        self.perm = np.empty(n, np.uint32)
        self.batches = np.empty(batch_count(n, S), BATCH_DTYPE)
        self.low = np.empty(n, np.uint32)
        self.med = np.empty(n, np.uint32)
        self.high = np.empty(n, np.uint32)
        self.nodes = None  # LOD layouts: float64 (nb, 5) = cube origin x, y, z, edge, level


def spread_multiplier(c: int) -> int:
    """The step m of the spread order of a c-point batch: position r holds Morton rank (r * m) mod c."""
    return int(_lib_().or_spread_multiplier(c))


def build_cloud(xyz, rgba, S: int = 10240, morton: int = 0) -> Built:
    """morton: 0 input order, 1 Morton order, 2 Morton order with every batch in the spread order (position r holds
    the batch's Morton rank (r * m) mod c, m = spread_multiplier(c))."""
    xyz = _c(xyz, np.float32)
    rgba = _c(rgba, np.uint32)
    n = xyz.shape[0]
    B = Built(n, S)
    rc = _lib_().or_build(_p(xyz), _p(rgba), n, S, int(morton), _p(B.xyz), _p(B.colors), _p(B.perm),
                          _p(B.batches), _p(B.low), _p(B.med), _p(B.high))
    if rc != 0:
        raise ValueError(f"or_build failed ({rc})")
    return B


def build_cloud_spans(xyz, rgba, spans, nodes=None) -> Built:
    """Variable-size batches given as spans (first, count) over xyz / rgba in render order (Sec. 3.5); slots
    outside every span are padding.  nodes: optional LOD node per batch (cube origin x, y, z, edge, level)."""
    xyz = _c(xyz, np.float32)
    rgba = _c(rgba, np.uint32)
    spans = _c(spans, np.uint32)
    n, nb = xyz.shape[0], spans.shape[0]
    if nb and (np.any(spans[:, 0] % 4) or int((spans[:, 0].astype(np.uint64) + spans[:, 1]).max()) > n):
        raise ValueError("spans must start at multiples of 4 and lie inside the cloud")
    B = Built(n, max(n, 1))
    B.xyz[:] = xyz
    B.colors[:] = rgba
    B.perm[:] = np.arange(n, dtype=np.uint32)
    B.batches = np.empty(nb, BATCH_DTYPE)
    _lib_().or_make_batches_spans(_p(xyz), _p(spans), nb, _p(B.batches))
    B.low[:] = 0
    B.med[:] = 0
    B.high[:] = 0
    _lib_().or_quantize(_p(xyz), _p(B.batches), nb, _p(B.low), _p(B.med), _p(B.high))
    B.nodes = None if nodes is None else _c(nodes, np.float64)
    return B


def frame_matrix(view, proj, w: int, h: int):
    view = _c(view, np.float32)
    proj = _c(proj, np.float32)
    Pm = np.empty((3, 4), np.float64)
    _lib_().or_frame_matrix(_p(view), _p(proj), w, h, _p(Pm))
    return Pm


def decide_all(batches, view, proj, w: int, h: int, o: Opts | None = None, nodes=None):
    o = o or opts()
    view = _c(view, np.float32)
    proj = _c(proj, np.float32)
    nd = None if nodes is None else _c(nodes, np.float64)
    out = np.empty(batches.shape[0], DECISION_DTYPE)
    _lib_().or_decide_all(_p(batches), _p(nd), batches.shape[0], _p(view), _p(proj), w, h, ctypes.byref(o),
                          _p(out))
    return out


def render(built: Built, view, proj, w: int, h: int, o: Opts | None = None, batch_ids=None, vb=None):
    """Returns (vb uint64[h*w], stats dict).  vb, if given, is updated in place."""
    o = o or opts()
    view = _c(view, np.float32)
    proj = _c(proj, np.float32)
    if vb is None:
        vb = np.full(w * h, EMPTY, np.uint64)
    ids = None if batch_ids is None else _c(batch_ids, np.uint64)
    st = Stats()
    nd = getattr(built, "nodes", None)
    _lib_().or_render(_p(built.batches), _p(nd), built.batches.shape[0], _p(ids), 0 if ids is None else ids.shape[0],
                      _p(built.low), _p(built.med), _p(built.high), _p(view), _p(proj), w, h,
                      ctypes.byref(o), _p(vb), ctypes.byref(st))
    return vb, st.as_dict()


def resolve(vb, colors, clear_rgba: int = 0):
    vb = _c(vb, np.uint64)
    colors = _c(colors, np.uint32)
    fb = np.empty(vb.shape[0], np.uint32)
    _lib_().or_resolve(_p(vb), vb.shape[0], _p(colors), colors.shape[0], clear_rgba, _p(fb))
    return fb


def accumulate(built: Built, view, proj, w: int, h: int, vb, window: float = 1.01, o: Opts | None = None,
               batch_ids=None, colors=None):
    """High-quality shading sums (Sec. 3.6): uint64[2*h*w] (R + G<<32, B + count<<32 per pixel) of the points
    within fl32(closest depth * window) of each pixel's closest point; vb is the render of the same view."""
    o = o or opts()
    view = _c(view, np.float32)
    proj = _c(proj, np.float32)
    vb = _c(vb, np.uint64)
    cols = _c(built.colors if colors is None else colors, np.uint32)
    acc = np.zeros(2 * w * h, np.uint64)
    ids = None if batch_ids is None else _c(batch_ids, np.uint64)
    nd = getattr(built, "nodes", None)
    _lib_().or_accumulate(_p(built.batches), _p(nd), built.batches.shape[0], _p(ids), 0 if ids is None else ids.shape[0],
                          _p(built.low), _p(built.med), _p(built.high), _p(cols), _p(view), _p(proj), w, h,
                          ctypes.byref(o), float(np.float32(window)), _p(vb), _p(acc))
    return acc


def resolve_hqs(acc, clear_rgba: int = 0):
    """The averaged colour per pixel (rounded to nearest, alpha 255), clear_rgba where no point joined."""
    acc = _c(acc, np.uint64)
    fb = np.empty(acc.shape[0] // 2, np.uint32)
    _lib_().or_resolve_hqs(_p(acc), fb.shape[0], clear_rgba, _p(fb))
    return fb

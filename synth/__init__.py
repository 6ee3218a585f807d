"""Seeded synthetic inputs: point clouds and cameras.

Shared by the CPU oracle (test infrastructure) and the GPU path; it holds none
of the rasterizer's arithmetic.  The point generators live in ``synth.c``
(SplitMix64 counter-based, so point i is a pure function of (seed, i)); the
camera helpers build textbook OpenGL view/projection matrices in float64 and
hand them over as float32, row-major storage, column-vector convention
(clip = proj @ view @ [x, y, z, 1]).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile synth.c into libsynth.so next to it (gcc, host only)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
               "-fno-fast-math", "-o", _SO + ".tmp", os.path.join(_HERE, "synth.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        lib.synth_primitives.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.synth_primitives.restype = ctypes.c_int
        lib.synth_terrain.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.synth_terrain.restype = ctypes.c_int
        lib.synth_terrain_range.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                            ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.synth_terrain_range.restype = ctypes.c_int
        lib.synth_terrain_gather.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64,
                                             ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.synth_terrain_gather.restype = ctypes.c_int
        lib.synth_lpc_layout.argtypes = [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
        lib.synth_lpc_layout.restype = ctypes.c_int
        lib.synth_terrain_height.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_double]
        lib.synth_terrain_height.restype = ctypes.c_double
        _lib = lib
    return _lib


def _alloc(n: int, out=None):
    if out is None:
        xyz = np.empty((n, 3), dtype=np.float32)
        rgba = np.empty(n, dtype=np.uint32)
    else:
        xyz, rgba = out
        assert xyz.dtype == np.float32 and xyz.shape == (n, 3) and xyz.flags.c_contiguous
        assert rgba.dtype == np.uint32 and rgba.shape == (n,) and rgba.flags.c_contiguous
    return xyz, rgba


def primitives(seed: int, n: int, sigma: float = 0.01, threads: int = 0, out=None):
    """8 random planes/spheres in [0,100]^3 m plus N(0, sigma) noise; primitive-major order."""
    xyz, rgba = _alloc(n, out)
    rc = _load().synth_primitives(seed, n, sigma, xyz.ctypes.data, rgba.ctypes.data, threads)
    if rc != 0:
        raise RuntimeError(f"synth_primitives failed ({rc})")
    return xyz, rgba


def terrain(seed: int, n: int, sigma: float = 0.01, order: int = 1, threads: int = 0, out=None):
    """1 km^2 fBm terrain with buildings and poles; order 1 = serpentine 10 m tiles."""
    xyz, rgba = _alloc(n, out)
    rc = _load().synth_terrain(seed, n, sigma, order, xyz.ctypes.data, rgba.ctypes.data, threads)
    if rc != 0:
        raise RuntimeError(f"synth_terrain failed ({rc})")
    return xyz, rgba


def terrain_range(seed: int, n: int, lo: int, hi: int, xyz_ptr: int, rgba_ptr: int, sigma: float = 0.01,
                  threads: int = 0) -> None:
    """Points [lo, hi) of the index-order terrain of n points into raw host buffers
    (float32[hi-lo][3] at xyz_ptr, uint32[hi-lo] at rgba_ptr)."""
    rc = _load().synth_terrain_range(seed, n, lo, hi, sigma, xyz_ptr, rgba_ptr, threads)
    if rc != 0:
        raise RuntimeError(f"synth_terrain_range failed ({rc})")


def terrain_gather(seed: int, n: int, idx, sigma: float = 0.01, threads: int = 0):
    """Points idx[j] (uint32, each < n) of the index-order terrain of n points, in the order of idx."""
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    xyz = np.empty((idx.shape[0], 3), dtype=np.float32)
    rgba = np.empty(idx.shape[0], dtype=np.uint32)
    rc = _load().synth_terrain_gather(seed, n, idx.ctypes.data, idx.shape[0], sigma, xyz.ctypes.data,
                                      rgba.ctypes.data, threads)
    if rc != 0:
        raise RuntimeError(f"synth_terrain_gather failed ({rc})")
    return xyz, rgba


def terrain_height(seed: int, x: float, y: float) -> float:
    return float(_load().synth_terrain_height(seed, x, y))


# ------------------------------------------------------------------ cameras
def look_at(eye, target, up) -> np.ndarray:
    """gluLookAt: world -> eye space, camera looks down -z, float64 4x4 (column vectors)."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    s = np.cross(f, np.asarray(up, dtype=np.float64))
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    m = np.eye(4)
    m[0, :3], m[1, :3], m[2, :3] = s, u, -f
    m[0, 3], m[1, 3], m[2, 3] = -s @ eye, -u @ eye, f @ eye
    return m


def perspective(fovy_deg: float, aspect: float, near: float, far: float) -> np.ndarray:
    """gluPerspective: OpenGL clip space, w_clip = -z_eye."""
    f = 1.0 / math.tan(math.radians(fovy_deg) / 2.0)
    m = np.zeros((4, 4))
    m[0, 0] = f / aspect
    m[1, 1] = f
    m[2, 2] = (far + near) / (near - far)
    m[2, 3] = 2.0 * far * near / (near - far)
    m[3, 2] = -1.0
    return m


@dataclass
class Camera:
    view: np.ndarray  # float32 (4,4) row-major storage, column vectors
    proj: np.ndarray  # float32 (4,4)
    width: int
    height: int


def camera(eye, target, up, fovy, width, height, near, far) -> Camera:
    v = look_at(eye, target, up).astype(np.float32)
    p = perspective(fovy, width / height, near, far).astype(np.float32)
    return Camera(np.ascontiguousarray(v), np.ascontiguousarray(p), int(width), int(height))


# ---------------------------------------------------------- named workloads
C1_SEED = 1
C2_SEED = 2
C3_SEED = 3


def c1_camera() -> Camera:
    """8 primitives in the 100 m cube, 1280x720, fixed camera."""
    return camera((50.0, -90.0, 120.0), (50.0, 50.0, 50.0), (0.0, 0.0, 1.0), 60.0, 1280, 720, 0.5, 1000.0)


def orbit_camera(frame: int, frames: int = 60, width: int = 1920, height: int = 1080) -> Camera:
    """60-frame orbit around the terrain centre, 800 m radius, 450 m altitude."""
    th = 2.0 * math.pi * frame / frames
    eye = (500.0 + 800.0 * math.cos(th), 500.0 + 800.0 * math.sin(th), 450.0)
    return camera(eye, (500.0, 500.0, 0.0), (0.0, 0.0, 1.0), 60.0, width, height, 0.5, 5000.0)


def stereo_cameras(seed: int = C3_SEED, width: int = 2016, height: int = 2240):
    """Stereo pair 30 m above the ground at the terrain centre, looking +x, pitch -15 deg,
    fovy 100 deg per eye, eyes +-0.032 m along the camera's right axis, near 0.05, far 3000."""
    ground = terrain_height(seed, 500.0, 500.0)
    mid = np.array([500.0, 500.0, ground + 30.0])
    pitch = math.radians(-15.0)
    fwd = np.array([math.cos(pitch), 0.0, math.sin(pitch)])
    right = np.array([0.0, -1.0, 0.0])  # looking +x with +z up: right is -y
    cams = []
    for s in (-1.0, 1.0):
        eye = mid + s * 0.032 * right
        cams.append(camera(eye, eye + fwd, (0.0, 0.0, 1.0), 100.0, width, height, 0.05, 3000.0))
    return cams


def random_camera(rng: np.random.Generator, width: int, height: int, inside: bool = False,
                  box=((0.0, 0.0, 0.0), (100.0, 100.0, 100.0))) -> Camera:
    """A random perspective camera aimed into an axis-aligned box (for tests)."""
    lo, hi = np.asarray(box[0], float), np.asarray(box[1], float)
    c = (lo + hi) / 2
    ext = float(np.max(hi - lo))
    if inside:
        eye = lo + (hi - lo) * rng.uniform(0.2, 0.8, 3)
    else:
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        eye = c + d * ext * rng.uniform(0.8, 2.0)
    target = c + (hi - lo) * rng.uniform(-0.3, 0.3, 3)
    if np.linalg.norm(target - eye) < 1e-3:
        target = eye + np.array([1.0, 0.0, 0.0])
    up = (0.0, 0.0, 1.0) if abs((target - eye)[2]) < 0.95 * np.linalg.norm(target - eye) else (0.0, 1.0, 0.0)
    fovy = float(rng.uniform(30.0, 100.0))
    return camera(eye, target, up, fovy, width, height, 0.1, 10.0 * ext)


# ------------------------------------------------------------- served mode
# Resident clouds of the served workload: (terrain seed, points).
SERVED_CLOUDS = [(1, 10_000_000), (2, 50_000_000), (3, 100_000_000), (4, 250_000_000), (5, 500_000_000),
                 (6, 500_000_000), (7, 1_000_000_000), (8, 1_000_000_000)]
SERVED_SIZES = [(640, 480), (1920, 1080), (3840, 2160)]


def served_camera(rng: np.random.Generator, seed: int, width: int, height: int) -> Camera:
    """A camera over the terrain of `seed`: uniform (x, y) in [0, 1000]^2, altitude U(20, 400) m above the ground
    there, yaw U(0, 2 pi), pitch U(-60, -10) deg, fovy 60 deg, near 0.5, far 5000."""
    x, y = rng.uniform(0.0, 1000.0, 2)
    alt = rng.uniform(20.0, 400.0)
    yaw = rng.uniform(0.0, 2.0 * math.pi)
    pitch = math.radians(rng.uniform(-60.0, -10.0))
    eye = np.array([x, y, terrain_height(seed, float(x), float(y)) + alt])
    fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    return camera(eye, eye + fwd, (0.0, 0.0, 1.0), 60.0, width, height, 0.5, 5000.0)


def camera_array(seed: int, n: int = 64, width: int = 1024, height: int = 1024, rng_seed: int = 64):
    """n cameras over the terrain of `seed`, each drawn as served_camera (the multi-view workload's camera array)."""
    rng = np.random.default_rng(rng_seed)
    return [served_camera(rng, seed, width, height) for _ in range(n)]


def request_stream(seed: int, n: int, rate: float, cloud_seeds, sizes=SERVED_SIZES):
    """n requests of a Poisson stream at `rate` per second: (arrival s, cloud index, Camera), in arrival order;
    uniform cloud and image size, camera by served_camera over that cloud's terrain."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
    out = []
    for i in range(n):
        c = int(rng.integers(len(cloud_seeds)))
        w, h = sizes[int(rng.integers(len(sizes)))]
        out.append((float(arrivals[i]), c, served_camera(rng, cloud_seeds[c], w, h)))
    return out


# ------------------------------------------------------------ LOD input
def lpc_depth(n: int, cap: int = 10240) -> int:
    """Deepest level so that the last level's nodes (3/4 of the points, 4^depth nodes on a surface) hold about cap."""
    d = 0
    while d < 15 and 0.75 * n / (4 ** d) > cap:
        d += 1
    return d


def lpc_layout(seed: int, xyz, rgba, depth: int, cap: int = 10240, spread: bool = True):
    """Layered-point-cloud layout (see synth_lpc_layout): (xyz_out, rgba_out, spans uint32 (nb, 2) = first, count,
    nodes float64 (nb, 5) = cube origin x, y, z, edge, level).  Padding slots between batches are zero.  spread: each
    batch's points in the spread order (slot t holds the batch's point of rank (t * m) mod count in the (level,
    Morton) order, m the first integer > count / 4 coprime with count), else in that order itself."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    rgba = np.ascontiguousarray(rgba, dtype=np.uint32)
    n = xyz.shape[0]
    npad, nb = ctypes.c_uint64(), ctypes.c_uint64()
    cap_b = n // max(1, cap // 4) + 2 * 4 ** min(depth, 10) + 16
    cap_p = n + 3 * cap_b
    for _ in range(2):
        xo = np.zeros((cap_p, 3), np.float32)
        ro = np.zeros(cap_p, np.uint32)
        spans = np.zeros((cap_b, 2), np.uint32)
        nodes = np.zeros((cap_b, 5), np.float64)
        rc = _load().synth_lpc_layout(seed, xyz.ctypes.data, rgba.ctypes.data, n, depth, cap, int(spread), xo.ctypes.data,
                                      ro.ctypes.data, cap_p, spans.ctypes.data, nodes.ctypes.data, cap_b,
                                      ctypes.byref(npad), ctypes.byref(nb))
        if rc == 0:
            return xo[:npad.value].copy(), ro[:npad.value].copy(), spans[:nb.value].copy(), nodes[:nb.value].copy()
        if rc != -3:
            raise RuntimeError(f"synth_lpc_layout failed ({rc})")
        cap_b, cap_p = nb.value, npad.value
    raise RuntimeError("synth_lpc_layout: capacity")

"""ctypes marshalling for libptraster.so (see include/ptraster.h for semantics)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptraster.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python {os.path.join(_HERE, 'build.py')}` "
        "(there is no fallback implementation)")

# PyTorch ships its own HIP runtime (libamdhip64, soname libamdhip64.so.7, which
# its libraries load by the unversioned file name).  Loaded first, it also
# serves the library's libamdhip64.so.7 dependency, so the process has one HIP
# runtime.  Loading the library first would bring in the system runtime and
# leave torch to load a second one, and the second runtime to initialise finds
# no device.
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

PR_ADAPTIVE, PR_FORCE10, PR_FORCE20, PR_FORCE30 = 0, 10, 20, 30
PR_ORDER_INPUT, PR_ORDER_MORTON, PR_ORDER_MORTON_SPREAD = 0, 1, 2  # point orders of pr_build_batches
PR_EMPTY = 0xFFFFFFFFFFFFFFFF
PR_MAX_VIEWS = 64
_STATUS = {0: "PR_OK", -1: "PR_EINVAL", -2: "PR_ENOMEM", -3: "PR_EDEVICE", -4: "PR_ESTATE",
           -5: "PR_ENONFINITE", -6: "PR_ERANGE"}

EXPORTED = ["pr_last_error", "pr_create", "pr_destroy", "pr_cloud_sizes", "pr_load_points", "pr_build_batches",
            "pr_clear", "pr_render", "pr_resolve", "pr_get_stats", "pr_sync", "pr_cloud_info", "pr_cloud_free",
            "pr_views_work_bytes", "pr_render_views", "pr_cloud_drop_load_buffers", "pr_render_hqs",
            "pr_cloud_sizes_spans", "pr_build_batches_spans", "pr_raster_shapes", "pr_set_tuning", "pr_get_tuning",
            "pr_autotune", "pr_stream_probe", "pr_render_views_static", "pr_time_kernels", "pr_kernel_times"]


class PrError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        self.name = _STATUS.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {pr_last_error()}")


BUFFER_FIELDS = ("xyz", "rgba", "low", "med", "high", "colors", "perm", "batches", "scratch", "nodes")


class Sizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in BUFFER_FIELDS]


class CloudBufs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in BUFFER_FIELDS] + [("capacity", Sizes)]


class LodNode(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("edge", ctypes.c_double), ("level", ctypes.c_uint32),
                ("pad", ctypes.c_uint32 * 3)]


class RenderOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("cull", ctypes.c_int32), ("t10", ctypes.c_float),
                ("t20", ctypes.c_float), ("counters", ctypes.c_int32), ("accumulate", ctypes.c_int32),
                ("lod_px", ctypes.c_float)]

    @classmethod
    def make(cls, precision=PR_ADAPTIVE, cull=1, t10=500.0, t20=512000.0, counters=0, accumulate=0, lod_px=0.0):
        return cls(precision, cull, t10, t20, counters, accumulate, lod_px)


class View(ctypes.Structure):
    _fields_ = [("view", ctypes.c_float * 16), ("proj", ctypes.c_float * 16), ("w", ctypes.c_uint32),
                ("h", ctypes.c_uint32), ("visbuf", ctypes.c_void_p)]


class RasterShape(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_uint32), ("depth", ctypes.c_uint32), ("tile_px", ctypes.c_uint32),
                ("max_wg_per_cu", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_uint32), ("tile_px", ctypes.c_uint32), ("wg_per_cu", ctypes.c_uint32),
                ("max_bands", ctypes.c_uint32)]

    def as_dict(self):
        return {"shape": self.shape, "tile_px": self.tile_px, "wg_per_cu": self.wg_per_cu, "max_bands": self.max_bands}


class TuneTrial(ctypes.Structure):
    _fields_ = [("tuning", Tuning), ("ms", ctypes.c_float), ("reserved", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("culled", ctypes.c_uint64), ("points", ctypes.c_uint64),
                ("level_batches", ctypes.c_uint64 * 3), ("level_points", ctypes.c_uint64 * 3),
                ("atomics", ctypes.c_uint64), ("words_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {"batches": self.batches, "culled": self.culled, "points": self.points,
                "level_batches": list(self.level_batches), "level_points": list(self.level_points),
                "atomics": self.atomics, "words_bytes": self.words_bytes}


_P, _U64, _U32, _I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
lib.pr_last_error.restype = ctypes.c_char_p
lib.pr_last_error.argtypes = []
lib.pr_create.argtypes = [_I, _P, ctypes.POINTER(_P)]
lib.pr_destroy.argtypes = [_P]
lib.pr_destroy.restype = None
lib.pr_cloud_sizes.argtypes = [_U64, _U32, _I, ctypes.POINTER(Sizes)]
lib.pr_load_points.argtypes = [_P, _P, _P, _U64, _I, ctypes.POINTER(CloudBufs), ctypes.POINTER(_P)]
lib.pr_build_batches.argtypes = [_P, _P, _U32, _I]
lib.pr_clear.argtypes = [_P, _P, _U32, _U32]
lib.pr_render.argtypes = [_P, _P, _P, _P, _U32, _U32, ctypes.POINTER(RenderOpts), _P]
lib.pr_resolve.argtypes = [_P, _P, _P, _U32, _U32, _U32, _P]
lib.pr_get_stats.argtypes = [_P, ctypes.POINTER(Stats)]
lib.pr_views_work_bytes.argtypes = [_P, _U32, ctypes.POINTER(_U64)]
lib.pr_cloud_drop_load_buffers.argtypes = [_P]
lib.pr_cloud_sizes_spans.argtypes = [_U64, _U64, ctypes.POINTER(Sizes)]
lib.pr_build_batches_spans.argtypes = [_P, _P, _P, _P, _U64]
lib.pr_render_hqs.argtypes = [_P, _P, _P, _P, _U32, _U32, ctypes.POINTER(RenderOpts), ctypes.c_float, _P, _P, _U32, _P]
lib.pr_render_views.argtypes = [_P, _P, ctypes.POINTER(View), _U32, ctypes.POINTER(RenderOpts), _P, _U64]
lib.pr_render_views_static.argtypes = [_P, _P, ctypes.POINTER(View), _U32, ctypes.POINTER(RenderOpts)]
lib.pr_sync.argtypes = [_P]
lib.pr_raster_shapes.argtypes = [_P, ctypes.POINTER(RasterShape), _U32, ctypes.POINTER(_U32)]
lib.pr_stream_probe.argtypes = [_P, _P, _P, _U64]
lib.pr_set_tuning.argtypes = [_P, ctypes.POINTER(Tuning)]
lib.pr_get_tuning.argtypes = [_P, ctypes.POINTER(Tuning)]
lib.pr_autotune.argtypes = [_P, _P, ctypes.POINTER(View), _U32, ctypes.POINTER(RenderOpts), _P, _U64, _U32,
                            ctypes.POINTER(TuneTrial), _U32, ctypes.POINTER(_U32), ctypes.POINTER(Tuning)]
lib.pr_cloud_info.argtypes = [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64), ctypes.POINTER(_U32)]
lib.pr_time_kernels.argtypes = [_P, _U32]
lib.pr_kernel_times.argtypes = [_P, ctypes.POINTER(ctypes.c_float), _U32, ctypes.POINTER(_U32)]
lib.pr_cloud_free.argtypes = [_P]
lib.pr_cloud_free.restype = None
for _f in ("pr_create", "pr_cloud_sizes", "pr_load_points", "pr_build_batches", "pr_clear", "pr_render", "pr_resolve",
           "pr_get_stats", "pr_sync", "pr_cloud_info", "pr_views_work_bytes", "pr_render_views",
           "pr_cloud_drop_load_buffers", "pr_render_hqs", "pr_cloud_sizes_spans", "pr_build_batches_spans",
           "pr_raster_shapes", "pr_set_tuning", "pr_get_tuning", "pr_autotune", "pr_stream_probe",
           "pr_time_kernels", "pr_kernel_times"):
    getattr(lib, _f).restype = ctypes.c_int


def _check(status: int, where: str):
    if status != 0:
        raise PrError(status, where)


def _ptr(x):
    """Device/host address of a torch tensor or numpy array (or an int / None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _mat16(m):
    a = np.ascontiguousarray(np.asarray(m, dtype=np.float32).reshape(16))
    return a, a.ctypes.data


def pr_last_error() -> str:
    return lib.pr_last_error().decode()


def pr_create(device: int = 0, stream=None):
    """Returns an opaque context handle (int).  stream: a hipStream_t as int, or a torch stream."""
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    h = _P()
    _check(lib.pr_create(device, stream, ctypes.byref(h)), "pr_create")
    return h.value


def pr_destroy(ctx):
    lib.pr_destroy(ctx)


def pr_cloud_sizes(n: int, batch_size: int, morton: int) -> Sizes:
    s = Sizes()
    _check(lib.pr_cloud_sizes(n, batch_size, int(morton), ctypes.byref(s)), "pr_cloud_sizes")
    return s


def pr_load_points(ctx, xyz, rgba, n: int, src_on_device: bool, bufs: CloudBufs):
    h = _P()
    _check(lib.pr_load_points(ctx, _ptr(xyz), _ptr(rgba), n, int(src_on_device), ctypes.byref(bufs), ctypes.byref(h)),
           "pr_load_points")
    return h.value


def pr_build_batches(ctx, cloud, batch_size: int, morton: int):
    """morton: PR_ORDER_INPUT (0 / False), PR_ORDER_MORTON (1 / True) or PR_ORDER_MORTON_SPREAD (2)."""
    _check(lib.pr_build_batches(ctx, cloud, batch_size, int(morton)), "pr_build_batches")


def pr_clear(ctx, visbuf, w: int, h: int):
    _check(lib.pr_clear(ctx, _ptr(visbuf), w, h), "pr_clear")


def pr_render(ctx, cloud, view, proj, w: int, h: int, opts: RenderOpts | None, visbuf):
    v, vp = _mat16(view)
    p, pp = _mat16(proj)
    _check(lib.pr_render(ctx, cloud, vp, pp, w, h, ctypes.byref(opts) if opts is not None else None, _ptr(visbuf)),
           "pr_render")


def pr_cloud_sizes_spans(n: int, nb: int) -> Sizes:
    s = Sizes()
    _check(lib.pr_cloud_sizes_spans(n, nb, ctypes.byref(s)), "pr_cloud_sizes_spans")
    return s


def lod_nodes(nodes) -> ctypes.Array:
    """LodNode array from a float64 (nb, 5) table: cube origin x, y, z, edge, level."""
    nodes = np.asarray(nodes, dtype=np.float64)
    arr = (LodNode * len(nodes))()
    for i, row in enumerate(nodes):
        arr[i].origin[:] = [float(row[0]), float(row[1]), float(row[2])]
        arr[i].edge = float(row[3])
        arr[i].level = int(row[4])
    return arr


def pr_build_batches_spans(ctx, cloud, spans, nodes=None):
    """spans: uint32 (nb, 2) = first, count; nodes: float64 (nb, 5) or None."""
    sp = np.ascontiguousarray(np.asarray(spans, dtype=np.uint32).reshape(-1, 2))
    nd = lod_nodes(nodes) if nodes is not None else None
    _check(lib.pr_build_batches_spans(ctx, cloud, sp.ctypes.data if len(sp) else None,
                                      ctypes.cast(nd, ctypes.c_void_p) if nd is not None else None, len(sp)),
           "pr_build_batches_spans")


def pr_cloud_drop_load_buffers(cloud):
    _check(lib.pr_cloud_drop_load_buffers(cloud), "pr_cloud_drop_load_buffers")


def pr_views_work_bytes(cloud, nviews: int) -> int:
    out = _U64()
    _check(lib.pr_views_work_bytes(cloud, nviews, ctypes.byref(out)), "pr_views_work_bytes")
    return out.value


def _views(views):
    arr = (View * len(views))()
    for i, (v, p, w, h, vb) in enumerate(views):
        arr[i].view[:] = [float(x) for x in np.asarray(v, dtype=np.float32).reshape(16)]
        arr[i].proj[:] = [float(x) for x in np.asarray(p, dtype=np.float32).reshape(16)]
        arr[i].w, arr[i].h, arr[i].visbuf = w, h, _ptr(vb)
    return arr


def pr_render_views(ctx, cloud, views, opts: RenderOpts | None, work, work_bytes: int):
    """views: sequence of (view, proj, w, h, visbuf); work: device buffer of pr_views_work_bytes bytes."""
    _check(lib.pr_render_views(ctx, cloud, _views(views), len(views),
                               ctypes.byref(opts) if opts is not None else None, _ptr(work), work_bytes),
           "pr_render_views")


def pr_render_views_static(ctx, cloud, views, opts: RenderOpts | None):
    """views: sequence of (view, proj, w, h, visbuf); the work area is the library's static one."""
    _check(lib.pr_render_views_static(ctx, cloud, _views(views), len(views),
                                      ctypes.byref(opts) if opts is not None else None),
           "pr_render_views_static")


PR_STATIC_WORK_BYTES = 64 << 20


def pr_stream_probe(ctx, src, dst, nbytes: int):
    """HBM streaming reference: copy src -> dst (or, dst None, read src only), nbytes a multiple of 16."""
    _check(lib.pr_stream_probe(ctx, _ptr(src), _ptr(dst), nbytes), "pr_stream_probe")


def pr_raster_shapes(ctx) -> list:
    """The compiled workgroup shapes, as dicts (waves, depth, tile_px, max_wg_per_cu); index 0 is the default."""
    n = _U32()
    _check(lib.pr_raster_shapes(ctx, None, 0, ctypes.byref(n)), "pr_raster_shapes")
    arr = (RasterShape * n.value)()
    _check(lib.pr_raster_shapes(ctx, arr, n.value, ctypes.byref(n)), "pr_raster_shapes")
    return [a.as_dict() for a in arr]


def pr_set_tuning(ctx, shape: int = 0, tile_px: int = 0, wg_per_cu: int = 0, max_bands: int = 0):
    t = Tuning(shape, tile_px, wg_per_cu, max_bands)
    _check(lib.pr_set_tuning(ctx, ctypes.byref(t)), "pr_set_tuning")


def pr_get_tuning(ctx) -> dict:
    t = Tuning()
    _check(lib.pr_get_tuning(ctx, ctypes.byref(t)), "pr_get_tuning")
    return t.as_dict()


def pr_autotune(ctx, cloud, views, opts: RenderOpts | None, work, work_bytes: int, reps: int = 3):
    """Times every candidate tuning on pr_render_views(views) and keeps the fastest on ctx.
    Returns (best tuning dict, [(tuning dict, ms), ...] in candidate order)."""
    arr = _views(views)
    n = _U32()
    cap = 256
    trials = (TuneTrial * cap)()
    best = Tuning()
    _check(lib.pr_autotune(ctx, cloud, arr, len(views), ctypes.byref(opts) if opts is not None else None, _ptr(work),
                           work_bytes, reps, trials, cap, ctypes.byref(n), ctypes.byref(best)), "pr_autotune")
    return best.as_dict(), [(trials[i].tuning.as_dict(), float(trials[i].ms)) for i in range(min(n.value, cap))]


def pr_render_hqs(ctx, cloud, view, proj, w: int, h: int, opts: RenderOpts | None, window: float, visbuf, accum,
                  clear_rgba: int, rgba_out):
    v, vp = _mat16(view)
    p, pp = _mat16(proj)
    _check(lib.pr_render_hqs(ctx, cloud, vp, pp, w, h, ctypes.byref(opts) if opts is not None else None, window,
                             _ptr(visbuf), _ptr(accum), clear_rgba & 0xFFFFFFFF, _ptr(rgba_out)), "pr_render_hqs")


def pr_resolve(ctx, cloud, visbuf, w: int, h: int, clear_rgba: int, rgba_out):
    _check(lib.pr_resolve(ctx, cloud, _ptr(visbuf), w, h, clear_rgba & 0xFFFFFFFF, _ptr(rgba_out)), "pr_resolve")


def pr_get_stats(ctx) -> dict:
    s = Stats()
    _check(lib.pr_get_stats(ctx, ctypes.byref(s)), "pr_get_stats")
    return s.as_dict()


def pr_sync(ctx):
    _check(lib.pr_sync(ctx), "pr_sync")


PR_MAX_TIMED_LAUNCHES = 4096


def pr_time_kernels(ctx, n: int):
    """Arm event pairs around the next n render-kernel launches of the context (0: off)."""
    _check(lib.pr_time_kernels(ctx, int(n)), "pr_time_kernels")


def pr_kernel_times(ctx, capacity: int = PR_MAX_TIMED_LAUNCHES) -> list:
    """Durations (ms) of the render-kernel launches recorded since pr_time_kernels, in launch order."""
    buf = (ctypes.c_float * max(int(capacity), 1))()
    cnt = _U32()
    _check(lib.pr_kernel_times(ctx, buf, int(capacity), ctypes.byref(cnt)), "pr_kernel_times")
    return [float(buf[i]) for i in range(cnt.value)]


def pr_cloud_info(cloud):
    n, nb, bs = _U64(), _U64(), _U32()
    _check(lib.pr_cloud_info(cloud, ctypes.byref(n), ctypes.byref(nb), ctypes.byref(bs)), "pr_cloud_info")
    return n.value, nb.value, bs.value


def pr_cloud_free(cloud):
    lib.pr_cloud_free(cloud)


# ------------------------------------------------- torch-owned memory plumbing
class Context:
    """A pr_ctx bound to a torch device and stream (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.handle = pr_create(device, self.stream.cuda_stream)

    def close(self):
        if self.handle:
            pr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceCloud:
    """Cloud buffers allocated as torch tensors (sized by pr_cloud_sizes), loaded and built."""

    FIELDS = BUFFER_FIELDS

    def __init__(self, ctx: Context, xyz, rgba, batch_size: int = 10240, morton: int = PR_ORDER_INPUT, spans=None,
                 nodes=None):
        """Fixed-size batches of batch_size points in one of the PR_ORDER_* orders (False / True for input / Morton
        order), or, with spans (uint32 (nb, 2) =
        first, count), the variable-size batches of a level-of-detail layout with optional nodes (float64 (nb, 5))."""
        import torch

        n = int(xyz.shape[0])
        self.ctx, self.n, self.batch_size, self.morton = ctx, n, batch_size, morton
        if spans is not None:
            spans = np.ascontiguousarray(np.asarray(spans, dtype=np.uint32).reshape(-1, 2))
            self.sizes = pr_cloud_sizes_spans(n, len(spans))
        else:
            self.sizes = pr_cloud_sizes(n, batch_size, morton)
        dev = torch.device("cuda", ctx.device)
        self.mem = {f: torch.empty(max(getattr(self.sizes, f), 256), dtype=torch.uint8, device=dev)
                    for f in self.FIELDS}
        self.bufs = CloudBufs(*[self.mem[f].data_ptr() for f in self.FIELDS], self.sizes)
        on_dev = hasattr(xyz, "is_cuda") and xyz.is_cuda
        if not on_dev:
            xyz = np.ascontiguousarray(xyz, dtype=np.float32)
            rgba = np.ascontiguousarray(rgba, dtype=np.uint32)
        self._src = (xyz, rgba)  # keep host sources alive until the copies are done
        self.handle = pr_load_points(ctx.handle, xyz, rgba, n, on_dev, self.bufs)
        if spans is not None:
            pr_build_batches_spans(ctx.handle, self.handle, spans, nodes)
        else:
            pr_build_batches(ctx.handle, self.handle, batch_size, morton)
        self._src = None
        self.nb = pr_cloud_info(self.handle)[1]

    def drop_load_buffers(self):
        """Keep only what rendering reads; frees positions, input colours, permutation and scratch.  Waits for
        the context's stream first: a pr_render enqueued there may still use the scratch buffer, and the caching
        allocator may hand the freed memory to work on another stream at once."""
        pr_cloud_drop_load_buffers(self.handle)
        pr_sync(self.ctx.handle)
        for f in ("xyz", "rgba", "perm", "scratch"):
            self.mem[f] = None

    def view(self, field: str, dtype, count: int):
        """A typed torch view of one buffer (e.g. view('low', torch.int32, n))."""
        import torch

        t = self.mem[field]
        esize = torch.empty(0, dtype=dtype).element_size()
        return t[: count * esize].view(dtype)

    def close(self):
        if self.handle:
            pr_cloud_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

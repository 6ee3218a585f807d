"""MI355X point rasterizer -- Python binding of libptraster.so.

Brute-force compute rasterization of one-pixel points into a 64-bit
visibility buffer (Schuetz, Kerbl & Wimmer, "Software Rasterization of 2
Billion Points in Real Time", Sec. 3).  Every step runs in the HIP kernels of
``libptraster.so`` (gfx950); this module only marshals arguments through the
C ABI of ``include/ptraster.h`` with the same function names.  PyTorch is used
for device memory and streams.

Importing fails loudly if the library has not been built
(``python paper_2204_01287_amd/build.py`` or ``__graft_entry__.build()``).
"""
from ._binding import (  # noqa: F401
    PR_ADAPTIVE, PR_EMPTY, PR_FORCE10, PR_FORCE20, PR_FORCE30, PR_MAX_VIEWS, PR_ORDER_INPUT, PR_ORDER_MORTON,
    PR_ORDER_MORTON_SPREAD, PrError, Sizes, CloudBufs, RenderOpts,
    Stats, View, pr_views_work_bytes, pr_render_views, pr_cloud_drop_load_buffers, pr_render_hqs, pr_cloud_sizes_spans,
    pr_build_batches_spans, LodNode, lod_nodes, BUFFER_FIELDS, RasterShape, Tuning, TuneTrial, pr_raster_shapes,
    pr_set_tuning, pr_get_tuning, pr_autotune, pr_stream_probe, pr_render_views_static, PR_STATIC_WORK_BYTES,
    LIB_PATH, lib, pr_last_error, pr_create, pr_destroy, pr_cloud_sizes, pr_load_points, pr_build_batches,
    pr_clear, pr_render, pr_resolve, pr_get_stats, pr_sync, pr_cloud_info, pr_cloud_free, EXPORTED,
    pr_time_kernels, pr_kernel_times, PR_MAX_TIMED_LAUNCHES,
    DeviceCloud, Context,
)

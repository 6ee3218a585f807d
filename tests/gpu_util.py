"""Helpers shared by the GPU tests: run the HIP path and the oracle on the same inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle

MODES = {
    "adaptive": dict(precision=0),
    "force10": dict(precision=10),
    "force20": dict(precision=20),
    "force30": dict(precision=30),
    "adaptive_nocull": dict(precision=0, cull=0),
}


def say(msg: str):
    """Name the case before each GPU step (flushed, so it survives a lost box)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch

    return torch.device("cuda", 0)


def gpu_build(ctx, xyz, rgba, S, morton):
    import paper_2204_01287_amd as pr

    return pr.DeviceCloud(ctx, xyz, rgba, batch_size=S, morton=morton)


def gpu_build_outputs(dc):
    import torch

    n, nb = dc.n, dc.nb
    out = {}
    for f in ("low", "med", "high", "colors", "perm"):
        out[f] = dc.view(f, torch.int32, n).cpu().numpy().view(np.uint32)
    out["xyz"] = dc.view("xyz", torch.float32, 3 * n).cpu().numpy().reshape(n, 3)
    out["batches"] = dc.view("batches", torch.uint8, 32 * nb).cpu().numpy().view(oracle.BATCH_DTYPE)
    return out


def gpu_render(ctx, dc, view, proj, w, h, precision=0, cull=1, counters=1, t10=500.0, t20=512000.0,
               clear_rgba=0, vb=None, fb=None, lod_px=0.0):
    import torch
    import paper_2204_01287_amd as pr

    if vb is None:
        vb = torch.empty(w * h, dtype=torch.int64, device=torch_dev())
    if fb is None:
        fb = torch.empty(w * h, dtype=torch.int32, device=torch_dev())
    opts = pr.RenderOpts.make(precision=precision, cull=cull, t10=t10, t20=t20, counters=counters, lod_px=lod_px)
    pr.pr_render(ctx.handle, dc.handle, view, proj, w, h, opts, vb)
    pr.pr_resolve(ctx.handle, dc.handle, vb, w, h, clear_rgba, fb)
    stats = pr.pr_get_stats(ctx.handle) if counters else None
    pr.pr_sync(ctx.handle)
    return vb.cpu().numpy().view(np.uint64), fb.cpu().numpy().view(np.uint32), stats


def assert_build_equal(g, B, check_xyz=True):
    for f in ("low", "med", "high", "colors", "perm"):
        a, b = g[f], getattr(B, f)
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{f}: {len(bad)} mismatches, first at {bad[:5]}: gpu {a[bad[:5]]} oracle {b[bad[:5]]}")
    gb, ob = g["batches"], B.batches
    assert gb.shape == ob.shape
    assert np.array_equal(gb.view(np.uint8), ob.view(np.uint8)), "batch records differ"
    if check_xyz:
        assert np.array_equal(g["xyz"].view(np.uint32), B.xyz.view(np.uint32)), "positions in render order differ"


def assert_vb_equal(vb_gpu, vb_ref, w):
    if np.array_equal(vb_gpu, vb_ref):
        return
    bad = np.nonzero(vb_gpu != vb_ref)[0]
    lines = [f"{len(bad)} of {len(vb_ref)} pixels differ"]
    for p in bad[:8]:
        lines.append(f"  pixel ({p % w},{p // w}): gpu {int(vb_gpu[p]):#018x} oracle {int(vb_ref[p]):#018x}")
    raise AssertionError("\n".join(lines))


def oracle_stats_match(st_gpu, st_ref):
    for k in ("batches", "culled", "points", "level_batches", "level_points"):
        assert st_gpu[k] == st_ref[k], (k, st_gpu[k], st_ref[k])

"""Autotuning of the render path over batch size, workgroup shape and grid.

The paper fixes one workgroup size and number of points per thread for its GPU
and reports a sweep of points per thread (Sec. 3.2).  Here the sweep is done
per device, cloud and set of views, in two levels:

  * the batch size S is fixed when a cloud is built, so ``tune`` rebuilds the
    caller's cloud once per candidate S (``build(S)`` returns a built
    DeviceCloud);
  * for each build, ``pr_autotune`` (C ABI) times every compiled workgroup
    shape (waves per workgroup, point groups in flight per wave, LDS tile) with
    its full and half tile bound and all or half of the workgroups that fit,
    on one multi-view frame of the given views, and keeps the fastest.

Points per thread follow as S / (64 * waves).  Every candidate computes the
same visibility buffers, bit for bit; only the time differs.
"""
from __future__ import annotations

from . import _binding as B


def tune(ctx, build, batch_sizes, cams, opts=None, reps: int = 3, log=None):
    """ctx: Context; build(S) -> a built DeviceCloud of the caller's points with batch size S; cams: up to
    PR_MAX_VIEWS objects with .view, .proj, .width, .height.

    Returns {"best": {"batch_size", "tuning", "ms"}, "trials": [{"batch_size", "tuning", "ms"}, ...]}.  The
    context keeps the winner's tuning; the caller builds its cloud with the winner's batch size."""
    import torch

    if not 1 <= len(cams) <= B.PR_MAX_VIEWS:
        raise ValueError("1..PR_MAX_VIEWS views")
    dev = torch.device("cuda", ctx.device)
    vbs = [torch.empty(c.width * c.height, dtype=torch.int64, device=dev) for c in cams]
    views = [(c.view, c.proj, c.width, c.height, vb) for c, vb in zip(cams, vbs)]
    trials, best = [], None
    for S in batch_sizes:
        dc = build(S)
        need = B.pr_views_work_bytes(dc.handle, len(cams))
        work = torch.empty(need, dtype=torch.uint8, device=dev)
        win, table = B.pr_autotune(ctx.handle, dc.handle, views, opts, work, need, reps)
        for t, ms in table:
            trials.append({"batch_size": S, "tuning": t, "ms": ms})
        ms = min(m for _, m in table)
        if log:
            log(f"autotune S={S}: best {win} {ms:.3f} ms over {len(table)} candidates")
        if best is None or ms < best["ms"]:
            best = {"batch_size": S, "tuning": win, "ms": ms}
        del work
        dc.close()
        del dc
        torch.cuda.empty_cache()
    B.pr_set_tuning(ctx.handle, **best["tuning"])
    return {"best": best, "trials": trials}

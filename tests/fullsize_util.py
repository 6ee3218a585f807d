"""Helpers of the full-size parity tests: device buffers as typed views, the threaded oracle frame, and the
chunked check of a device Morton build against the oracle."""
from __future__ import annotations

import time
import types
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
import synth
from gpu_util import say

S = 10240
CLEAR = 0xFF000000
CH = 64_000_000  # host chunk: 6250 whole batches
WORKERS = 4      # build-check workers, each generator call on 4 threads: 16 host threads
RENDER_WORKERS = 16


def _t():
    return time.perf_counter()


def _u32(t):
    """A torch int32 tensor (device) as a host numpy uint32 array."""
    return t.cpu().numpy().view(np.uint32)


def device_views(cloud, n, nb):
    """Typed torch views of a cloud loaded by bench.load_cloud."""
    import torch

    m = cloud["mem"]
    return types.SimpleNamespace(
        xyz=m["xyz"][: 12 * n].view(torch.int32), perm=m["perm"][: 4 * n].view(torch.int32),
        colors=m["colors"][: 4 * n].view(torch.int32), low=m["low"][: 4 * n].view(torch.int32),
        med=m["med"][: 4 * n].view(torch.int32), high=m["high"][: 4 * n].view(torch.int32),
        batches=m["batches"][: 32 * nb])


def oracle_frame(built, cam, nb, o=None):
    """The oracle over every batch, on worker threads (interleaved batch sets, private buffers, min-merge)."""
    groups = [np.arange(g, nb, 4 * RENDER_WORKERS, dtype=np.uint64) for g in range(min(nb, 4 * RENDER_WORKERS))]

    def job(ids):
        return oracle.render(built, cam.view, cam.proj, cam.width, cam.height, o, batch_ids=ids)

    vb, st = None, None
    with ThreadPoolExecutor(RENDER_WORKERS) as ex:
        for v, s in ex.map(job, groups):
            vb = v if vb is None else np.minimum(vb, v)
            if st is None:
                st = s
            else:
                for k in ("batches", "culled", "points"):
                    st[k] += s[k]
                for k in ("level_batches", "level_points"):
                    st[k] = [a + b for a, b in zip(st[k], s[k])]
    return vb, st


def check_morton_build(ns, tag):
    """Check the device's Morton build of the generator's index-order cloud against the oracle, chunk by chunk
    (permutation, order, stability, positions, colours, batch records, Eq. 1 words); keep the oracle's build."""
    import torch

    n, nb, seed = ns.n, ns.nb, ns.wl["seed"]
    v = device_views(ns.cloud, n, nb)
    t0 = _t()
    # 1. perm is a permutation of 0..n-1 (bounds first: an out-of-range index must not reach the GPU)
    say(f"{tag}: permutation check on the device")
    marks = torch.zeros(n, dtype=torch.uint8, device=v.perm.device)
    for lo in range(0, n, CH):
        idx = v.perm[lo:min(n, lo + CH)].to(torch.int64) & 0xFFFFFFFF
        assert int(idx.max()) < n, "perm holds an index >= n"
        marks[idx] = 1
    assert int(marks.min()) == 1, "perm is not a permutation"
    del marks, idx
    torch.cuda.synchronize()
    say(f"{tag}: permutation ok ({_t() - t0:.1f} s); chunked pass over the build")
    # 2. chunked pass: generator points in device order -> oracle codes, batches, words; compare
    cmin, cmax = ns.cloud_box
    built = types.SimpleNamespace(batches=np.empty(nb, oracle.BATCH_DTYPE), low=np.empty(n, np.uint32),
                                  med=np.empty(n, np.uint32), high=np.empty(n, np.uint32))
    colors = np.empty(n, np.uint32)
    gb_all = v.batches.cpu().numpy()

    spread = int(ns.wl["morton"]) == 2  # PR_ORDER_MORTON_SPREAD: every batch stored in the spread order

    def job(lo):
        hi = min(n, lo + CH)
        perm = _u32(v.perm[lo:hi])
        ox, oc = synth.terrain_gather(seed, n, perm, threads=4)
        # the Morton order: with the spread order, position r of a batch of c points holds its Morton rank
        # (r * m) mod c (the oracle's step m), so the ranks are put back first (chunks hold whole batches)
        mperm, mx = perm, ox
        if spread:
            mperm = np.empty_like(perm)
            mx = np.empty_like(ox)
            for b0 in range(0, hi - lo, S):
                c = min(S, hi - lo - b0)
                rank = (np.arange(c, dtype=np.uint64) * np.uint64(oracle.spread_multiplier(c))) % np.uint64(c)
                mperm[b0 + rank.astype(np.int64)] = perm[b0:b0 + c]
                mx[b0 + rank.astype(np.int64)] = ox[b0:b0 + c]
        codes = oracle.morton_codes(mx, cmin, cmax)
        tie = codes[1:] == codes[:-1]
        r = dict(lo=lo, mono=bool(np.all(codes[1:] >= codes[:-1])),
                 stable=bool(np.all(mperm[1:][tie] > mperm[:-1][tie])),
                 head=(int(codes[0]), int(mperm[0])), tail=(int(codes[-1]), int(mperm[-1])))
        r["xyz"] = bool(np.array_equal(_u32(v.xyz[3 * lo:3 * hi]), ox.view(np.uint32).reshape(-1)))
        r["colors"] = bool(np.array_equal(_u32(v.colors[lo:hi]), oc))
        ob = oracle.make_batches(ox, S)
        words = oracle.quantize(ox, ob)
        for f, w in zip(("low", "med", "high"), words):
            r[f] = bool(np.array_equal(_u32(getattr(v, f)[lo:hi]), w))
            getattr(built, f)[lo:hi] = w
        ob["first"] += np.uint32(lo)
        b0 = lo // S
        r["batches"] = bool(np.array_equal(gb_all[32 * b0:32 * (b0 + len(ob))], ob.view(np.uint8)))
        built.batches[b0:b0 + len(ob)] = ob
        colors[lo:hi] = oc
        return r

    with ThreadPoolExecutor(WORKERS) as ex:
        res = []
        for r in ex.map(job, range(0, n, CH)):
            res.append(r)
            if len(res) % 8 == 0:
                say(f"{tag}: {len(res)} chunks checked ({_t() - t0:.1f} s)")
    say(f"{tag}: chunked pass done ({_t() - t0:.1f} s)")
    return res, built, colors

"""Served-mode policy on the host alone: the Scheduler with an injected clock, fake launches and a fake budget.

The clock moves only when the scheduler has nothing to do (its idle callback), and a launched group completes
after a service time proportional to its pixels, so every run is deterministic.  Checked: every request completes
once and after it arrived; admission keeps the admitted bytes within the budget (one oversize request runs alone);
a group holds one cloud and at most max_group requests, launched in arrival order; no stream has more than `depth`
groups in flight; at low load every request starts when it arrives; at saturation groups carry several requests.
"""
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2204_01287_amd.serve import Request, Scheduler


def _requests(seed, n, rate, nclouds, sizes):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n)) if rate else np.zeros(n)
    out = []
    for i in range(n):
        w, h = sizes[rng.integers(len(sizes))]
        out.append(Request(i, int(rng.integers(nclouds)), SimpleNamespace(width=w, height=h), float(t[i])))
    return out


class FakeDevice:
    """Launches that finish after `per_px` seconds per pixel plus `fixed`; records everything the scheduler does."""

    def __init__(self, sched, per_px=1e-9, fixed=1e-4, dt=2e-5):
        self.sched, self.per_px, self.fixed, self.dt = sched, per_px, fixed, dt
        self.t = 0.0
        self.inflight = {}      # token -> (stream, group, finish)
        self.per_stream = [0] * sched.nstreams
        self.launches = []      # (time, stream, cloud, [rid], admitted bytes in flight or waiting)
        self.next = 0

    def now(self):
        return self.t

    def idle(self):
        self.t += self.dt

    def launch(self, si, cloud, group):
        finish = self.t + self.fixed + self.per_px * sum(r.cam.width * r.cam.height for r in group)
        tok = self.next
        self.next += 1
        self.inflight[tok] = (si, group, finish)
        self.per_stream[si] += 1
        assert self.per_stream[si] <= self.sched.depth, "more groups in flight on a stream than depth"
        self.launches.append((self.t, si, cloud, [r.rid for r in group]))
        return tok

    def is_done(self, tok):
        return self.t >= self.inflight[tok][2]

    def retire(self, tok, group):
        si, g, _ = self.inflight.pop(tok)
        assert g is group
        self.per_stream[si] -= 1

    def run(self, reqs):
        return self.sched.run(reqs, self.launch, self.is_done, self.retire, self.now, self.idle)


def _check_common(sched, dev, reqs, done):
    assert sorted(d.rid for d in done) == [r.rid for r in reqs], "every request completes exactly once"
    by_id = {r.rid: r for r in reqs}
    for d in done:
        assert d.completed >= d.launched >= d.arrival - 1e-12
        assert d.arrival == by_id[d.rid].arrival and d.cloud == by_id[d.rid].cloud
    largest = max(sched.request_bytes(r) for r in reqs)
    assert sched.peak_bytes <= max(sched.budget, largest)
    launched_order = {}
    for t, si, cloud, rids in dev.launches:
        assert 1 <= len(rids) <= sched.max_group
        assert all(by_id[i].cloud == cloud for i in rids), "a group holds one cloud"
        for i in rids:
            launched_order[i] = (t, len(launched_order))
    for c in {r.cloud for r in reqs}:  # within a cloud, requests start in arrival order
        rs = sorted((r for r in reqs if r.cloud == c), key=lambda r: (r.arrival, r.rid))
        seq = [launched_order[r.rid][1] for r in rs]
        assert seq == sorted(seq), f"cloud {c}: launch order differs from arrival order"


@pytest.mark.parametrize("nstreams,depth,max_group", [(4, 1, 64), (2, 2, 8), (1, 1, 1), (3, 1, 64)])
def test_saturated(nstreams, depth, max_group):
    reqs = _requests(1, 300, 0, 5, [(640, 480), (1920, 1080), (3840, 2160)])
    sched = Scheduler(nstreams, budget_bytes=4 << 30, max_group=max_group, depth=depth)
    dev = FakeDevice(sched)
    done = dev.run(reqs)
    _check_common(sched, dev, reqs, done)
    if max_group > 1:
        assert np.mean([d.group for d in done]) > 2.0, "at saturation groups should carry several requests"
    else:
        assert all(d.group == 1 for d in done)


def test_low_load_starts_each_request_on_arrival():
    reqs = _requests(2, 200, 50.0, 3, [(640, 480), (1920, 1080)])   # 20 ms apart on average, service < 3 ms
    sched = Scheduler(4, budget_bytes=1 << 30)
    dev = FakeDevice(sched)
    done = dev.run(reqs)
    _check_common(sched, dev, reqs, done)
    for d in done:
        assert d.launched - d.arrival <= dev.dt + 1e-12, "an idle server starts a request when it arrives"
    assert max(d.group for d in done) == 1


def test_budget_and_oversize_request():
    sizes = [(640, 480), (1920, 1080)]
    reqs = _requests(3, 120, 0, 2, sizes)
    big = Request(len(reqs), 0, SimpleNamespace(width=3840, height=2160), 0.0)   # 99.5 MB > the 64 MB budget
    reqs.append(big)
    sched = Scheduler(4, budget_bytes=64 << 20, max_group=64)
    dev = FakeDevice(sched)
    held = []

    real_launch = dev.launch

    def launch(si, cloud, group):
        tok = real_launch(si, cloud, group)
        held.append((dev.t, sum(sched.request_bytes(r) for g in dev.inflight.values() for r in g[1])))
        if any(r.rid == big.rid for r in group):
            assert len(dev.inflight) == 1 and len(group) == 1, "the oversize request runs alone"
        return tok

    done = sched.run(reqs, launch, dev.is_done, dev.retire, dev.now, dev.idle)
    _check_common(sched, dev, reqs, done)
    for t, nbytes in held:
        assert nbytes <= max(sched.budget, sched.request_bytes(big))


def test_rejects_bad_parameters():
    with pytest.raises(ValueError):
        Scheduler(max_group=0)
    with pytest.raises(ValueError):
        Scheduler(max_group=65)
    with pytest.raises(ValueError):
        Scheduler(depth=0)

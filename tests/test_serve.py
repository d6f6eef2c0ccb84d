"""Serving loop: admission, budget, rejection, cancellation and statistics
with a host executor (CPU), and alone-vs-mix equality on the GPU."""
import threading
import time

import numpy as np
import pytest

from paper_2510_01785_amd.serve import AdmissionError, Request, Scheduler


class FakeData:
    def __init__(self, batch):
        self.shape = (batch, 1)

    def dim(self):
        return 2


class HostExecutor:
    """Each request 'runs' for dur seconds; records concurrency and memory."""

    def __init__(self, dur=0.01):
        self.dur = dur
        self.lock = threading.Lock()
        self.live = 0
        self.max_live = 0
        self.launched = []

    def need(self, req):
        return req.nside  # the tests set the byte need through nside

    def launch(self, req, slot):
        with self.lock:
            self.live += 1
            self.max_live = max(self.max_live, self.live)
            self.launched.append((req.lmax, slot))
        return [time.perf_counter() + self.dur, req]

    def done(self, h):
        return time.perf_counter() >= h[0]

    def finish(self, h):
        with self.lock:
            self.live -= 1
        return ("out", h[1].lmax)


def make(need, tag, batch=1, timeout=None):
    return Request("map2alm", need, tag, FakeData(batch), timeout=timeout)


def test_budget_never_exceeded_and_fifo():
    """max_skips=0: strict arrival order under the budget and slot count."""
    ex = HostExecutor(0.005)
    s = Scheduler(ex, budget_bytes=100, slots=4, max_skips=0)
    reqs = [make(30 + (i % 3) * 20, i) for i in range(40)]
    futs = [s.submit(r) for r in reqs]
    for f in futs:
        f.result(timeout=10)
    st = s.stats()
    s.close()
    assert st["requests"] == 40
    assert s.peak_in_use <= 100
    assert ex.max_live <= 4
    assert [t for t, _ in ex.launched] == list(range(40))  # admitted in arrival order
    assert s.in_use == 0


def test_small_requests_pass_a_blocked_head_without_starving_it():
    """A head request that does not fit yet lets later ones that fit start,
    at most max_skips times; then it starts before anything behind it."""
    ex = HostExecutor(0.03)
    s = Scheduler(ex, budget_bytes=100, slots=8, max_skips=3)
    first = s.submit(make(60, "first"))
    time.sleep(0.005)
    big = s.submit(make(80, "big"))            # blocked while "first" runs
    small = [s.submit(make(10, "s%d" % i)) for i in range(6)]
    for f in [first, big] + small:
        f.result(timeout=10)
    s.close()
    order = [t for t, _ in ex.launched]
    assert order[0] == "first"
    # exactly max_skips small requests went ahead of the blocked head, the
    # rest waited behind it
    assert order.index("big") == 1 + 3
    assert s.peak_in_use <= 100 and s.in_use == 0


class TableExecutor(HostExecutor):
    """need = (transient, resident): 'tables' of a new key stay resident."""

    def __init__(self, dur=0.005):
        super().__init__(dur)
        self.keys = set()

    def need(self, req):
        return (req.nside, 0 if req.lmax in self.keys else 25)

    def launch(self, req, slot):
        self.keys.add(req.lmax)
        return super().launch(req, slot)


def test_resident_tables_stay_charged():
    ex = TableExecutor()
    s = Scheduler(ex, budget_bytes=100, slots=2)
    futs = [s.submit(make(10, k % 3)) for k in range(9)]
    for f in futs:
        f.result(timeout=10)
    st = s.stats()
    s.close()
    assert st["resident_bytes"] == 3 * 25 and s.in_use == 3 * 25
    assert s.peak_in_use <= 100
    # a request that no longer fits beside the resident tables is rejected
    s2 = Scheduler(ex, budget_bytes=100, slots=2)
    s2.resident = s2.in_use = 80
    with pytest.raises(AdmissionError):
        s2.submit(make(30, 0)).result(timeout=1)
    s2.close()


class GroupExecutor(HostExecutor):
    """Supports merged jobs: requests with the same lmax tag share a key;
    need = sum of the members' nside (bytes) plus 1 per merged member."""

    def __init__(self, dur=0.02):
        super().__init__(dur)
        self.jobs = []

    def group_key(self, req):
        return req.lmax

    def need_group(self, reqs):
        return sum(r.nside for r in reqs) + (len(reqs) - 1)

    def launch_group(self, reqs, slot):
        with self.lock:
            self.live += 1
            self.max_live = max(self.max_live, self.live)
            self.jobs.append([r.lmax for r in reqs])
            self.launched.extend((r.lmax, slot) for r in reqs)
        return [time.perf_counter() + self.dur, reqs]

    def launch(self, req, slot):
        return self.launch_group([req], slot)

    def finish(self, h):
        with self.lock:
            self.live -= 1
        reqs = h[1]
        out = [("out", r.lmax, r.batch) for r in reqs]
        return out if len(reqs) > 1 else out[0]


def test_queued_requests_of_one_key_are_merged():
    """While the only slot is busy, queued requests with the same key are
    admitted together (channel cap, budget), each future gets its own result."""
    ex = GroupExecutor(0.03)
    s = Scheduler(ex, budget_bytes=100, slots=1, max_merge_channels=10)
    first = s.submit(make(10, "a", batch=2))
    time.sleep(0.005)
    later = [s.submit(make(10, k, batch=3)) for k in ("a", "b", "a", "a", "b", "a")]
    res = [f.result(timeout=10) for f in [first] + later]
    s.close()
    assert res[0] == ("out", "a", 2)
    assert [r[1] for r in res[1:]] == ["a", "b", "a", "a", "b", "a"] and all(r[2] == 3 for r in res[1:])
    assert ex.jobs[0] == ["a"]
    # the next job is the queued head "a" with the later "a"s that fit in
    # 10 channels (3 + 3 + 3), then the "b"s together, then the last "a"
    assert ex.jobs[1] == ["a", "a", "a"] and ex.jobs[2] == ["b", "b"] and ex.jobs[3] == ["a"]
    assert s.peak_in_use <= 100 and s.in_use == 0
    st = s.stats()
    assert st["requests"] == 7 and st["maps"] == 2 + 6 * 3


def test_merge_respects_the_budget():
    ex = GroupExecutor(0.03)
    s = Scheduler(ex, budget_bytes=45, slots=1, max_merge_channels=64)
    first = s.submit(make(20, "x"))
    time.sleep(0.005)
    later = [s.submit(make(20, "x")) for _ in range(3)]
    for f in [first] + later:
        f.result(timeout=10)
    s.close()
    # two members need 20 + 20 + 1 = 41 <= 45; three would need 62
    assert ex.jobs == [["x"], ["x", "x"], ["x"]]
    assert s.peak_in_use <= 45


def test_over_budget_rejected_without_launch():
    ex = HostExecutor()
    s = Scheduler(ex, budget_bytes=100, slots=2)
    f = s.submit(make(101, "big"))
    with pytest.raises(AdmissionError):
        f.result(timeout=1)
    ok = s.submit(make(100, "fits"))
    assert ok.result(timeout=5) == ("out", "fits")
    s.close()
    assert [t for t, _ in ex.launched] == ["fits"]


def test_cancel_and_timeout_in_queue():
    ex = HostExecutor(0.2)
    s = Scheduler(ex, budget_bytes=10, slots=1)
    first = s.submit(make(10, "first"))
    time.sleep(0.02)
    cancelled = s.submit(make(10, "cancelled"))
    timed = s.submit(make(10, "timed", timeout=0.05))
    last = s.submit(make(10, "last"))
    assert cancelled.cancel()
    assert first.result(timeout=5) == ("out", "first")
    with pytest.raises(TimeoutError):
        timed.result(timeout=5)
    assert last.result(timeout=5) == ("out", "last")
    s.close()
    assert [t for t, _ in ex.launched] == ["first", "last"]


def test_stats_well_formed():
    ex = HostExecutor(0.002)
    s = Scheduler(ex, budget_bytes=1000, slots=3)
    rng = np.random.default_rng(17856)
    futs = []
    for i in range(30):
        futs.append(s.submit(make(int(rng.integers(50, 400)), i, batch=int(rng.integers(1, 33)))))
        time.sleep(float(rng.exponential(0.001)))
    for f in futs:
        f.result(timeout=10)
    st = s.stats()
    s.close()
    assert st["requests"] == 30 and st["maps"] > 0
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    assert st["queue_depth"] == 0 and st["in_use_bytes"] == 0 and st["resident_bytes"] == 0
    assert st["peak_in_use_bytes"] <= 1000 and st["maps_per_s"] > 0


@pytest.mark.gpu
def test_gpu_mix_equals_alone():
    """Each request's output is bit-identical alone and in a concurrent mix of
    several (nside, lmax), directions and batch sizes; with queued requests
    of one geometry merged into one call, equal within the FP32 tolerance."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_01785_amd as shtx
    from paper_2510_01785_amd import synth
    from paper_2510_01785_amd.serve import Server
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(17856)
    reqs = []
    for i in range(12):
        nside = int(rng.choice([16, 32, 64]))
        lmax = int(rng.choice([2 * nside - 1, 3 * nside - 1]))
        B = int(rng.integers(1, 20))
        if i % 2 == 0:
            x = torch.tensor(synth.white_map(100 + i, B, 12 * nside * nside), dtype=torch.float32, device=dev)
            reqs.append(("map2alm", nside, lmax, x))
        else:
            a = torch.tensor(synth.random_alm(100 + i, B, lmax), dtype=torch.complex64, device=dev)
            reqs.append(("alm2map", nside, lmax, a))
    alone = []
    for d, nside, lmax, x in reqs:
        alone.append(shtx.map2alm_raw(x, lmax) if d == "map2alm" else shtx.alm2map_raw(x, nside, lmax))
    torch.cuda.synchronize()
    # without merging: every request is its own call, bit-identical to alone
    srv = Server(dev, budget_bytes=2 << 30, slots=4, max_merge_channels=0)
    futs = [srv.submit(Request(d, nside, lmax, x)) for d, nside, lmax, x in reqs]
    outs = [f.result(timeout=60) for f in futs]
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    for a, o in zip(alone, outs):
        assert torch.equal(a, o)
    assert st["requests"] == 12 and st["peak_in_use_bytes"] <= 2 << 30
    # with merging (one slot, so that queued requests of one geometry merge):
    # a merged call may take the matrix-core kernels where the request alone
    # took the vector ones, so the results agree to the FP32 tolerance
    srv = Server(dev, budget_bytes=2 << 30, slots=1, max_merge_channels=64)
    futs = [srv.submit(Request(d, nside, lmax, x)) for d, nside, lmax, x in reqs]
    merged = [f.result(timeout=60) for f in futs]
    srv.close()
    torch.cuda.synchronize()
    for a, o in zip(alone, merged):
        assert o.shape == a.shape
        err = float(torch.linalg.vector_norm((o - a).flatten()) / torch.linalg.vector_norm(a.flatten()))
        assert err <= 1e-5, err
    # and each served result is the transform: FP32 parity with the FP64 oracle
    from oracle import sht
    for (d, nside, lmax, x), o in zip(reqs, outs):
        xin = x.cpu().numpy()
        if d == "map2alm":
            ref = sht.map2alm(xin.astype(np.float64), lmax, nside)
        else:
            ref = sht.alm2map(xin.astype(np.complex128), nside, lmax)
        got = o.cpu().numpy()
        err = np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel())
        assert err <= 1e-5, (d, nside, lmax, err)

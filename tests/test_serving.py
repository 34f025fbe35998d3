"""The serving scheduler on the CPU: a simulated executor stands in for the
GPU (virtual clock, batch duration proportional to its rays), so admission,
ordering, overlap and the failure paths are checked without a device."""

import time

import numpy as np
import pytest

from paper_2205_15401_amd import scenes as S
from paper_2205_15401_amd.serving import Executor, Request, Server, latency_stats, serve_trace


class FakeExecutor(Executor):
    """Batches take `base + per_ray * rays` seconds of virtual time."""

    def __init__(self, shapes, n_slots=2, base=1e-3, per_ray=1e-8, real_time=False):
        self.shapes = shapes
        self.n_slots = n_slots
        self.base, self.per_ray = base, per_ray
        self.t = 0.0
        self.real_time = real_time
        self.t0 = time.perf_counter()
        self.launches = []          # (time, slot, [rid], end)
        self.fail_launch = set()    # batch numbers whose launch raises
        self.fail_collect = set()   # batch numbers whose collect raises

    def now(self):
        return time.perf_counter() - self.t0 if self.real_time else self.t

    def scene_shape(self, scene):
        return self.shapes.get(scene)

    def item_bytes(self, req):
        N, C = self.shapes[req.scene]
        b = 4 * req.rays * C
        if req.backward:
            b += 4 * req.rays * C + 4 * N * (9 + C)
        return b + 100 * req.rays

    def launch(self, slot, reqs):
        k = len(self.launches)
        if k in self.fail_launch:
            self.launches.append((self.now(), slot, [r.rid for r in reqs], None))
            raise RuntimeError("injected launch failure")
        end = self.now() + self.base + self.per_ray * sum(r.rays for r in reqs)
        self.launches.append((self.now(), slot, [r.rid for r in reqs], end))
        return {"end": end, "k": k, "reqs": reqs}

    def ready(self, h):
        return self.now() >= h["end"]

    def collect(self, h):
        if h["k"] in self.fail_collect:
            raise RuntimeError("injected device failure")
        for r in h["reqs"]:
            r.image = ("image", r.rid)


def cam(size):
    return S.identity_camera(size)


def simulate(server, ex, reqs, check=None):
    """Drive the server on the virtual clock: jump to the next arrival or the
    next batch end, submit arrivals, pump; `check` runs after every pump."""
    pending = sorted(reqs, key=lambda r: r.arrival)
    i = 0
    while i < len(pending) or not server.idle():
        while i < len(pending) and pending[i].arrival <= ex.t:
            server.submit(pending[i])
            i += 1
        server.pump()
        if check:
            check(server)
        ends = [b.handle["end"] for b in server.inflight.values()]
        nxt = [pending[i].arrival] if i < len(pending) else []
        waiting = list(server.queue) + [r for b in server.inflight.values() for r in b.reqs if r.done is None]
        dls = [r.deadline for r in waiting if r.deadline is not None]
        cand = [t for t in ends + nxt + dls if t > ex.t]
        if not cand:
            if server.idle() and i >= len(pending):
                break
            cand = [ex.t + 1e-6]
        ex.t = min(cand)
    return server


def random_requests(rng, n, scenes=(0, 1), sizes=(16, 32, 64, 128), rate=2000.0):
    t = 0.0
    out = []
    for _ in range(n):
        t += rng.exponential(1.0 / rate)
        bwd = bool(rng.uniform() < 0.5)
        out.append(Request(scene=int(rng.choice(scenes)), camera=cam(int(rng.choice(sizes))), backward=bwd,
                           grad_image=np.zeros(1) if bwd else None, arrival=t))
    return out


SHAPES = {0: (1000, 3), 1: (20000, 3)}


def test_budget_is_never_exceeded_and_every_request_completes():
    rng = np.random.default_rng(1)
    ex = FakeExecutor(SHAPES)
    reqs = random_requests(rng, 400)
    budget = 4 * max(ex.item_bytes(r) for r in reqs)
    srv = Server(ex, budget, max_batch_items=16)

    def check(s):
        assert s.inflight_bytes <= budget
        assert len(s.inflight) <= ex.n_slots

    simulate(srv, ex, reqs, check)
    assert len(srv.completed) == len(reqs)
    assert all(r.error is None and r.image == ("image", r.rid) for r in reqs)
    assert 0 < srv.peak_bytes <= budget
    assert srv.batches < len(reqs)          # requests were batched
    st = latency_stats(reqs)
    assert st["n"] == len(reqs) and 0 < st["p50_ms"] <= st["p99_ms"]


def test_requests_of_one_kind_are_admitted_in_arrival_order():
    rng = np.random.default_rng(2)
    ex = FakeExecutor(SHAPES)
    reqs = random_requests(rng, 300)
    srv = Server(ex, 3 * max(ex.item_bytes(r) for r in reqs), max_batch_items=8)
    simulate(srv, ex, reqs)
    for kind in (False, True):
        adm = [r.admitted for r in sorted(reqs, key=lambda r: r.rid) if r.backward == kind]
        assert all(a <= b for a, b in zip(adm, adm[1:]))


def test_arrivals_during_a_batch_run_in_the_second_slot():
    ex = FakeExecutor(SHAPES, base=10e-3)
    a = Request(scene=0, camera=cam(64), arrival=0.0)
    b = Request(scene=1, camera=cam(64), arrival=1e-3)        # arrives while a's batch runs
    srv = simulate(Server(ex, 1 << 30), ex, [a, b])
    assert len(ex.launches) == 2
    (t_a, slot_a, ids_a, end_a), (t_b, slot_b, ids_b, end_b) = ex.launches
    assert ids_a == [a.rid] and ids_b == [b.rid] and slot_a != slot_b
    assert t_b < end_a                                        # the two batches overlap
    assert srv.idle()


def test_waiting_requests_join_one_batch_when_a_slot_frees():
    ex = FakeExecutor(SHAPES, n_slots=1, base=10e-3)
    first = Request(scene=0, camera=cam(32), arrival=0.0)
    later = [Request(scene=0, camera=cam(32), arrival=1e-3 * (i + 1)) for i in range(5)]
    simulate(Server(ex, 1 << 30), ex, [first] + later)
    assert [len(ids) for _, _, ids, _ in ex.launches] == [1, 5]


def test_rejections_leave_the_rest_running():
    ex = FakeExecutor(SHAPES)
    budget = 10_000_000
    srv = Server(ex, budget)
    bad = [Request(scene=7, camera=cam(32)),                                 # unknown scene
           Request(scene=0, camera=cam(32), backward=True),                  # no upstream gradient
           Request(scene=0, camera=cam(32), K=0),
           Request(scene=1, camera=cam(2048))]                               # larger than the budget
    good = [Request(scene=0, camera=cam(32)), Request(scene=1, camera=cam(16), backward=True,
                                                      grad_image=np.zeros(1))]
    assert [srv.submit(r) for r in bad] == [False] * 4
    assert all(r.error for r in bad)
    assert "budget" in bad[3].error
    for r in good:
        assert srv.submit(r)
    simulate(srv, ex, [])
    assert all(r.error is None and r.done is not None for r in good)
    assert len(srv.completed) == 6


def test_a_failed_batch_fails_its_requests_only():
    ex = FakeExecutor(SHAPES, n_slots=1)
    ex.fail_collect = {0}
    ex.fail_launch = {1}
    reqs = [Request(scene=0, camera=cam(32), arrival=0.0),
            Request(scene=0, camera=cam(32), arrival=0.5e-3),      # batch 1 (launch fails)
            Request(scene=0, camera=cam(32), arrival=5e-3)]
    srv = Server(ex, 1 << 30)
    simulate(srv, ex, reqs)
    assert "device failure" in reqs[0].error
    assert "launch failed" in reqs[1].error
    assert reqs[2].error is None and reqs[2].image is not None
    assert srv.inflight_bytes == 0 and srv.idle()


def test_batch_limits():
    ex = FakeExecutor(SHAPES, n_slots=1, base=10e-3)
    reqs = [Request(scene=0, camera=cam(64), arrival=0.0)] + \
           [Request(scene=0, camera=cam(64), arrival=1e-4) for _ in range(9)] + \
           [Request(scene=0, camera=cam(512), arrival=2e-4)]            # more rays than a batch may hold
    simulate(Server(ex, 1 << 34, max_batch_items=4, max_batch_rays=64 * 64 * 3), ex, reqs)
    sizes = [len(ids) for _, _, ids, _ in ex.launches]
    assert sizes == [1, 3, 3, 3, 1]
    assert all(r.error is None for r in reqs)


def test_a_large_waiting_request_does_not_block_the_other_kind():
    ex = FakeExecutor(SHAPES, n_slots=2, base=10e-3)
    small = Request(scene=0, camera=cam(32), arrival=0.0)
    big_grad = Request(scene=1, camera=cam(256), backward=True, grad_image=np.zeros(1), arrival=1e-4)
    render = Request(scene=0, camera=cam(32), arrival=2e-4)
    budget = ex.item_bytes(big_grad) + ex.item_bytes(render) // 2     # big_grad must wait for `small`
    assert ex.item_bytes(small) + ex.item_bytes(render) <= budget
    simulate(Server(ex, budget), ex, [small, big_grad, render])
    assert render.admitted < big_grad.admitted
    assert all(r.error is None for r in (small, big_grad, render))


def test_serve_trace_in_real_time():
    rng = np.random.default_rng(3)
    ex = FakeExecutor(SHAPES, base=0.5e-3, per_ray=1e-9, real_time=True)
    reqs = random_requests(rng, 200, rate=5000.0)
    srv = Server(ex, 1 << 30, max_batch_items=32)
    elapsed = serve_trace(srv, reqs)
    assert len(srv.completed) == 200 and all(r.error is None for r in reqs)
    assert elapsed < 5.0
    assert all(r.latency >= 0 for r in reqs)


def test_cancel_a_queued_and_an_inflight_request():
    ex = FakeExecutor(SHAPES, n_slots=1, base=10e-3)
    srv = Server(ex, 1 << 30)
    a = Request(scene=0, camera=cam(32))
    b = Request(scene=0, camera=cam(32))
    assert srv.submit(a)
    srv.pump()                                   # a is launched
    assert srv.submit(b)                         # b waits for the slot
    assert srv.cancel(b) and b.error == "cancelled" and b.done == ex.t
    ex.t = 2e-3
    assert srv.cancel(a) and a.error == "cancelled" and a.done == 2e-3 and a.image is None
    assert srv.inflight_bytes > 0                # the batch still runs: its memory is held
    assert not srv.cancel(a)                     # already done
    c = Request(scene=0, camera=cam(16), arrival=3e-3)
    simulate(srv, ex, [c])
    assert c.error is None and c.image == ("image", c.rid)
    assert [ids for _, _, ids, _ in ex.launches] == [[a.rid], [c.rid]]    # b never ran
    assert a.image is None                       # the finished batch hands back nothing for a
    assert srv.idle() and srv.inflight_bytes == 0
    assert len(srv.completed) == 3


def test_deadlines_fail_late_requests_and_the_server_runs_on():
    ex = FakeExecutor(SHAPES, n_slots=1, base=10e-3)
    long_ = Request(scene=0, camera=cam(32), arrival=0.0)
    slow = Request(scene=0, camera=cam(32), arrival=0.0, deadline=4e-3)       # shares the first batch
    queued = Request(scene=0, camera=cam(32), arrival=1e-3, deadline=5e-3)    # the slot is busy until 10 ms
    fine = Request(scene=0, camera=cam(32), arrival=2e-3, deadline=1.0)
    srv = Server(ex, 1 << 30)
    simulate(srv, ex, [long_, slow, queued, fine])
    assert slow.error == "deadline exceeded" and abs(slow.done - 4e-3) < 1e-12 and slow.image is None
    assert queued.error == "deadline exceeded" and abs(queued.done - 5e-3) < 1e-12
    assert long_.error is None and long_.image == ("image", long_.rid)
    assert fine.error is None and fine.image == ("image", fine.rid)
    launched = [rid for _, _, ids, _ in ex.launches for rid in ids]
    assert queued.rid not in launched and slow.rid in launched
    assert srv.idle() and srv.inflight_bytes == 0
    st = latency_stats([long_, slow, queued, fine])
    assert st["n"] == 2


def test_admission_at_serving_sizes_under_a_tight_budget():
    """The serving workload's shapes (scenes of 10k-200k kernels, 128^2 to
    1024^2 images, half gradient requests) under a budget that holds little
    more than one of the largest requests: the budget is never exceeded,
    every request completes, and the largest ones are not starved."""
    shapes = {i: (n, 3) for i, n in enumerate((10_000, 25_000, 50_000, 100_000, 150_000, 200_000))}
    ex = FakeExecutor(shapes, n_slots=2, base=0.5e-3, per_ray=2e-9)
    rng = np.random.default_rng(5)
    reqs = random_requests(rng, 600, scenes=tuple(shapes), sizes=(128, 256, 512, 1024), rate=800.0)
    biggest = max(ex.item_bytes(r) for r in reqs)
    budget = int(1.3 * biggest)
    srv = Server(ex, budget, max_batch_items=64)

    def check(s):
        assert s.inflight_bytes <= budget

    simulate(srv, ex, reqs, check)
    assert all(r.error is None and r.image is not None for r in reqs)
    big = [r for r in reqs if r.rays == 1024 * 1024 and r.backward]
    assert big and all(r.done is not None for r in big)
    assert srv.peak_bytes > 0.5 * budget

"""CPU tests of the serving loop's admission and bookkeeping, against a host
stand-in for the device backend (no GPU work is simulated numerically)."""
import dataclasses

import numpy as np
import pytest

from paper_1812_00390_amd.serve import Request, Server, summarize


@dataclasses.dataclass
class FakeMesh:
    n: int


@dataclasses.dataclass
class FakeInst:
    n_cells: int


class FakeBackend:
    """Residual decays geometrically per chunk at a per-request rate; bytes = 100 per cell."""

    def __init__(self, decay=0.1):
        self.decay = decay
        self.live = {}
        self.created = []
        self.freed = []
        self.batches = []

    def footprint(self, inst):
        return inst.n_cells * 100

    def prepare(self, inst):
        h = len(self.created)
        self.created.append(inst.n_cells)
        self.live[h] = dict(res=1.0, steps=0)
        return h

    def advance(self, handles, steps):
        self.batches.append(tuple(handles))
        for h in handles:
            self.live[h]["res"] *= self.decay
            self.live[h]["steps"] += steps

    def residuals(self, handles):
        return [self.live[h]["res"] for h in handles]

    def fields(self, h):
        return np.zeros(1), np.zeros((1, 2))

    def free(self, h):
        self.freed.append(h)
        del self.live[h]


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 0.001
        return self.t


def test_all_requests_complete_and_bytes_return():
    be = FakeBackend(decay=0.01)
    reqs = [Request(k, FakeInst(1000 * (k + 1)), tol=1e-5, budget=10_000, arrival=0.0) for k in range(10)]
    srv = Server(be, hbm_budget=3_000_000, max_slots=4, chunk=100)
    res = srv.run(reqs, clock=Clock())
    assert sorted(r.rid for r in res) == list(range(10))
    assert srv.used == 0 and not srv.active and not be.live
    assert all(r.converged and r.steps == 300 for r in res)
    assert max(len(b) for b in be.batches) <= 4


def test_byte_budget_limits_concurrency_fifo():
    be = FakeBackend(decay=0.5)
    # two big requests (2.5 MB each) cannot run together under a 4 MB budget
    reqs = [Request(0, FakeInst(25_000), 1e-2, 10_000), Request(1, FakeInst(25_000), 1e-2, 10_000),
            Request(2, FakeInst(1_000), 1e-2, 10_000)]
    srv = Server(be, hbm_budget=4_000_000, max_slots=8, chunk=10)
    res = srv.run(reqs, clock=Clock())
    assert {r.rid for r in res} == {0, 1, 2}
    # FIFO: request 2 (small) waits behind request 1 even though it would fit
    first_batch = be.batches[0]
    assert len(first_batch) == 1
    order = [r.rid for r in sorted(res, key=lambda r: r.admitted)]
    assert order == [0, 1, 2]


def test_oversized_request_rejected():
    be = FakeBackend()
    reqs = [Request(0, FakeInst(10**6), 1e-2, 100), Request(1, FakeInst(100), 1e-2, 100)]
    srv = Server(be, hbm_budget=1_000_000, max_slots=8, chunk=10)
    res = srv.run(reqs, clock=Clock())
    assert srv.rejected == [0]
    assert [r.rid for r in res] == [1]


def test_budget_stops_unconverged_requests():
    be = FakeBackend(decay=1.0)        # never converges
    srv = Server(be, hbm_budget=10**9, max_slots=8, chunk=100)
    res = srv.run([Request(0, FakeInst(100), 1e-6, budget=700)], clock=Clock())
    assert res[0].steps == 700 and not res[0].converged


def test_cancel_frees_slot_and_bytes():
    be = FakeBackend()
    srv = Server(be, hbm_budget=10**9, max_slots=8, chunk=100)
    srv.queue.extend([Request(0, FakeInst(500)), Request(1, FakeInst(700))])
    srv._admit(0.0)
    assert srv.used == 120_000 and len(srv.active) == 2
    assert srv.cancel(0)
    assert srv.used == 70_000 and 0 not in srv.active and be.freed == [0]
    assert not srv.cancel(42)


def test_summary_percentiles():
    from paper_1812_00390_amd.serve import Result
    res = [Result(i, 10, 100, 1e-7, True, 0.0, 0.0, float(i + 1)) for i in range(100)]
    s = summarize(res, wall=10.0, cell_updates=10**8)
    assert s["p50_latency_s"] == pytest.approx(50.5)
    assert s["p99_latency_s"] == pytest.approx(99.01)
    assert s["M_cell_updates_per_s"] == 10.0


class SlowFakeBackend(FakeBackend):
    """Preparation takes a while and runs on the server's worker threads."""

    def prepare(self, inst):
        import time
        time.sleep(0.002)
        return super().prepare(inst)


def test_threaded_preparation_completes_every_request():
    be = SlowFakeBackend(decay=0.1)
    reqs = [Request(k, FakeInst(100 * (k + 1)), tol=1e-3, budget=10_000, arrival=0.0005 * k) for k in range(24)]
    srv = Server(be, hbm_budget=1_000_000, max_slots=5, chunk=10, prep_workers=2)
    res = srv.run(reqs)
    assert sorted(r.rid for r in res) == list(range(24))
    assert srv.used == 0 and not srv.active and not srv.preparing and not be.live
    assert all(r.converged and r.steps == 40 for r in res)      # 0.1^4 < 1e-3 after four chunks
    assert max(len(b) for b in be.batches) <= 5
    assert all(r.admitted >= r.arrival for r in res)


"""Host-side logic of the serving loop (bucketing, flush, admission), with the
C ABI's submit/poll replaced by a stand-in: no GPU involved."""
import numpy as np
import pytest

import synth
from paper_2209_05069_amd import dock as D
from paper_2209_05069_amd import serve as S


class FakeABI:
    """dock_submit/dock_poll stand-in: EAGAIN for the first `refuse` submissions,
    tickets complete `delay` polls after submission."""

    def __init__(self, refuse=0, delay=2):
        self.refuse, self.delay = refuse, delay
        self.sizes, self.pockets = [], []
        self.ticks = {}
        self.next = 1

    def submit(self, ctx, pocket, lib, params, res):
        if self.refuse > 0:
            self.refuse -= 1
            raise D.DockError(D.DOCK_EAGAIN, "busy")
        self.sizes.append(lib.n_ligands)
        self.pockets.append(pocket)
        res.best_score[:] = np.arange(lib.n_ligands)
        t = self.next
        self.next += 1
        self.ticks[t] = self.delay
        return t

    def poll(self, ctx, t):
        self.ticks[t] -= 1
        return self.ticks[t] <= 0


@pytest.fixture
def fake(monkeypatch):
    f = FakeABI(refuse=2)
    monkeypatch.setattr(D, "dock_submit", f.submit)
    monkeypatch.setattr(D, "dock_poll", f.poll)
    return f


def test_buckets_flush_by_size_and_by_age(fake):
    lib = synth.library_uniform(5, 50, (10, 20), (1, 3))
    q = synth.start_quats(5, 4)
    params = D.SearchParams(q, torsion_steps=8, top_k=2)
    srv = S.Server(None, {0: 11, 1: 12}, lib, params, max_batch=8, flush_ms=10.0)
    for i in range(20):
        srv.add(S.Request(i, i % 2, i, 0.0))
    srv.pump(now=0.001)            # pockets 0 and 1 hold 10 each: one full bucket each,
    assert fake.sizes == []        # but both submissions are refused (EAGAIN) and stay queued
    assert srv.stats.eagain == 2
    srv.pump(now=0.002)            # retried: two full buckets; the 2 + 2 leftovers are young
    assert fake.sizes == [8, 8]
    srv.pump(now=0.5)              # leftovers flushed by age
    assert fake.sizes == [8, 8, 2, 2]
    for _ in range(5):
        srv.pump(now=0.6)
    assert srv.idle() and srv.stats.done == 20
    assert set(fake.pockets) == {11, 12}
    assert len(srv.results) == 20


def test_poisson_arrivals_rate():
    a = S.poisson_arrivals(1000.0, 20000, 3)
    assert np.all(np.diff(a) > 0)
    assert abs(20000 / a[-1] - 1000.0) < 30


def test_work_conserving_policy_caps_inflight_and_takes_oldest_first(fake):
    fake.refuse, fake.delay = 0, 3   # a batch finishes on its third poll
    lib = synth.library_uniform(6, 60, (10, 20), (1, 3))
    q = synth.start_quats(6, 4)
    params = D.SearchParams(q, torsion_steps=8, top_k=2)
    srv = S.Server(None, {0: 21, 1: 22, 2: 23}, lib, params, max_batch=16, max_inflight=2)
    # an idle device takes a lone request at once, without waiting for a flush
    srv.add(S.Request(0, 1, 0, 0.0))
    srv.pump(now=0.0)
    assert fake.sizes == [1] and fake.pockets == [22]
    # while the device is busy, requests gather; oldest bucket first, then next
    for i in range(1, 31):
        srv.add(S.Request(i, [2, 0, 1][i % 3], i, 0.001 * i))
    srv.pump(now=0.05)               # one slot free: the oldest head (request 1) is pocket 0's
    assert len(srv.inflight) == 2
    assert fake.pockets[-1] == 21 and fake.sizes[-1] == 10
    for _ in range(3):
        srv.pump(now=0.06)
    assert len(fake.sizes) >= 4 and max(fake.sizes) <= 16
    for _ in range(10):
        srv.pump(now=0.1)
    assert srv.idle() and srv.stats.done == 31
    assert sorted(fake.sizes) == [1, 10, 10, 10]

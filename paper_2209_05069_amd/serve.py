"""Screening service loop over the asynchronous C ABI (dock_submit / dock_poll).

Requests (one ligand each, naming a device-resident pocket) arrive over time.
Per pocket they collect in a bucket.  Two submission policies:
- size/age (max_inflight = 0): a bucket is submitted when it holds `max_batch`
  ligands or its oldest request has waited `flush_ms` (so an underfilled bucket
  does not wait for ever), the way the paper's batched host fills buckets and
  launches them when full (Batched Implementation subsection);
- work-conserving (max_inflight > 0): at most `max_inflight` batches are in
  flight; whenever one finishes (or at once, when the device is idle) the
  bucket whose oldest request has waited longest is submitted, up to
  `max_batch` ligands.  Requests gather while the device is busy, so batches
  grow with the load and stay small (low latency) when it is light.
Admission is by free device memory: when dock_submit answers DOCK_EAGAIN the
bucket stays queued and is retried after completions.  Every request's latency
runs from its arrival to the moment its result is visible on the host.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import dock as D


@dataclass
class Request:
    rid: int
    pocket: int          # key into Server.pockets
    ligand: int          # index into the host library
    t_arrival: float


@dataclass
class _Batch:
    ticket: int
    reqs: list
    res: D.HostResults
    t_submit: float


@dataclass
class ServeStats:
    latencies: list = field(default_factory=list)   # seconds, per request
    done: int = 0
    batches: int = 0
    eagain: int = 0
    t_first: float = None
    t_last: float = None


class Server:
    def __init__(self, ctx, pockets: dict, library, params: D.SearchParams, max_batch=1024,
                 flush_ms=20.0, max_inflight=0, return_poses=False):
        self.ctx = ctx
        self.return_poses = return_poses  # False: scores only (no pose coordinates moved)
        self.max_inflight = max_inflight
        self.pockets = pockets            # key -> pocket id from dock_pocket_load
        self.lib = library                # host CSR library the requests index into
        self.params = params
        self.max_batch = max_batch
        self.flush_s = flush_ms * 1e-3
        self.queues = {k: deque() for k in pockets}
        self.inflight: list[_Batch] = []
        self.stats = ServeStats()
        self.results = {}                 # rid -> best score

    def add(self, req: Request):
        self.queues[req.pocket].append(req)
        if self.stats.t_first is None:
            self.stats.t_first = req.t_arrival

    def _submit(self, key, reqs, now):
        sub = self.lib.subset([r.ligand for r in reqs])
        res = D.HostResults(sub.n_ligands, int(sub.atom_off[-1]), int(sub.rot_off[-1]),
                            self.params, poses=self.return_poses)
        try:
            t = D.dock_submit(self.ctx, self.pockets[key], sub, self.params, res)
        except D.DockError as e:
            if e.code == D.DOCK_EAGAIN:
                self.stats.eagain += 1
                return False
            raise
        self.inflight.append(_Batch(t, reqs, res, now))
        self.stats.batches += 1
        return True

    def pump(self, now=None):
        """Submit due buckets, collect finished batches.  Returns requests done now."""
        now = time.perf_counter() if now is None else now
        if self.max_inflight > 0:
            while len(self.inflight) < self.max_inflight:
                live = [(q[0].t_arrival, k) for k, q in self.queues.items() if q]
                if not live:
                    break
                key = min(live)[1]
                q = self.queues[key]
                take = [q.popleft() for _ in range(min(self.max_batch, len(q)))]
                if not self._submit(key, take, now):
                    q.extendleft(reversed(take))
                    break
        else:
            for key, q in self.queues.items():
                while q and (len(q) >= self.max_batch or now - q[0].t_arrival >= self.flush_s):
                    take = [q.popleft() for _ in range(min(self.max_batch, len(q)))]
                    if not self._submit(key, take, now):
                        q.extendleft(reversed(take))
                        break
        finished = 0
        still = []
        for b in self.inflight:
            if D.dock_poll(self.ctx, b.ticket):
                t = time.perf_counter()
                for i, r in enumerate(b.reqs):
                    self.stats.latencies.append(t - r.t_arrival)
                    self.results[r.rid] = float(b.res.best_score[i])
                self.stats.done += len(b.reqs)
                self.stats.t_last = t
                finished += len(b.reqs)
            else:
                still.append(b)
        self.inflight = still
        return finished

    def idle(self):
        return not self.inflight and all(not q for q in self.queues.values())


def poisson_arrivals(rate, n, seed):
    """n arrival offsets (seconds) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def run(server: Server, requests: list, arrival_offsets, time_limit_s=600.0):
    """Replay requests at their arrival offsets against the server in real time."""
    t0 = time.perf_counter()
    i = 0
    n = len(requests)
    while True:
        now = time.perf_counter()
        while i < n and arrival_offsets[i] <= now - t0:
            r = requests[i]
            r.t_arrival = t0 + arrival_offsets[i]
            server.add(r)
            i += 1
        server.pump(now)
        if i == n and server.idle():
            break
        if now - t0 > time_limit_s:
            raise TimeoutError("serving run exceeded its time limit")
        time.sleep(0.0002)
    st = server.stats
    lat = np.array(st.latencies)
    return dict(requests=n, completed=st.done, batches=st.batches, eagain=st.eagain,
                ligands_per_s=st.done / (st.t_last - st.t_first),
                p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_ms=float(lat.mean() * 1e3))

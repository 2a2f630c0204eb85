"""Serving loop over a job pool: continuous batching of simulation requests.

Requests arrive over time.  Between supersteps (a fixed number of time steps
of every running job) the server admits waiting requests whose particles,
cells and job slot fit in the pool's free device memory, steps the pool,
collects the jobs that finished and frees their memory.  Work of requests
that arrive while others run overlaps on the device in the same launches.

Admission is first-come-first-served with backfilling: a request that does
not fit lets later, smaller requests in, unless it has waited for more than
`max_bypass` supersteps, after which nothing is admitted past it until it
fits.

Host policy only: every time step runs in the HIP library through the pool
(anything with the methods of binding.Pool works, which lets the policy be
tested without a GPU).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

EBUSY = -6


@dataclass
class Request:
    rid: int
    scene: object          # anything with the attributes of gen.Scene
    steps: int
    arrival: float         # seconds since the start of the run
    admitted: float = -1.0
    done: float = -1.0
    job: int = -1
    status: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def work(self) -> int:
        return int(self.scene.n) * int(self.steps)


class Server:
    def __init__(self, pool, superstep=20, max_bypass=50, clock=time.perf_counter,
                 sleep=time.sleep, add_kw=None, on_done=None, prepare_workers=4, lookahead=16,
                 target_s=None, max_superstep=200):
        self.pool = pool
        # with target_s the superstep adapts so that one lasts about target_s
        # seconds: fewer host round trips when the pool is large
        self.target_s = target_s
        self.max_superstep = int(max_superstep)
        # host-side preparation of queued requests on worker threads (the
        # library releases the interpreter lock), when the pool offers it
        self.lookahead = int(lookahead)
        self._exec = None
        if prepare_workers and hasattr(pool, "prepare_scene"):
            import concurrent.futures as cf
            self._exec = cf.ThreadPoolExecutor(int(prepare_workers))
        self.superstep = int(superstep)
        self.max_bypass = int(max_bypass)
        self.clock = clock
        self.sleep = sleep
        self.add_kw = dict(add_kw or {})
        self.on_done = on_done
        self.queue = collections.deque()
        self.running = {}            # job id -> Request
        self.finished = []
        self.supersteps = 0
        self._bypassed = 0           # supersteps the queue head has been passed over
        self._t0 = None

    # --------------------------------------------------------------- time
    def now(self) -> float:
        return self.clock() - self._t0

    # ---------------------------------------------------------- admission
    def _prepare_ahead(self):
        if self._exec is None:
            return
        for k, r in enumerate(self.queue):
            if k >= self.lookahead:
                break
            if "prep" not in r.extra:
                r.extra["prep"] = self._exec.submit(self.pool.prepare_scene, r.scene,
                                                    **self.add_kw)

    def _try_add(self, req) -> bool:
        from .binding import DemError
        try:
            fut = req.extra.get("prep")
            if fut is not None:
                req.job = self.pool.add_prepared(fut.result(), req.steps)
            else:
                req.job = self.pool.add_scene(req.scene, steps=req.steps, **self.add_kw)
        except DemError as e:
            if e.code == EBUSY:
                return False
            raise
        req.extra.pop("prep", None)
        req.admitted = self.now()
        self.running[req.job] = req
        return True

    def admit(self) -> int:
        """Admit waiting requests that fit; returns how many were admitted."""
        self._prepare_ahead()
        k = 0
        while self.queue and self._fits(self.queue[0]) and self._try_add(self.queue[0]):
            self.queue.popleft()
            self._bypassed = 0
            k += 1
        if not self.queue or self._bypassed >= self.max_bypass:
            return k
        # backfill: later requests that fit now pass the head
        rest = collections.deque([self.queue.popleft()])
        passed = 0
        while self.queue:
            r = self.queue.popleft()
            if self._fits(r) and self._try_add(r):
                passed += 1
            else:
                rest.append(r)
        self.queue = rest
        if passed:
            self._bypassed += 1
        return k + passed

    def _adapt(self, seconds):
        if not self.target_s or seconds <= 0.0:
            return
        k = int(self.superstep * self.target_s / seconds)
        k = max(self.superstep // 2, min(2 * self.superstep, k))
        self.superstep = max(1, min(self.max_superstep, k))

    def _fits(self, req) -> bool:
        return self.pool.fits(req.scene, cell_size=self.add_kw.get("cell_size", 0.0))

    # --------------------------------------------------------------- loop
    def _retire(self):
        for j in self.pool.poll():
            req = self.running.pop(j)
            req.done = self.now()
            req.status = self.pool.job_info(j)["status"] if hasattr(self.pool, "job_info") else "done"
            if self.on_done is not None:
                self.on_done(req, self.pool)
            self.pool.remove(j)
            self.finished.append(req)

    def run(self, requests, deadline=None):
        """Serve `requests` (sorted by arrival) to completion; returns stats."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        self._t0 = self.clock()
        while pending or self.queue or self.running:
            now = self.now()
            if deadline is not None and now > deadline:
                raise TimeoutError("serving run exceeded %.1f s" % deadline)
            while pending and pending[0].arrival <= now:
                self.queue.append(pending.popleft())
            self._prepare_ahead()
            if self.running:
                # the superstep is enqueued first: the host work of admitting
                # new requests overlaps it on the device
                t0 = self.clock()
                self.pool.step(self.superstep)
                self.supersteps += 1
                self.admit()
                self._retire()
                self._adapt(self.clock() - t0)
                continue
            self.admit()
            if self.running:
                continue
            if pending:
                # idle until the next arrival
                self.sleep(max(0.0, pending[0].arrival - self.now()))
            elif self.queue:
                raise RuntimeError("request %d can never fit in the pool" % self.queue[0].rid)
        if self._exec is not None:
            self._exec.shutdown(wait=True)
        return self.stats()

    def stats(self) -> dict:
        fin = [r for r in self.finished if r.done >= 0]
        if not fin:
            return dict(jobs=0)
        lat = np.array([r.latency for r in fin])
        wait = np.array([r.admitted - r.arrival for r in fin])
        service = lat - wait
        span = max(r.done for r in fin) - min(r.arrival for r in fin)
        work = sum(r.work for r in fin if r.status in ("done", ""))
        return dict(jobs=len(fin), failed=sum(1 for r in fin if r.status == "failed"),
                    p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    mean_s=float(lat.mean()), max_s=float(lat.max()),
                    wait_p50_s=float(np.percentile(wait, 50)),
                    wait_p99_s=float(np.percentile(wait, 99)),
                    service_p50_s=float(np.percentile(service, 50)),
                    service_p99_s=float(np.percentile(service, 99)),
                    makespan_s=float(span), particle_steps=int(work),
                    particle_steps_per_s=float(work / span) if span > 0 else 0.0,
                    supersteps=self.supersteps)

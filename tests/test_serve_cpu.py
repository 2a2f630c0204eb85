"""CPU tests of the serving policy (continuous batching, admission by
footprint, backfilling with a bypass limit) against a simulated pool and a
simulated clock: no GPU and no library calls."""
import types

import numpy as np
import pytest

from paper_1503_03553_amd.binding import DemError
from paper_1503_03553_amd.serve import Request, Server


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, s):
        self.t += max(0.0, s)


class FakePool:
    """Pool with a particle and a job-slot budget; a step costs `cost` seconds
    per particle of the running jobs on the shared clock."""

    def __init__(self, clock, max_particles, max_jobs, cost=1e-6):
        self.clock, self.cap, self.max_jobs, self.cost = clock, max_particles, max_jobs, cost
        self.jobs = {}
        self.next = 1
        self.log = []          # (time, running job ids) after each step

    def used(self):
        return sum(j["n"] for j in self.jobs.values())

    def fits(self, sc, cell_size=0.0):
        return len(self.jobs) < self.max_jobs and self.used() + sc.n <= self.cap

    def add_scene(self, sc, steps):
        if not self.fits(sc):
            raise DemError(-6, "dem_pool_add")
        j = self.next
        self.next += 1
        self.jobs[j] = dict(n=sc.n, steps=steps, done=0, reported=False)
        return j

    def step(self, k):
        running = [j for j, v in self.jobs.items() if v["done"] < v["steps"]]
        self.clock.t += k * self.cost * sum(self.jobs[j]["n"] for j in running)
        for j in running:
            v = self.jobs[j]
            v["done"] = min(v["steps"], v["done"] + k)
        assert self.used() <= self.cap and len(self.jobs) <= self.max_jobs
        self.log.append((self.clock.t, tuple(running)))

    def poll(self):
        out = []
        for j, v in self.jobs.items():
            if v["done"] >= v["steps"] and not v["reported"]:
                v["reported"] = True
                out.append(j)
        return out

    def job_info(self, j):
        return dict(status="done")

    def remove(self, j):
        del self.jobs[j]


def scene(n):
    return types.SimpleNamespace(n=n)


def run(reqs, cap=1000, max_jobs=4, superstep=10, max_bypass=50):
    clk = Clock()
    pool = FakePool(clk, cap, max_jobs)
    srv = Server(pool, superstep=superstep, max_bypass=max_bypass, clock=clk, sleep=clk.sleep)
    st = srv.run(reqs)
    return srv, pool, st


def test_every_request_completes_and_latency_is_consistent():
    rng = np.random.default_rng(0)
    t = np.cumsum(rng.exponential(0.05, size=40))
    reqs = [Request(k, scene(int(rng.integers(10, 400))), int(rng.integers(5, 200)), float(t[k]))
            for k in range(40)]
    srv, pool, st = run(reqs)
    assert st["jobs"] == 40
    for r in srv.finished:
        assert r.arrival <= r.admitted <= r.done
        # at least its own steps' worth of device time at the step cost
        assert r.done - r.admitted >= 0.0
    assert st["p50_s"] <= st["p99_s"] <= st["max_s"]
    assert st["particle_steps"] == sum(r.work for r in reqs)


def test_arrivals_join_running_jobs():
    # a long job runs; short ones arriving later are admitted beside it
    reqs = [Request(0, scene(300), 1000, 0.0)] + \
           [Request(k, scene(50), 20, 0.01 * k) for k in range(1, 6)]
    srv, pool, st = run(reqs)
    overlap = [ids for _, ids in pool.log if len(ids) >= 2]
    assert overlap, "no step ran two jobs together"
    first = min(srv.finished, key=lambda r: r.rid)
    assert all(r.done < first.done for r in srv.finished if r.rid != 0)


def test_backfill_then_bypass_limit():
    # head needs the whole pool; small requests behind it may pass it only
    # for max_bypass supersteps
    reqs = [Request(0, scene(600), 50, 0.0),
            Request(1, scene(900), 10, 0.001)] + \
           [Request(k, scene(100), 10, 0.001 + 0.0005 * k) for k in range(2, 30)]
    srv, pool, st = run(reqs, cap=1000, max_jobs=8, superstep=5, max_bypass=3)
    done = {r.rid: r for r in srv.finished}
    assert len(done) == 30
    passed = [r for r in srv.finished if r.rid >= 2 and r.admitted < done[1].admitted]
    assert passed, "no backfilling happened"
    # once the bypass limit is reached, request 1 is admitted before the rest
    later = [r for r in srv.finished if r.rid >= 2 and r.admitted > done[1].admitted]
    assert later, "the bypass limit never held the queue"


def test_request_that_can_never_fit_is_an_error():
    reqs = [Request(0, scene(2000), 10, 0.0)]
    with pytest.raises(RuntimeError):
        run(reqs, cap=1000)


# ------------------------------------------------------------------ tuner
from paper_1503_03553_amd import tune  # noqa: E402


class TimedPool:
    """Pool whose step time depends on the candidate it was built for."""

    def __init__(self, clock, cand, cost):
        self.clock, self.cand, self.cost = clock, cand, cost
        self.added = []

    def add_scene(self, sc, steps, cell_size=0.0):
        self.added.append((sc.n, cell_size))
        return len(self.added)

    def step(self, k):
        self.clock.t += k * self.cost(self.cand)

    def sync(self):
        pass

    def close(self):
        pass


def test_autotuner_picks_the_fastest_candidate_and_lays_jobs_out_in_order():
    clk = Clock()
    scenes = [types.SimpleNamespace(n=n, r=np.full(n, 1e-6, np.float32), lo=np.zeros(3),
                                    hi=np.full(3, 1e-4 * (k + 1)))
              for k, n in enumerate([50, 400, 10, 200])]
    cost = lambda c: 1.0 + abs(c["cell_factor"] - 1.25) + (0.5 if c["order"] != "size_desc" else 0)
    pools = []

    def make(c):
        pools.append(TimedPool(clk, c, cost))
        return pools[-1]

    best, table = tune.autotune(make, scenes, steps=4, warmup=1, clock=clk)
    assert best == dict(cell_factor=1.25, order="size_desc")
    assert len(table) == len(tune.candidates())
    sec = dict((tuple(sorted(c.items())), s) for c, s in table)
    assert sec[tuple(sorted(best.items()))] == pytest.approx(1.0)
    p = [q for q in pools if q.cand == best][0]
    assert [n for n, _ in p.added] == [400, 200, 50, 10]
    assert all(cs == pytest.approx(1.25 * 2e-6) for _, cs in p.added)
    # density order: the smallest box is the densest
    assert tune.job_order(scenes, "density_desc")[0] == 0
    assert tune.cell_size_for(scenes[0], 1.0) == 0.0


class PreparingPool(FakePool):
    """FakePool with the prepare / add-prepared split of binding.Pool."""

    def __init__(self, *a, **kw):
        super().__init__(*a, **kw)
        self.prepared = []

    def prepare_scene(self, sc):
        self.prepared.append(sc)
        return types.SimpleNamespace(sc=sc, n=sc.n)

    def add_prepared(self, prep, steps):
        return self.add_scene(prep.sc, steps)


def test_requests_are_prepared_ahead_once_each():
    clk = Clock()
    pool = PreparingPool(clk, 1000, 4)
    reqs = [Request(k, scene(100 + 10 * k), 30, 0.001 * k) for k in range(20)]
    srv = Server(pool, superstep=10, clock=clk, sleep=clk.sleep, lookahead=3)
    st = srv.run(reqs)
    assert st["jobs"] == 20
    assert len(pool.prepared) == 20
    assert len({id(s) for s in pool.prepared}) == 20

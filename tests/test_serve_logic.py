"""Host logic of the serving loop (admission, continuous batching, retirement)
on a fake backend with a virtual clock: no GPU involved."""
import numpy as np
import pytest

from paper_1704_04551_amd.serve import Job, Server, poisson_jobs


class Spec:
    def __init__(self, n, steps):
        self.n = (n, n, n)
        self.steps = steps


class FakeSim:
    def __init__(self, spec):
        self.spec = spec
        self.done = 0


class FakeBackend:
    """Footprint = cells; one step of a batch costs 1 ms of virtual time per
    million resident cells (plus 0.1 ms per launch sequence)."""

    def __init__(self, clock):
        self.clock = clock
        self.live = set()
        self.batches = []

    def footprint(self, spec):
        return int(np.prod(spec.n))

    def create(self, spec):
        s = FakeSim(spec)
        self.live.add(id(s))
        return s

    def step(self, sims, steps):
        assert all(id(s) in self.live for s in sims)
        assert all(k > 0 for k in steps)
        self.batches.append([(s.spec, k) for s, k in zip(sims, steps)])
        for s, k in zip(sims, steps):
            s.done += k
        cells = sum(int(np.prod(s.spec.n)) for s in sims)
        self.clock.t += 1e-4 + max(steps) * cells * 1e-9

    def wait(self, sims):
        pass

    def result(self, sim, spec):
        return {"steps": sim.done}

    def release(self, sim):
        self.live.discard(id(sim))

    def close(self):
        pass


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def make(pool, chunk=10, max_resident=8, queue_cap=100):
    c = Clock()
    be = FakeBackend(c)
    return Server(be, pool, chunk=chunk, max_resident=max_resident, queue_cap=queue_cap, clock=c,
                  sleep=c.sleep), be, c


def test_every_job_runs_exactly_its_steps():
    srv, be, _ = make(pool=10 ** 7)
    jobs = [Job(i, Spec(16 + 8 * (i % 3), 5 + 7 * i), arrival=0.001 * i, steps=5 + 7 * i) for i in range(12)]
    st = srv.run(jobs)
    assert st["finished"] == 12 and st["rejected"] == 0 and st["unfinished"] == 0
    for j in jobs:
        assert j.result["steps"] == j.steps
        assert j.admitted >= j.arrival and j.done >= j.admitted
    assert not be.live  # every arena released


def test_pool_bound_and_fcfs_admission():
    pool = 3 * 32 ** 3
    srv, be, _ = make(pool=pool, max_resident=64)
    jobs = [Job(i, Spec(32, 30), arrival=0.0, steps=30) for i in range(7)]
    srv.run(jobs)
    assert srv.peak_used <= pool
    assert max(len(b) for b in be.batches) == 3
    order = sorted(jobs, key=lambda j: (j.admitted, j.jid))
    assert [j.jid for j in order] == list(range(7))


def test_slots_bound():
    srv, be, _ = make(pool=10 ** 9, max_resident=2)
    jobs = [Job(i, Spec(16, 20), arrival=0.0, steps=20) for i in range(5)]
    srv.run(jobs)
    assert max(len(b) for b in be.batches) == 2


def test_rejections():
    srv, _, _ = make(pool=20 ** 3, queue_cap=2, max_resident=1)
    jobs = [Job(0, Spec(32, 10), 0.0, 10)] + [Job(i, Spec(8, 10), 0.0, 10) for i in range(1, 6)]
    st = srv.run(jobs)
    reasons = sorted(j.rejected for j in jobs if j.rejected)
    assert "larger than the pool" in reasons
    assert reasons.count("queue full") == 3  # jobs 3..5 find the two queue places taken
    assert st["finished"] == 2


def test_continuous_batching_joins_running_set():
    """A job arriving while another runs joins it at a chunk boundary; the
    first keeps its own step count; uneven lengths finish independently."""
    srv, be, _ = make(pool=10 ** 8, chunk=10)
    long = Job(0, Spec(64, 200), arrival=0.0, steps=200)
    short = Job(1, Spec(32, 15), arrival=0.003, steps=15)
    srv.run([long, short])
    assert short.admitted < long.done and short.done < long.done
    mixed = [b for b in be.batches if len(b) == 2]
    assert mixed, "the two jobs never shared a launch"
    assert sum(k for b in be.batches for s, k in b if s is short.spec) == 15
    assert sum(k for b in be.batches for s, k in b if s is long.spec) == 200


def test_time_limit_and_stats():
    srv, _, _ = make(pool=10 ** 8, chunk=50)
    jobs = poisson_jobs(200.0, 0.05, lambda rng: Spec(int(rng.choice([16, 24])), int(rng.integers(10, 60))), seed=3)
    assert jobs and all(jobs[i].arrival <= jobs[i + 1].arrival for i in range(len(jobs) - 1))
    st = srv.run(jobs)
    assert st["finished"] == len(jobs)
    assert st["p50_s"] <= st["p99_s"]
    assert st["mlups"] > 0


class FailingBackend(FakeBackend):
    """Jobs whose spec sets `fail_at` report an unstable health word once they
    have run that many steps."""

    def failed(self, sim):
        at = getattr(sim.spec, "fail_at", None)
        return "unstable" if at is not None and sim.done >= at else None


def test_unstable_job_is_retired_as_failed():
    c = Clock()
    be = FailingBackend(c)
    srv = Server(be, 10 ** 7, chunk=10, max_resident=8, queue_cap=100, clock=c, sleep=c.sleep)
    jobs = [Job(i, Spec(16, 50), arrival=0.0, steps=50) for i in range(4)]
    jobs[2].spec.fail_at = 20
    st = srv.run(jobs)
    assert st["finished"] == 3 and st["failed"] == 1 and st["unfinished"] == 0
    bad = srv.failed[0]
    assert bad.jid == 2 and bad.failed == "unstable" and bad.result is None
    assert be.live == set() and srv.used == 0  # its arena was released
    assert all(j.result["steps"] == 50 for j in srv.finished)


def test_bad_arguments():
    with pytest.raises(ValueError):
        Server(None, 0)


class HealthBackend(FakeBackend):
    """Results carry a health word: jobs whose spec sets `bad_health` finish
    with it; jobs whose spec sets `wall_speed` above 0.3 are refused."""

    def admissible(self, spec):
        v = getattr(spec, "wall_speed", 0.0)
        return "wall speed above the low-Mach bound" if v > 0.3 else None

    def result(self, sim, spec):
        return {"steps": sim.done, "health": getattr(spec, "bad_health", 0)}


def test_flagged_result_and_inadmissible_job_are_not_goodput():
    """A job that ends with a non-zero health word is counted as failed (not in
    goodput or latency); a job whose walls move faster than the low-Mach bound
    is rejected at arrival and never takes a slot."""
    c = Clock()
    be = HealthBackend(c)
    srv = Server(be, 10 ** 7, chunk=10, max_resident=8, queue_cap=100, clock=c, sleep=c.sleep)
    jobs = [Job(i, Spec(16, 30), arrival=0.0, steps=30) for i in range(4)]
    jobs[1].spec.bad_health = 0x4
    jobs[3].spec.wall_speed = 0.315
    st = srv.run(jobs)
    assert st["finished"] == 2 and st["failed"] == 1 and st["rejected"] == 1
    assert srv.failed[0].jid == 1 and srv.failed[0].failed == "health word 0x4"
    assert jobs[3].rejected == "wall speed above the low-Mach bound" and jobs[3].admitted is None
    assert st["goodput_jobs_s"] == 2 / st["wall_s"]
    assert be.live == set() and srv.used == 0

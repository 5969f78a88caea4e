"""Serving loop on the GPU: jobs arriving at different times share batched
launches (continuous batching), and every job's result is bitwise the one it
gets when run alone."""
import numpy as np
import pytest

from paper_1704_04551_amd import ibl
from paper_1704_04551_amd import workloads as W
from paper_1704_04551_amd.serve import GpuBackend, Job, Server

pytestmark = pytest.mark.gpu


def _jobs():
    rng = np.random.default_rng(1005)
    jobs = []
    # three jobs at once, then arrivals while they run (and one once the
    # first wave has likely drained)
    arrivals = (0.0, 0.0, 0.0, 0.002, 0.005, 0.05)
    for i, t in enumerate(arrivals):
        spec = W.job_served(rng, edges=(32, 40, 48), steps=(60, 200))
        jobs.append(Job(i, spec, arrival=t, steps=int(spec.steps)))
    return jobs


def test_served_results_equal_alone():
    jobs = _jobs()
    srv = Server(GpuBackend("f32"), pool_bytes=1 << 32, chunk=10, max_resident=4)
    try:
        st = srv.run(jobs, time_limit=120)
    finally:
        srv.close()
    print("serve stats", st)
    assert st["finished"] == len(jobs) and st["rejected"] == 0
    assert st["max_concurrent"] >= 2, "jobs never overlapped on the device"
    for j in jobs:
        alone = ibl.Sim.from_spec(j.spec, storage="f32")
        alone.step(j.steps)
        alone.sync()
        mass, mom, health = alone.conservation()
        assert j.result["steps"] == j.steps == alone.step_count
        assert j.result["health"] == health == 0
        assert j.result["mass"] == mass
        for m in range(len(j.spec.capsules)):
            assert np.array_equal(j.result["X"][m], alone.nodes(m)[0]), (j.jid, m)
        alone.close()

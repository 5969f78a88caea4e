"""Serving loop: continuous batching of independent IB-LBM jobs on one GPU.

Jobs (``workloads.SimSpec``) arrive over time.  The server keeps a resident
set of simulations in device memory and advances all of them together, one
batched launch sequence (``ibl_batch_step``: one launch per kernel phase over
the flattened work list of every resident simulation, replayed as HIP graphs)
per *chunk* of steps.  At every chunk boundary it

1. retires the jobs that finished: reads their node positions, health word
   and conservation sums back to the host, then frees their device arena;
   a job whose health word reports an unstable or invalid state (non-finite
   values, rho <= 0, a fluid velocity above 0.3, a node outside the lattice;
   the timestep latches these per cell) is retired at once as failed, and so
   is a finished job whose final health word is not clean: failed jobs count
   neither in goodput nor in latency;
2. admits queued jobs, first come first served, while their footprint
   (``ibl_sim_bytes``) fits in the free part of the memory pool and a slot is
   free; a job that can never fit, or whose walls move faster than the
   low-Mach bound, is rejected, and arrivals beyond the queue bound are
   rejected on arrival;
3. launches the next chunk: each resident job advances min(chunk, steps
   left), so jobs of different lengths finish at their own step counts.

While a chunk runs, the host creates the simulations of the jobs that
arrived (their initialisation runs on their own streams); the batch stream
waits for it before the next chunk.  A job's arithmetic does not depend on
what else is resident (every kernel computes a simulation's cells and nodes
from its own state only, in a fixed order), so its result is bitwise the
same alone and in any mix.

Timing is wall-clock: latency = completion (result on the host) - arrival.
The backend is pluggable so the scheduling logic runs without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, List, Optional

import numpy as np

from . import workloads as W


@dataclasses.dataclass
class Job:
    jid: int
    spec: object               # workloads.SimSpec
    arrival: float             # seconds since the start of the run
    steps: int
    left: int = 0
    footprint: int = 0
    admitted: Optional[float] = None
    done: Optional[float] = None
    rejected: Optional[str] = None
    failed: Optional[str] = None   # why a resident job was stopped (its health word)
    result: Optional[dict] = None
    handle: object = None      # backend simulation while resident

    @property
    def cells(self) -> int:
        n = self.spec.n
        return int(n[0]) * int(n[1]) * int(n[2])

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class GpuBackend:
    """Resident simulations through the C-ABI (libibl.so).  `skin` is the
    candidate-list skin of every job (1 by default: served jobs are small
    suspensions, where keeping the lists between rebuilds pays)."""

    def __init__(self, storage="f32", device="cuda:0", skin=1):
        from . import ibl
        self.ibl = ibl
        self.storage = storage
        self.device = device
        self.skin = int(skin)
        self._batch = None
        self._members = ()     # the batch's simulations (they must outlive it)

    # lattice Boltzmann is valid at low Mach number only: the step flags any
    # fluid velocity above this bound (health word), so a job whose walls move
    # faster is refused at admission rather than run to a flagged result
    MACH_BOUND = 0.3

    def admissible(self, spec) -> Optional[str]:
        vmax = 0.0
        for a in range(3):
            if spec.wall[a]:
                vmax = max(vmax, float(np.linalg.norm(spec.u_lo[a])), float(np.linalg.norm(spec.u_hi[a])))
        if vmax > self.MACH_BOUND:
            return "wall speed %.3g above the low-Mach bound %.1f" % (vmax, self.MACH_BOUND)
        return None

    def footprint(self, spec) -> int:
        ibl = self.ibl
        groups = W.template_groups(spec)
        tn = sum(spec.capsules[g[0]].x.shape[0] for g in groups)
        te = sum(3 * spec.capsules[g[0]].tris.shape[0] // 2 for g in groups)
        desc = ibl.make_desc(spec.n, spec.tau, spec.g_body, spec.wall, spec.u_lo, spec.u_hi,
                             self.storage, spec.delta, spec.init_profile, max_nodes=spec.nodes,
                             max_meshes=len(spec.capsules), max_templates=len(groups),
                             max_template_nodes=tn, max_template_edges=te, skin=self.skin)
        return ibl.sim_bytes(desc)

    def create(self, spec):
        return self.ibl.Sim.from_spec(spec, storage=self.storage, device=self.device, skin=self.skin)

    def step(self, sims, steps):
        if self._batch is None or len(sims) != len(self._members) or any(
                a is not b for a, b in zip(sims, self._members)):
            self._drop_batch()
            self._batch = self.ibl.Batch(sims)
            self._members = tuple(sims)
        self._batch.step(np.asarray(steps, np.int64))

    def _drop_batch(self):
        if self._batch is not None:
            self._batch.close()
        self._batch = None
        self._members = ()

    def wait(self, sims):
        if sims:  # one stream for the batch; health is checked per job by failed()
            sims[0].sync_status()

    def failed(self, sim) -> Optional[str]:
        st = sim.sync_status()
        if st == 0:
            return None
        why = {-4: "invalid state", -5: "unstable"}.get(st, "error %d" % st)
        try:  # the latched health bits (a rare path: one reduction)
            why += " (health 0x%x)" % sim.conservation()[2]
        except Exception:  # the reduction reports the same error: the bits stay unknown
            pass
        return why

    def result(self, sim, spec) -> dict:
        mass, mom, health = sim.conservation()
        X = [sim.nodes(m)[0] for m in range(len(spec.capsules))]
        return {"X": X, "mass": mass, "momentum": mom, "health": health, "steps": sim.step_count}

    def release(self, sim):
        if any(sim is m for m in self._members):
            self._drop_batch()  # a batch must not outlive its simulations
        sim.close()
        sim.arena = None

    def close(self):
        self._drop_batch()


class Server:
    """Continuous-batching server over one backend (see the module docstring).

    pool_bytes   device memory the resident set may hold
    chunk        steps per batched launch sequence (admission granularity)
    max_resident resident simulations at most (slots)
    queue_cap    queued jobs at most; later arrivals are rejected
    """

    def __init__(self, backend, pool_bytes: int, chunk: int = 200, max_resident: int = 64,
                 queue_cap: int = 256, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        if chunk <= 0 or max_resident <= 0 or pool_bytes <= 0:
            raise ValueError("chunk, max_resident and pool_bytes must be positive")
        self.be = backend
        self.pool = int(pool_bytes)
        self.chunk = int(chunk)
        self.max_resident = int(max_resident)
        self.queue_cap = int(queue_cap)
        self.clock = clock
        self.sleep = sleep
        self.queue: collections.deque = collections.deque()
        self.resident: List[Job] = []
        self.finished: List[Job] = []
        self.rejected: List[Job] = []
        self.failed: List[Job] = []
        self.used = 0
        self.peak_used = 0
        self.cell_steps = 0
        self.chunks = 0
        self.max_concurrent = 0

    # -- bookkeeping -------------------------------------------------------
    def _offer(self, job: Job):
        job.left = job.steps
        job.footprint = self.be.footprint(job.spec)
        check = getattr(self.be, "admissible", None)
        why = check(job.spec) if check is not None else None
        if why is not None:
            job.rejected = why
            self.rejected.append(job)
        elif job.footprint > self.pool:
            job.rejected = "larger than the pool"
            self.rejected.append(job)
        elif len(self.queue) >= self.queue_cap:
            job.rejected = "queue full"
            self.rejected.append(job)
        else:
            self.queue.append(job)

    def _admit(self, now: float):
        while (self.queue and len(self.resident) < self.max_resident
               and self.used + self.queue[0].footprint <= self.pool):
            job = self.queue.popleft()
            job.handle = self.be.create(job.spec)
            job.admitted = now
            self.used += job.footprint
            self.peak_used = max(self.peak_used, self.used)
            self.resident.append(job)

    def _retire(self, t0: float):
        keep = []
        check = getattr(self.be, "failed", None)
        for job in self.resident:
            why = check(job.handle) if check is not None else None
            if why is not None:
                job.failed = why
                self.be.release(job.handle)
                job.handle = None
                self.used -= job.footprint
                job.done = self.clock() - t0
                self.failed.append(job)
                continue
            if job.left > 0:
                keep.append(job)
                continue
            job.result = self.be.result(job.handle, job.spec)
            self.be.release(job.handle)
            job.handle = None
            self.used -= job.footprint
            job.done = self.clock() - t0
            if job.result.get("health", 0):
                # the library flagged the final state (unstable, out of range):
                # not a result; it counts neither in goodput nor in latency
                job.failed = "health word 0x%x" % job.result["health"]
                self.failed.append(job)
            else:
                self.finished.append(job)
        self.resident = keep

    # -- the loop -----------------------------------------------------------
    def run(self, jobs: List[Job], time_limit: Optional[float] = None) -> dict:
        """Serve `jobs` (sorted by arrival time, seconds from now) to the
        end, or until `time_limit` seconds have passed (jobs still queued or
        resident then count as unfinished)."""
        pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
        t0 = self.clock()
        while pending or self.queue or self.resident:
            now = self.clock() - t0
            if time_limit is not None and now > time_limit:
                break
            while pending and pending[0].arrival <= now:
                self._offer(pending.popleft())
            self._admit(now)
            if not self.resident:
                if pending:  # idle until the next arrival
                    self.sleep(max(0.0, min(pending[0].arrival - now, 0.01)))
                continue
            running = list(self.resident)
            self.max_concurrent = max(self.max_concurrent, len(running))
            sims = [j.handle for j in running]
            steps = [min(self.chunk, j.left) for j in running]
            self.be.step(sims, steps)
            # host work overlapping the chunk: take in arrivals and build the
            # simulations of those that fit (they join at the next boundary)
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                self._offer(pending.popleft())
            self._admit(now)
            self.be.wait(sims)
            for j, k in zip(running, steps):
                j.left -= k
                self.cell_steps += j.cells * k
            self.chunks += 1
            self._retire(t0)
        wall = self.clock() - t0
        return self.stats(wall, not_arrived=len(pending))

    def stats(self, wall: float, not_arrived: int = 0) -> dict:
        lat = sorted(j.latency for j in self.finished)
        def pct(p):
            if not lat:
                return None
            return lat[min(len(lat) - 1, max(0, math.ceil(p / 100.0 * len(lat)) - 1))]
        return {
            "wall_s": wall,
            "finished": len(self.finished),
            "rejected": len(self.rejected),
            "failed": len(self.failed),
            "unfinished": len(self.queue) + len(self.resident) + not_arrived,
            "p50_s": pct(50),
            "p99_s": pct(99),
            "mlups": self.cell_steps / wall / 1e6 if wall > 0 else 0.0,
            "goodput_jobs_s": len(self.finished) / wall if wall > 0 else 0.0,
            "peak_pool_bytes": self.peak_used,
            "chunks": self.chunks,
            "max_concurrent": self.max_concurrent,
            "failed_reasons": dict(collections.Counter(str(j.failed) for j in self.failed)),
            "rejected_reasons": dict(collections.Counter(str(j.rejected) for j in self.rejected)),
        }

    def close(self):
        for job in self.resident:
            self.be.release(job.handle)
            job.handle = None
        self.resident = []
        self.be.close()


def poisson_jobs(rate: float, duration: float, make_spec, seed: int) -> List[Job]:
    """Arrivals of a Poisson process of `rate` jobs/s over `duration` s;
    make_spec(rng) draws each job's workload."""
    rng = np.random.default_rng(seed)
    t, jobs = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            return jobs
        spec = make_spec(rng)
        jobs.append(Job(jid=len(jobs), spec=spec, arrival=t, steps=int(spec.steps)))

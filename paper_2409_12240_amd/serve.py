"""Continuous-batching anneal server over the pool ABI.

Annealing jobs (an Ising instance, a bond dimension chi, a schedule T, dt)
arrive over time.  One pool per chi keeps the admitted jobs' tensor
networks and BP messages resident in HBM; the pool's budget bounds the
HBM footprint of the resident jobs (gtqa_footprint_bytes).  Every pool
iteration advances all resident jobs of that pool by one Trotter step in
one set of launches, each job at its own step index and angles; a job that
finishes is read out and released, and waiting jobs are admitted as soon as
budget and slots allow (first come, first served per chi).  Pools of
different chi run in their own host threads on their own HIP streams, so
their launches overlap on the device.

A job's result does not depend on which other jobs share its launches: all
per-instance arithmetic, including BP's stop decision, is independent of
the batch composition.
"""

from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import gtqa


@dataclass
class Job:
    job_id: int
    instance: object
    chi: int
    T: float
    dt: float
    arrival: float = 0.0            # seconds after the server clock starts
    # filled by the server
    admitted: float | None = None
    finished: float | None = None
    result: dict | None = None
    steps: int = 0
    k: int = 0
    slot: int = -1
    _tz: np.ndarray | None = field(default=None, repr=False)
    _tx: np.ndarray | None = field(default=None, repr=False)

    def schedule(self):
        if self._tz is None:
            K = int(round(self.T / self.dt))
            k = np.arange(1, K + 1, dtype=np.float64)
            self._tz = self.dt * k / K
            self._tx = self.dt * (K - k) / K
            self.steps = K
        return self._tz, self._tx

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival

    @property
    def gate_updates(self):
        return self.steps * int(self.instance.n_edges)


class _PoolWorker:
    def __init__(self, chi, precision, budget_bytes, max_vertices, max_slots, clock, device_factory,
                 on_done=None, **opts):
        self.chi = chi
        self.on_done = on_done
        self.precision = precision
        self.budget = budget_bytes
        self.max_vertices = max_vertices
        self.max_slots = max_slots
        self.clock = clock
        self.device_factory = device_factory
        self.opts = opts
        self.queue: deque[Job] = deque()
        self.lock = threading.Lock()
        self.resident: dict[int, Job] = {}
        self.done: list[Job] = []
        self.iterations = 0
        self.error: BaseException | None = None

    def submit(self, job: Job):
        with self.lock:
            self.queue.append(job)

    def _admit(self, pool):
        while True:
            with self.lock:
                if not self.queue or self.queue[0].arrival > self.clock():
                    return
                job = self.queue[0]
            slot = pool.admit(job.instance)
            if slot < 0:
                return                      # budget or capacity full: wait for a release
            with self.lock:
                self.queue.popleft()
            job.slot = slot
            job.admitted = self.clock()
            job.schedule()
            self.resident[slot] = job

    def run(self, stop_when_idle: threading.Event):
        try:
            dev = self.device_factory()
            pool = gtqa.Pool(chi=self.chi, precision=self.precision, max_vertices=self.max_vertices,
                             max_slots=self.max_slots, budget_bytes=self.budget, device=dev, **self.opts)
            try:
                while True:
                    self._admit(pool)
                    if not self.resident:
                        with self.lock:
                            empty = not self.queue
                        if empty and stop_when_idle.is_set():
                            return
                        time.sleep(0.0005)
                        continue
                    slots = np.array(sorted(self.resident), dtype=np.int32)
                    tz = np.empty(slots.size)
                    tx = np.empty(slots.size)
                    for i, s in enumerate(slots):
                        j = self.resident[int(s)]
                        a, b = j.schedule()
                        tz[i] = a[j.k]
                        tx[i] = b[j.k]
                    pool.step(slots, tz, tx)
                    self.iterations += 1
                    for s in slots:
                        j = self.resident[int(s)]
                        j.k += 1
                        if j.k == j.steps:
                            j.result = pool.readout(int(s))
                            j.finished = self.clock()
                            pool.release(int(s))
                            del self.resident[int(s)]
                            self.done.append(j)
                            if self.on_done is not None:
                                self.on_done(j)
            finally:
                pool.close()
        except BaseException as exc:          # surfaced by Server.run
            self.error = exc


class Server:
    """Runs a list of jobs with arrival times and returns them completed."""

    def __init__(self, precision="mixed", budget_bytes=8 << 30, max_vertices=1 << 18, max_slots=512,
                 device_factory=None, on_done=None, **opts):
        self.precision = precision
        self.on_done = on_done
        self.budget = budget_bytes
        self.max_vertices = max_vertices
        self.max_slots = max_slots
        self.device_factory = device_factory or self._torch_device
        self.opts = opts

    @staticmethod
    def _torch_device():
        # one stream per pool: the pools' launches overlap on the device
        return gtqa.TorchDevice(stream="own")

    def run(self, jobs, timeout_s: float = 600.0):
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0      # noqa: E731
        workers = {}
        for chi in sorted({j.chi for j in jobs}):
            workers[chi] = _PoolWorker(chi, self.precision, self.budget, self.max_vertices, self.max_slots,
                                       clock, self.device_factory, on_done=self.on_done, **self.opts)
        for j in sorted(jobs, key=lambda j: (j.arrival, j.job_id)):
            workers[j.chi].submit(j)
        stop = threading.Event()
        stop.set()                                    # all jobs are already queued
        threads = [threading.Thread(target=w.run, args=(stop,), daemon=True) for w in workers.values()]
        for th in threads:
            th.start()
        for th in threads:
            th.join(timeout=max(1.0, timeout_s - clock()))
        for w in workers.values():
            if w.error is not None:
                raise w.error
        if any(th.is_alive() for th in threads):
            raise TimeoutError("serving run did not finish")
        wall = clock()
        done = [j for w in workers.values() for j in w.done]
        lat = np.array([j.latency for j in done])
        return {
            "jobs": len(done),
            "wall_s": wall,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "gate_updates_per_s": sum(j.gate_updates for j in done) / wall if wall > 0 else None,
            "iterations": {chi: w.iterations for chi, w in workers.items()},
            "completed": done,
        }


def poisson_jobs(seed: int, count: int, rate_per_s: float, n_range=(100, 2000), chis=(4, 8),
                 steps_range=(200, 2000), dt=0.05, first_id=0):
    """Synthetic job stream: Poisson arrivals at `rate_per_s`, n = 2*U{n0/2..n1/2},
    chi uniform over `chis`, steps uniform over `steps_range` (T = steps*dt);
    job j's instance uses seed 3_000_000 + j."""
    from synthetic import SplitMix64, random_regular_instance
    rng = SplitMix64(seed)
    t = 0.0
    jobs = []
    for j in range(count):
        u = (rng.next() >> 11) * 2.0 ** -53
        t += -np.log1p(-u) / rate_per_s
        n = 2 * (n_range[0] // 2 + rng.bounded(n_range[1] // 2 - n_range[0] // 2 + 1))
        chi = chis[rng.bounded(len(chis))]
        steps = steps_range[0] + rng.bounded(steps_range[1] - steps_range[0] + 1)
        inst = random_regular_instance(3_000_000 + first_id + j, n)
        jobs.append(Job(job_id=first_id + j, instance=inst, chi=chi, T=steps * dt, dt=dt, arrival=t))
    return jobs


def rate_sweep(fractions=(0.25, 0.5, 0.75, 0.9, 1.1), jobs_per_rate=20, chis=(4, 8), precision="mixed",
               budget_bytes=16 << 30, small_budget_jobs=3, seed=3000, n_range=(100, 2000),
               steps_range=(200, 2000), dt=0.05, timeout_s=900.0, progress=None):
    """Latency against load.  Capacity mu (jobs/s) is measured by a burst:
    every job of a stream present at t = 0, mu = jobs / wall.  Then, for each
    fraction rho, a Poisson stream at rate rho * mu (its own jobs) is served
    and p50/p99 latency (completion - arrival) and gate-updates/s reported.
    A last run at rho = 0.5 with an admission budget of `small_budget_jobs`
    of the largest job's footprint forces queueing."""
    burst = poisson_jobs(seed=seed, count=jobs_per_rate, rate_per_s=1e9, n_range=n_range, chis=chis,
                         steps_range=steps_range, dt=dt)
    for j in burst:
        j.arrival = 0.0
    def done(j):
        if progress:
            progress(f"  job {j.job_id} (n={j.instance.n}, chi={j.chi}, {j.steps} steps) done, "
                     f"latency {j.latency:.2f} s")

    cap = Server(precision=precision, budget_bytes=budget_bytes, max_vertices=1 << 18, max_slots=512,
                 on_done=done).run(burst, timeout_s=timeout_s)
    mu = cap["jobs"] / cap["wall_s"]
    if progress:
        progress(f"serving capacity: {mu:.3f} jobs/s ({cap['wall_s']:.1f} s burst)")
    rows = []

    def one(rho, budget, first_id, label):
        jobs = poisson_jobs(seed=seed + 1 + first_id, count=jobs_per_rate, rate_per_s=rho * mu, n_range=n_range,
                            chis=chis, steps_range=steps_range, dt=dt, first_id=first_id)
        out = Server(precision=precision, budget_bytes=budget, max_vertices=1 << 18, max_slots=512,
                     on_done=done).run(jobs, timeout_s=timeout_s)
        waits = [j.admitted - j.arrival for j in out["completed"]]
        rows.append({"run": label, "rho": rho, "arrival_rate_per_s": round(rho * mu, 4), "jobs": out["jobs"],
                     "budget_bytes": budget, "wall_s": round(out["wall_s"], 3),
                     "p50_latency_s": round(out["p50_latency_s"], 4), "p99_latency_s": round(out["p99_latency_s"], 4),
                     "max_admission_wait_s": round(max(waits), 4),
                     "gate_updates_per_s": round(out["gate_updates_per_s"], 1)})
        if progress:
            progress(f"serving {label} rho={rho}: p50 {out['p50_latency_s']:.2f} s, p99 {out['p99_latency_s']:.2f} s")

    for i, rho in enumerate(fractions):
        one(rho, budget_bytes, 1000 * (i + 1), "rate")
    from . import gtqa as _g
    prec = 1 if precision == "mixed" else 0
    big = max(_g.gtqa_footprint_bytes(n_range[1], 3 * n_range[1] // 2, max(chis), prec), 1)
    one(0.5, small_budget_jobs * big, 1000 * (len(fractions) + 1), "small_budget")
    return {"capacity_jobs_per_s": round(mu, 4), "capacity_gate_updates_per_s": round(cap["gate_updates_per_s"], 1),
            "capacity_wall_s": round(cap["wall_s"], 3), "jobs_per_run": jobs_per_rate, "chis": list(chis),
            "precision": precision, "runs": rows}

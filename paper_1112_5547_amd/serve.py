"""Serving loop: continuous batching of Shan-Chen lattice jobs on one GPU.

Requests (drop / spinodal jobs of different lattice types, sizes and step
counts) arrive over time.  The loop:

* queues every request whose arrival time has passed;
* admits queued jobs first-fit while the device-memory budget and the member
  slots allow (a job's state stays resident on the device until it finishes);
* advances all resident jobs together in epochs of ``epoch_steps`` steps with
  one batch launch per epoch (persistent, fused or per-lattice form);
* while an epoch runs on the device, prepares the next admissions on the host
  (input fields, lattice creation, upload); jobs that arrive mid-epoch join at
  the next epoch boundary;
* reads out finished jobs (FP64 totals, optional fields), frees their memory
  and reports latency = completion - arrival.

Each job's result is bitwise the one it would have alone: a batch runs the
same per-site device code for every member.

The loop talks to a backend (the GPU library by default) and a clock, so the
admission and accounting logic also runs on the CPU with an oracle-driven
backend and a simulated clock.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class JobResult:
    job_id: int
    lattice: int
    shape: tuple
    steps: int
    arrival: float
    admitted: float
    completed: float
    status: str                 # "ok" or "nonfinite"
    totals: dict
    populations: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.completed - self.arrival

    @property
    def site_updates(self) -> float:
        return float(np.prod(self.shape)) * self.steps


@dataclasses.dataclass
class ServeReport:
    results: List[JobResult]
    makespan: float
    epochs: int
    queue_depth: List[tuple]    # (time, queued, resident)
    refused: int                # jobs that can never fit the budget

    def latencies(self) -> np.ndarray:
        return np.array([r.latency for r in self.results])

    def summary(self) -> dict:
        lat = self.latencies()
        su = sum(r.site_updates for r in self.results)
        return {
            "jobs": len(self.results),
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_latency_s": float(lat.mean()) if len(lat) else None,
            "makespan_s": self.makespan,
            "aggregate_mlups": su / self.makespan / 1e6 if self.makespan > 0 else None,
            "epochs": self.epochs,
            "max_queue": max((q for _, q, _ in self.queue_depth), default=0),
            "max_resident": max((r for _, _, r in self.queue_depth), default=0),
            "nonfinite": sum(r.status != "ok" for r in self.results),
            "nonfinite_jobs": [r.job_id for r in self.results if r.status != "ok"],
            "refused": self.refused,
        }


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep_until(self, t: float):
        dt = t - self.now()
        if dt > 0:
            time.sleep(dt)


class GpuBackend:
    """The HIP library: lattices with torch arenas, one Batch."""

    def __init__(self, precision: str = "fp32_shifted", tuned: bool = True):
        self.precision = precision
        self.tuned = tuned

    def bytes_needed(self, job) -> int:
        from .lattice import bytes_needed
        return bytes_needed(job.lattice, job.nx, job.ny, job.nz, self.precision)

    def make_lattice(self, job):
        from .lattice import Lattice
        lat = Lattice(job.lattice, job.nx, job.ny, job.nz, tau_A=job.tau, G=job.G,
                      precision=self.precision)
        if self.tuned:  # solo launches use the autotuned kernel (batches their own tiles)
            from . import autotune
            autotune.apply(lat)
        fl = job.fields()
        lat.init(fl.rho_A, fl.rho_B)
        if fl.radius > 0:
            lat.set_probe(*fl.centre, fl.radius)
        return lat

    def make_batch(self, budget: int):
        from .batch import Batch
        return Batch(hbm_budget=budget)

    def finish(self, lat, keep_populations: bool):
        T = lat.totals(allow_nonfinite=True)
        pops = lat.get_populations() if keep_populations else None
        return T, pops

    def release(self, lat):
        lat.close()


class Server:
    def __init__(self, hbm_budget: int = 0, *, epoch_steps: int = 200, mode: str = "persistent",
                 max_resident: int = 256, backend=None, clock=None,
                 keep_populations: bool = False, admit_hook: Optional[Callable] = None,
                 tiles: Optional[dict] = None):
        self.budget = int(hbm_budget)
        self.epoch_steps = int(epoch_steps)
        self.mode = mode
        self.max_resident = int(max_resident)
        self.backend = backend if backend is not None else GpuBackend()
        self.clock = clock if clock is not None else WallClock()
        self.keep_populations = keep_populations
        self.admit_hook = admit_hook
        self.tiles = tiles

    def run(self, jobs: Sequence) -> ServeReport:
        be, clock = self.backend, self.clock
        pending = sorted(jobs, key=lambda j: j.arrival)
        queue: List = []
        resident: Dict[int, tuple] = {}       # job_id -> (job, lattice, admitted_at)
        used = 0
        results: List[JobResult] = []
        depth: List[tuple] = []
        refused = 0
        batch = be.make_batch(self.budget)
        if self.tiles:
            batch.set_tiles(self.tiles["tx9"], self.tiles["tx19"], self.tiles["ty19"],
                            self.tiles["mb9"], self.tiles["mb19"])
        epochs = 0
        need = {j.job_id: be.bytes_needed(j) for j in pending}

        def admit():
            nonlocal used, refused
            now = clock.now()
            while pending and pending[0].arrival <= now:
                queue.append(pending.pop(0))
            k = 0
            while k < len(queue):
                job = queue[k]
                if self.budget and need[job.job_id] > self.budget:
                    queue.pop(k)           # can never fit: report, do not block the queue
                    refused += 1
                    continue
                fits = not self.budget or used + need[job.job_id] <= self.budget
                if len(resident) < self.max_resident and fits:
                    lat = be.make_lattice(job)
                    if not batch.add(lat, job.steps):
                        be.release(lat)
                        k += 1
                        continue
                    used += need[job.job_id]
                    resident[job.job_id] = (job, lat, clock.now())
                    queue.pop(k)
                    if self.admit_hook:
                        self.admit_hook(job, clock.now())
                else:
                    k += 1
            depth.append((clock.now(), len(queue), len(resident)))

        admit()
        while pending or queue or resident:
            if not resident:
                if queue:
                    admit()
                    if not resident:       # nothing fits and nothing runs: wait for arrivals
                        if pending:
                            clock.sleep_until(pending[0].arrival)
                            admit()
                        else:
                            break
                    continue
                clock.sleep_until(pending[0].arrival)
                admit()
                continue
            batch.run(self.epoch_steps, self.mode)   # asynchronous on the device
            epochs += 1
            admit()                                    # host work overlaps the epoch
            done = batch.poll()                        # waits for the epoch
            t_done = clock.now()
            for lat in done:
                jid = next(j for j, (_, l, _) in resident.items() if l is lat)
                job, _, t_adm = resident.pop(jid)
                batch.remove(lat)
                T, pops = be.finish(lat, self.keep_populations)
                status = "ok" if T.get("n_nonfinite", 0) == 0 else "nonfinite"
                results.append(JobResult(job.job_id, job.lattice, (job.nz, job.ny, job.nx),
                                         job.steps, job.arrival, t_adm, t_done, status, T, pops))
                be.release(lat)
                used -= need[jid]
            if done:
                admit()
        makespan = clock.now()
        if hasattr(batch, "close"):
            batch.close()
        results.sort(key=lambda r: r.job_id)
        return ServeReport(results, makespan, epochs, depth, refused)


def offered_rate(jobs, capacity_mlups: float, load: float = 0.7) -> float:
    """Arrival rate (jobs/s) at which the stream offers `load` x capacity."""
    mean_work = np.mean([j.sites * j.steps for j in jobs]) / 1e6
    return load * capacity_mlups / mean_work


def sequential_baseline(jobs, backend=None, clock=None) -> dict:
    """Jobs run one after another, each alone (one lattice per launch),
    in arrival order: the reference the served figures are compared with."""
    be = backend if backend is not None else GpuBackend()
    clock = clock if clock is not None else WallClock()
    lat_s = []
    su = 0.0
    for job in sorted(jobs, key=lambda j: j.arrival):
        clock.sleep_until(job.arrival)
        lat = be.make_lattice(job)
        lat.step(job.steps)
        lat.sync()
        be.finish(lat, False)
        be.release(lat)
        lat_s.append(clock.now() - job.arrival)
        su += job.sites * job.steps
    t = clock.now()
    return {"p50_latency_s": float(np.percentile(lat_s, 50)),
            "p99_latency_s": float(np.percentile(lat_s, 99)),
            "makespan_s": t, "aggregate_mlups": su / t / 1e6}

"""Serving loop: continuous batching of Shan-Chen lattice jobs on one GPU.

Requests (drop / spinodal jobs of different lattice types, sizes and step
counts) arrive over time.  The loop:

* queues every request whose arrival time has passed;
* admits queued jobs first-fit while the device-memory budget and the member
  slots allow (a job's state stays resident on the device until it finishes);
* advances resident jobs in epochs of ``epoch_steps`` steps with one batch
  launch per epoch (fused, persistent or per-lattice form).  Which resident
  jobs an epoch advances is the scheduling policy:
    - ``"srpt"`` (default): shortest remaining work first.  Resident jobs are
      ordered by remaining work (priced as below) and taken until their lattices hold
      ``sat_sites`` sites, the size at which one batch launch keeps the whole
      device busy; the rest wait, resident, for a later epoch.  A lattice of
      ``sat_sites`` or more never joins a batch: the prefix stops before it,
      and it runs alone once it is first in order.  A small job
      then never pays the step time of a large one, and a large job still runs
      at full rate once it is the shortest.  An epoch whose only member fills
      the device by itself (at least ``sat_sites`` sites) steps that lattice
      alone with its own tuned kernel instead of the batch launch, and so
      does any lone member (``solo_alone``, the default).  Work is priced
      in seconds of solo service: a job's remaining steps times its lattice
      shape's measured solo step time (``step_seconds``, keyed by
      (lattice, nx, ny, nz)), or its remaining site updates at
      ``nominal_rate`` for shapes without one.  With ``aging`` > 0 the order
      key is the remaining work minus ``aging`` times the time
      the job has spent in the system, so that a large job cannot be passed
      over indefinitely by a stream of smaller ones.  With ``guard`` set,
      every job also carries a deadline, the completion time it would have
      under one-job-at-a-time service in arrival order (at those prices),
      and the SRPT order only runs on the slack of the deadlines: before
      each epoch the server takes the resident jobs in deadline order and
      the least, over that order, of a job's deadline minus now minus the
      remaining work of it and of the jobs due before it.  While that slack
      exceeds ``guard`` seconds the epoch keeps the SRPT order; otherwise it
      serves the deadline order (earliest deadline first), which meets every
      deadline the slack still allows.  No job then finishes much later
      than it would have in arrival order (by about an epoch with a guard
      of 0 or more, by about an epoch plus |guard| with a negative one, the
      service prices being right), while small jobs overtake large ones
      whenever the deadlines leave room;
    - ``"all"``: every resident job advances every epoch (each job gets the
      same number of steps per epoch, whatever its size);
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
    deadline_epochs: int = 0    # epochs served in deadline order (guard)

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
            "deadline_epochs": self.deadline_epochs,
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
    def __init__(self, hbm_budget: int = 0, *, epoch_steps: int = 200, mode: str = "fused",
                 max_resident: int = 256, backend=None, clock=None,
                 keep_populations: bool = False, admit_hook: Optional[Callable] = None,
                 tiles: Optional[dict] = None, policy: str = "srpt",
                 sat_sites: int = 4_000_000, aging: float = 0.0,
                 nominal_rate: float = 1e10, solo_alone: bool = True,
                 guard: Optional[float] = None,
                 step_seconds: Optional[Dict[tuple, float]] = None):
        if policy not in ("srpt", "all"):
            raise ValueError(f"unknown scheduling policy {policy!r}")
        self.policy = policy
        self.sat_sites = int(sat_sites)
        self.aging = float(aging)
        self.solo_alone = bool(solo_alone)
        self.nominal_rate = float(nominal_rate)
        self.step_seconds = dict(step_seconds) if step_seconds else {}
        self.guard = None if guard is None else float(guard)
        self.budget = int(hbm_budget)
        self.epoch_steps = int(epoch_steps)
        self.mode = mode
        self.max_resident = int(max_resident)
        self.backend = backend if backend is not None else GpuBackend()
        self.clock = clock if clock is not None else WallClock()
        self.keep_populations = keep_populations
        self.admit_hook = admit_hook
        self.tiles = tiles

    def service_s(self, job, steps: int) -> float:
        """Seconds of `steps` steps of `job` served alone: its lattice shape's
        measured solo step time when known, else its site updates at the
        nominal rate."""
        t = self.step_seconds.get((job.lattice, job.nx, job.ny, job.nz))
        if t is not None:
            return steps * t
        return steps * job.sites / self.nominal_rate

    def run(self, jobs: Sequence) -> ServeReport:
        be, clock = self.backend, self.clock
        srpt = self.policy == "srpt"
        pending = sorted(jobs, key=lambda j: j.arrival)
        queue: List = []
        resident: Dict[int, tuple] = {}       # job_id -> (job, lattice, admitted_at)
        done_steps: Dict[int, int] = {}       # job_id -> steps advanced so far
        active: set = set()                   # job_ids that are members of the batch
        used = 0
        results: List[JobResult] = []
        depth: List[tuple] = []
        refused = 0
        # the server accounts the memory of every resident job; under SRPT the
        # batch only holds the jobs of the current epoch
        batch = be.make_batch(0 if srpt else self.budget)
        if self.tiles:
            batch.set_tiles(self.tiles["tx9"], self.tiles["tx19"], self.tiles["ty19"],
                            self.tiles["mb9"], self.tiles["mb19"])
        epochs = 0
        deadline_epochs = 0   # epochs the guard put in deadline order
        phase = None       # "deadline" when the guard put the epoch in deadline order
        need = {j.job_id: be.bytes_needed(j) for j in pending}
        # completion time of each job under one-job-at-a-time service in
        # arrival order (depends on earlier arrivals only)
        deadline: Dict[int, float] = {}
        v = 0.0
        for j in pending:
            v = max(v, j.arrival) + self.service_s(j, j.steps)
            deadline[j.job_id] = v

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
                    if not srpt:
                        if not batch.add(lat, job.steps):
                            be.release(lat)
                            k += 1
                            continue
                        active.add(job.job_id)
                    used += need[job.job_id]
                    resident[job.job_id] = (job, lat, clock.now())
                    done_steps[job.job_id] = 0
                    queue.pop(k)
                    if self.admit_hook:
                        self.admit_hook(job, clock.now())
                else:
                    k += 1
            depth.append((clock.now(), len(queue), len(resident)))

        def remaining(jid: int) -> int:
            return resident[jid][0].steps - done_steps[jid]

        def schedule() -> Optional[int]:
            """SRPT: the next epoch's members are the resident jobs with the
            least remaining work, taken until their sites reach sat_sites.
            Returns the job to step alone when it is the only member and fills
            the device by itself, else None (the batch runs the epoch)."""
            nonlocal phase
            phase = None
            if not srpt:
                return None
            now = clock.now()

            def key(j):
                job = resident[j][0]
                work_s = self.service_s(job, remaining(j))
                return (work_s - self.aging * (now - job.arrival), job.arrival, j)

            order = sorted(resident, key=key)
            if self.guard is not None:
                # slack of the earliest-deadline-first schedule of the resident
                # jobs: the least, over the deadline order, of a job's deadline
                # minus now minus the remaining work of it and of every job due
                # before it.  Above the guard an epoch in SRPT order can be
                # spared; at or below it the epoch serves the deadline order.
                by_deadline = sorted(resident, key=lambda j: (deadline[j], j))
                cum, slack = 0.0, float("inf")
                for j in by_deadline:
                    cum += self.service_s(resident[j][0], remaining(j))
                    slack = min(slack, deadline[j] - now - cum)
                if slack <= self.guard:
                    order, phase = by_deadline, "deadline"
            chosen, sites = [], 0
            for jid in order:
                n = resident[jid][0].sites
                if n >= self.sat_sites:
                    # a lattice that fills the device never shares a batch (every
                    # batch step would take its step time): it runs alone, once
                    # it is the first in order
                    if not chosen:
                        chosen, sites = [jid], n
                    break
                if chosen and sites >= self.sat_sites:
                    break
                chosen.append(jid)
                sites += n
            lone = len(chosen) == 1 and (self.solo_alone or sites >= self.sat_sites)
            solo = chosen[0] if lone else None
            keep = set() if solo is not None else set(chosen)
            for jid in sorted(active - keep):
                batch.remove(resident[jid][1])
                active.discard(jid)
            for jid in sorted(keep - active):
                batch.add(resident[jid][1], remaining(jid))
                active.add(jid)
            return solo

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
            solo = schedule()
            if solo is not None:
                lat = resident[solo][1]
                lat.step(min(self.epoch_steps, remaining(solo)))   # its own stream and kernel
                epochs += 1
                done_steps[solo] += min(self.epoch_steps, remaining(solo))
                admit()                                    # host work overlaps the epoch
                lat.sync()
                done = [lat] if remaining(solo) == 0 else []
            else:
                batch.run(self.epoch_steps, self.mode)   # asynchronous on the device
                epochs += 1
                for jid in active:
                    done_steps[jid] += min(self.epoch_steps, remaining(jid))
                admit()                                    # host work overlaps the epoch
                done = batch.poll()                        # waits for the epoch
            t_done = clock.now()
            if phase == "deadline":
                deadline_epochs += 1
            for lat in done:
                jid = next(j for j, (_, l, _) in resident.items() if l is lat)
                job, _, t_adm = resident.pop(jid)
                if jid in active:
                    batch.remove(lat)
                    active.discard(jid)
                done_steps.pop(jid)
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
        return ServeReport(results, makespan, epochs, depth, refused, deadline_epochs)


def solo_step_seconds(jobs, backend=None, *, warm: int = 32, timed: int = 64) -> Dict[tuple, float]:
    """Seconds per step of each distinct lattice shape of `jobs` run alone
    (one lattice per launch, the backend's tuned kernel), timed on the device
    after `warm` steps (which include any graph capture).  Keys are
    (lattice, nx, ny, nz)."""
    be = backend if backend is not None else GpuBackend()
    out: Dict[tuple, float] = {}
    for job in jobs:
        key = (job.lattice, job.nx, job.ny, job.nz)
        if key in out:
            continue
        lat = be.make_lattice(job)
        lat.step(warm)
        out[key] = lat.time_steps(timed) * 1e-3 / timed
        be.release(lat)
    return out


def solo_capacity(jobs, step_seconds: Dict[tuple, float]) -> float:
    """Site updates per second (in millions) of the job mix served one job at
    a time: total work over the sum of the jobs' solo service times."""
    work = sum(j.sites * j.steps for j in jobs)
    busy = sum(j.steps * step_seconds[(j.lattice, j.nx, j.ny, j.nz)] for j in jobs)
    return work / busy / 1e6


def batched_capacity(jobs, *, backend=None, clock=None, tiles: Optional[dict] = None,
                     epoch_steps: int = 250, step_fraction: float = 0.1,
                     sat_sites: int = 4_000_000) -> float:
    """Site updates per second (in millions) of the job mix served by the
    batching server with every job present from the start: the jobs'
    lattices with their step counts cut to `step_fraction` (at least one
    epoch), shortest remaining work first, total work over the time from the
    last admission (the lattices are created first) to the last completion."""
    short = [dataclasses.replace(j, arrival=0.0,
                                 steps=max(epoch_steps, int(j.steps * step_fraction)))
             for j in jobs]
    rep = Server(hbm_budget=0, epoch_steps=epoch_steps, mode="fused", backend=backend,
                 clock=clock, tiles=tiles, policy="srpt", sat_sites=sat_sites).run(short)
    start = max(r.admitted for r in rep.results)
    busy = max(r.completed for r in rep.results) - start
    return sum(j.sites * j.steps for j in short) / busy / 1e6


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
            "mean_latency_s": float(np.mean(lat_s)),
            "makespan_s": t, "aggregate_mlups": su / t / 1e6}

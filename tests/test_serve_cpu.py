"""Serving-loop logic on the CPU: an oracle-driven backend and a simulated
clock stand in for the GPU library, so admission by memory budget, epochs,
joins between epochs, scheduling (shortest remaining work first, or every
resident job each epoch), read-out, refusal and latency accounting are tested
without a device.  Results must equal each job's solo oracle run bitwise
(the backend advances every member with the same oracle code)."""
import numpy as np
import pytest

import oracle
import sc_inputs
from paper_1112_5547_amd.serve import Server, batched_capacity, offered_rate


class SimClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)

    def advance(self, dt):
        self.t += dt


class FakeLattice:
    def __init__(self, job, backend):
        self.job = job
        self.be = backend
        self.q = job.lattice
        self.shape = (job.nz, job.ny, job.nx)
        fl = job.fields()
        self.f = oracle.init(job.lattice, fl.rho_A, fl.rho_B)
        self.steps_done = 0

    def advance(self, n):
        if n > 0:
            self.f = oracle.run(self.f, self.job.tau, self.job.tau, self.job.G, n)
            self.steps_done += n

    def step(self, n):
        """A solo launch: same oracle arithmetic, the clock moves by its work."""
        self.advance(n)
        self.be.clock.advance(n * np.prod(self.shape) / self.be.capacity + 1e-4)
        self.be.log.append(("solo", self.job.job_id, n))

    def sync(self):
        pass


class FakeBatch:
    """Members advance by up to epoch steps per run; the clock moves by the
    epoch's site updates over a fixed capacity (site updates per second)."""

    def __init__(self, budget, clock, capacity, bytes_of, log):
        self.budget, self.clock, self.capacity = budget, clock, capacity
        self.bytes_of, self.log = bytes_of, log
        self.members = {}
        self.used = 0

    def add(self, lat, steps):
        b = self.bytes_of(lat.job)
        if self.budget and self.used + b > self.budget:
            return False
        self.members[id(lat)] = [lat, steps]
        self.used += b
        self.log.append(("used", self.used))
        return True

    def remove(self, lat):
        self.members.pop(id(lat))
        self.used -= self.bytes_of(lat.job)

    def run(self, epoch, mode):
        work = 0.0
        for m in self.members.values():
            k = min(epoch, m[1])
            m[0].advance(k)
            m[1] -= k
            work += k * np.prod(m[0].shape)
        self.clock.advance(work / self.capacity + 1e-4)
        self.log.append(("epoch", self.clock.now(), len(self.members)))
        self.log.append(("members", [m[0].job.job_id for m in self.members.values()]))

    def poll(self):
        return [m[0] for m in self.members.values() if m[1] == 0]


class FakeBackend:
    def __init__(self, clock, capacity=2e6):
        self.clock, self.capacity, self.log = clock, capacity, []

    def bytes_needed(self, job):
        return 2 * 2 * job.lattice * job.sites * 4       # FP32 ping-pong populations

    def make_lattice(self, job):
        return FakeLattice(job, self)

    def make_batch(self, budget):
        return FakeBatch(budget, self.clock, self.capacity, self.bytes_needed, self.log)

    def finish(self, lat, keep):
        rho = lat.f.sum(axis=1)
        bad = int((~np.isfinite(rho)).sum())
        return {"n_nonfinite": bad, "mass_A": float(rho[0].sum())}, (lat.f.copy() if keep else None)

    def release(self, lat):
        lat.f = None


def _jobs(n=10, seed=21, rate=40.0):
    return sc_inputs.serving_jobs(n, seed=seed, rate=rate, step_range=(5, 40), l2=(8, 20),
                                  l3=(4, 7), frac_3d=0.3)


def test_every_job_completes_with_its_solo_result():
    clock = SimClock()
    be = FakeBackend(clock)
    jobs = _jobs()
    rep = Server(hbm_budget=0, epoch_steps=8, backend=be, clock=clock,
                 keep_populations=True).run(jobs)
    assert len(rep.results) == len(jobs) and rep.refused == 0
    for r, job in zip(rep.results, sorted(jobs, key=lambda j: j.job_id)):
        assert r.job_id == job.job_id and r.status == "ok"
        fl = job.fields()
        solo = oracle.run(oracle.init(job.lattice, fl.rho_A, fl.rho_B), job.tau, job.tau, job.G,
                          job.steps)
        assert np.array_equal(r.populations, solo)
        assert r.arrival <= r.admitted <= r.completed
    s = rep.summary()
    assert s["jobs"] == len(jobs) and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_budget_is_never_exceeded_and_forces_queueing():
    clock = SimClock()
    be = FakeBackend(clock)
    jobs = _jobs(14, seed=5, rate=1000.0)      # near-simultaneous arrivals
    budget = max(be.bytes_needed(j) for j in jobs) * 2
    rep = Server(hbm_budget=budget, epoch_steps=8, backend=be, clock=clock).run(jobs)
    used = [u for tag, u in ((e[0], e[1]) for e in be.log) if tag == "used"]
    assert max(used) <= budget
    assert len(rep.results) == len(jobs)
    assert rep.summary()["max_queue"] > 0       # someone had to wait for memory


def test_jobs_that_can_never_fit_are_refused_without_blocking():
    clock = SimClock()
    be = FakeBackend(clock)
    jobs = _jobs(8, seed=9)
    big = max(jobs, key=lambda j: j.sites)
    budget = be.bytes_needed(big) - 1
    rep = Server(hbm_budget=budget, epoch_steps=8, backend=be, clock=clock).run(jobs)
    too_big = [j for j in jobs if be.bytes_needed(j) > budget]
    assert rep.refused == len(too_big) >= 1
    assert len(rep.results) == len(jobs) - len(too_big)


def test_arrivals_during_an_epoch_join_at_the_next_boundary():
    clock = SimClock()
    be = FakeBackend(clock, capacity=1e4)       # slow device: long epochs
    jobs = _jobs(6, seed=3, rate=200.0)
    rep = Server(hbm_budget=0, epoch_steps=10, backend=be, clock=clock).run(jobs)
    bounds = sorted({0.0} | {e[1] for e in be.log if e[0] == "epoch"})
    for r in rep.results:
        # admitted at the first epoch boundary at or after its arrival
        nxt = min(b for b in bounds if b >= r.arrival - 1e-12) if r.arrival > 0 else 0.0
        assert r.admitted >= r.arrival
        assert r.admitted <= max(nxt, r.arrival) + 1e-9
    resident = [e[2] for e in be.log if e[0] == "epoch"]
    assert max(resident) >= 2                    # jobs overlapped on the device


def test_a_diverging_job_is_reported_and_the_others_finish():
    clock = SimClock()
    be = FakeBackend(clock)
    jobs = _jobs(5, seed=11)
    bad = jobs[2]
    bad.G, bad.tau, bad.steps = 40.0, 0.51, 40   # far past any stable coupling
    rep = Server(hbm_budget=0, epoch_steps=8, backend=be, clock=clock).run(jobs)
    by_id = {r.job_id: r for r in rep.results}
    assert by_id[bad.job_id].status == "nonfinite"
    assert all(r.status == "ok" for r in rep.results if r.job_id != bad.job_id)


def test_offered_rate_scales_with_capacity():
    jobs = _jobs(20)
    r1 = offered_rate(jobs, capacity_mlups=1000.0, load=0.7)
    r2 = offered_rate(jobs, capacity_mlups=2000.0, load=0.7)
    assert abs(r2 / r1 - 2.0) < 1e-12


def _job(jid, L, steps, arrival, q=9):
    nz = L if q == 19 else 1
    return sc_inputs.JobSpec(jid, q, L, L, nz, 1.0, 1.3, steps, "drop", L / 5.0, seed=jid,
                             arrival=arrival)


def test_srpt_lets_a_short_job_overtake_a_long_one():
    """A long job is running when a short one arrives: shortest remaining work
    first finishes the short one first; advancing every resident job each
    epoch makes it wait for the long job's step time, and it completes later."""
    done_at = {}
    for policy in ("srpt", "all"):
        clock = SimClock()
        be = FakeBackend(clock, capacity=2e4)
        jobs = [_job(0, 24, 200, 0.0), _job(1, 8, 20, 0.05)]
        rep = Server(hbm_budget=0, epoch_steps=10, backend=be, clock=clock, policy=policy,
                     sat_sites=64).run(jobs)
        by_id = {r.job_id: r for r in rep.results}
        done_at[policy] = (by_id[0].completed, by_id[1].completed)
    assert done_at["srpt"][1] < done_at["srpt"][0]
    assert done_at["srpt"][1] < done_at["all"][1]


def test_srpt_epochs_hold_at_most_the_saturating_prefix():
    """Every epoch's members are a shortest-remaining-work prefix that stops
    once sat_sites is reached: dropping its largest lattice leaves fewer
    sites than sat_sites."""
    clock = SimClock()
    be = FakeBackend(clock)
    jobs = _jobs(12, seed=7, rate=1000.0)
    sat = 600
    Server(hbm_budget=0, epoch_steps=6, backend=be, clock=clock, sat_sites=sat).run(jobs)
    sites = {j.job_id: j.sites for j in jobs}
    epochs = [e[1] for e in be.log if e[0] == "members"]
    assert epochs and max(len(m) for m in epochs) >= 2
    for members in epochs:
        tot = sum(sites[j] for j in members)
        assert len(members) == 1 or tot - max(sites[j] for j in members) < sat


def test_both_policies_give_each_job_its_solo_result():
    res = {}
    for policy in ("srpt", "all"):
        clock = SimClock()
        be = FakeBackend(clock)
        jobs = _jobs(8, seed=13, rate=300.0)
        rep = Server(hbm_budget=0, epoch_steps=7, backend=be, clock=clock, policy=policy,
                     sat_sites=300, keep_populations=True).run(jobs)
        res[policy] = {r.job_id: r.populations for r in rep.results}
    assert res["srpt"].keys() == res["all"].keys()
    for k in res["srpt"]:
        assert np.array_equal(res["srpt"][k], res["all"][k])


def test_unknown_policy_is_rejected():
    with pytest.raises(ValueError):
        Server(policy="fifo")


def test_solo_capacity_is_work_over_summed_service_time():
    from paper_1112_5547_amd.serve import solo_capacity
    jobs = [_job(0, 10, 100, 0.0), _job(1, 20, 50, 0.0), _job(2, 10, 300, 0.0)]
    step_s = {(9, 10, 10, 1): 1e-5, (9, 20, 20, 1): 4e-5}
    work = 100 * 100 + 400 * 50 + 100 * 300
    busy = 100 * 1e-5 + 50 * 4e-5 + 300 * 1e-5
    assert abs(solo_capacity(jobs, step_s) - work / busy / 1e6) < 1e-12


def test_srpt_steps_a_saturating_lone_job_by_itself():
    """A job whose lattice alone reaches sat_sites never joins a batch: the
    two small jobs run first (their remaining work is smaller), then the big
    job's 30 steps all run as solo launches; every result is its solo result."""
    clock = SimClock()
    be = FakeBackend(clock)
    jobs = [_job(0, 20, 30, 0.0), _job(1, 6, 12, 0.0), _job(2, 7, 9, 0.0)]
    rep = Server(hbm_budget=0, epoch_steps=8, backend=be, clock=clock, sat_sites=400,
                 keep_populations=True).run(jobs)
    solo = [e for e in be.log if e[0] == "solo"]
    assert solo and all(e[1] == 0 for e in solo)
    assert sum(e[2] for e in solo) == 30
    members = [e[1] for e in be.log if e[0] == "members"]
    assert all(0 not in m for m in members)
    by_id = {r.job_id: r for r in rep.results}
    assert by_id[1].completed < by_id[0].completed and by_id[2].completed < by_id[0].completed
    for job in jobs:
        fl = job.fields()
        ref = oracle.run(oracle.init(job.lattice, fl.rho_A, fl.rho_B), job.tau, job.tau, job.G,
                         job.steps)
        assert np.array_equal(by_id[job.job_id].populations, ref)


def test_aging_lets_a_waiting_large_job_ahead_of_new_small_ones():
    """A large job keeps losing to a stream of small ones under pure SRPT; with
    aging its key drops with its waiting time and it completes earlier."""
    done = {}
    for aging in (0.0, 4.0):
        clock = SimClock()
        be = FakeBackend(clock, capacity=1e4)
        # one 5.4 s job at t = 0, then 0.11 s jobs every 0.15 s
        jobs = [_job(0, 30, 60, 0.0)] + [_job(k, 6, 30, 0.15 * k) for k in range(1, 40)]
        rep = Server(hbm_budget=0, epoch_steps=10, backend=be, clock=clock, sat_sites=30,
                     aging=aging, nominal_rate=1e4).run(jobs)
        done[aging] = {r.job_id: r.completed for r in rep.results}
    assert done[4.0][0] < done[0.0][0] - 1.0


def test_deadline_guard_keeps_each_job_near_its_arrival_order_completion():
    """Pure SRPT lets a stream of small jobs pass a large one indefinitely; with
    the deadline guard every job completes by about the time it would under
    one-job-at-a-time service in arrival order at the nominal rate (within an
    epoch for a guard >= 0, within an epoch plus |guard| for a negative one),
    while small jobs still overtake the large one as long as the deadlines
    leave slack (here the nominal rate is half the device's)."""
    nominal = 0.5e4
    res = {}
    for guard in (None, 0.5, -1.0):
        clock = SimClock()
        be = FakeBackend(clock, capacity=1e4)
        # ten small jobs, then a large one, then a small one every 0.15 s
        jobs = ([_job(k, 6, 30, 0.0) for k in range(1, 11)] + [_job(0, 30, 60, 0.001)]
                + [_job(k, 6, 30, 0.15 * (k - 10)) for k in range(11, 160)])
        rep = Server(hbm_budget=0, epoch_steps=10, backend=be, clock=clock, sat_sites=30,
                     guard=guard, nominal_rate=nominal).run(jobs)
        res[guard] = {r.job_id: r for r in rep.results}
    v, deadline = 0.0, {}
    for j in sorted(jobs, key=lambda j: j.arrival):
        v = max(v, j.arrival) + j.sites * j.steps / nominal
        deadline[j.job_id] = v
    epoch_s = 10 * 30 * 30 / 1e4          # the longest epoch (the large job alone)
    late_srpt = max(r.completed - deadline[k] for k, r in res[None].items())
    late_guard = max(r.completed - deadline[k] for k, r in res[0.5].items())
    late_neg = max(r.completed - deadline[k] for k, r in res[-1.0].items())
    assert late_srpt > 2.0                              # SRPT alone starves the large job
    assert late_guard <= epoch_s + 0.1
    assert late_neg <= epoch_s + 1.0 + 0.1
    assert late_neg > late_guard                        # the allowance is used
    # small jobs that arrive after the large one still overtake it while it has slack
    for g in (0.5, -1.0):
        later = [r for r in res[g].values() if r.arrival > 0.001]
        assert sum(r.completed < res[g][0].completed for r in later) >= 5


def test_deadline_guard_backlog_of_due_jobs():
    """Several large jobs that are due on arrival (the device is behind their
    arrival-order completion times) are served in deadline order ahead of a
    stream of small jobs: the guard looks at the cumulative work of the jobs
    due first, not at each job alone."""
    nominal = 1e4
    clock = SimClock()
    be = FakeBackend(clock, capacity=1e4)
    jobs = ([_job(k, 30, 40, 0.001 * k) for k in range(3)]
            + [_job(k, 6, 20, 0.05 * (k - 2)) for k in range(3, 80)])
    rep = Server(hbm_budget=0, epoch_steps=10, backend=be, clock=clock, sat_sites=30,
                 guard=0.0, nominal_rate=nominal).run(jobs)
    v, deadline = 0.0, {}
    for j in sorted(jobs, key=lambda j: j.arrival):
        v = max(v, j.arrival) + j.sites * j.steps / nominal
        deadline[j.job_id] = v
    epoch_s = 10 * 30 * 30 / 1e4
    assert max(r.completed - deadline[r.job_id] for r in rep.results) <= epoch_s + 0.1
    assert rep.summary()["deadline_epochs"] > 0


def test_service_prices_from_solo_step_times():
    """With measured solo step times the server prices a job by its shape's
    step time, else by its site updates at the nominal rate."""
    clock = SimClock()
    be = FakeBackend(clock, capacity=1e4)
    a, b = _job(0, 30, 40, 0.0), _job(1, 6, 20, 0.0)
    srv = Server(backend=be, clock=clock, nominal_rate=1e4,
                 step_seconds={(a.lattice, a.nx, a.ny, a.nz): 2e-3})
    assert srv.service_s(a, 40) == pytest.approx(40 * 2e-3)
    assert srv.service_s(b, 20) == pytest.approx(20 * b.sites / 1e4)


def test_batched_capacity_is_the_servers_rate_on_the_whole_mix():
    """All jobs present from the start with a tenth of their steps (at least
    an epoch): work over the time from the last admission to the last
    completion, which the fake device runs at its capacity plus a small cost
    per launch."""
    clock = SimClock()
    be = FakeBackend(clock, capacity=1e4)
    jobs = _jobs(12, seed=7, rate=5.0)
    cap = batched_capacity(jobs, backend=be, clock=clock, epoch_steps=8, sat_sites=10_000)
    assert 0.9e-2 < cap <= 1e-2          # MLUPS: 1e4 site updates per second
